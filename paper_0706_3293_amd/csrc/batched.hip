// Batched Lanczos: many independent problems (basis, couplings) with up to 16
// start vectors each, all steps in one persistent cooperative launch.
//
// Vectors are stored in FP32 as [dim][NV] rows (NV = 1, 2, 4, 8 or 16), so the
// multi-vector product H X decodes each basis state and encodes each target
// once (Sec. 3.1, 3.2) and gathers the NV entries of a target row with
// contiguous 16-byte loads; with 8 or 16 vectors a row is spread over 2 or 4
// lanes, which share its decoding and bond work.  Dots and norms are FP64.  Each (instance,
// vector) pair runs its own recurrence (Paige's ordering, as hm_lanczos):
//
//   init  norms of the start vectors, r_0 = v0 / |v0|            (2 barriers)
//   step  A:  w = sigma H r - cprev r_prev, alpha partials per item and vector
//         A': alpha per pair, one wave per pair summing the instance's item
//             partials in a fixed order
//         B:  w -= alpha sigma r, |w|^2 partials
//         B': beta, breakdown test, sigma and cprev of the next step
// Work items are 256-row tiles of one instance; persistent workgroups take
// chunks of consecutive items in a fixed order and reduce once per run of
// items of one instance, so every sum has a fixed order for a given grid.  The grid
// barrier is a counter and a generation word with a bounded spin: a wave that
// waits too long raises an abort flag and every wave leaves the kernel.
#include <algorithm>
#include <cmath>
#include <vector>

#include "device_common.h"
#include "hm_internal.h"

namespace hm {

constexpr int kBatchBlock = 256;
constexpr int kBatchMaxVec = 16;
constexpr size_t kBatchPrefixLds = 24 * 1024;
constexpr long long kSpinLimit = 1ll << 22;

struct InstDesc {
    int N, A, two_s, nb;
    uint32_t dim;
    uint32_t vec_off;          // first row of this instance in the stacked vectors
    uint32_t item_first, item_count;
    const uint32_t *prefix;    // 32-bit prefix table of the basis
    const double *ladder;
    const BondDev *bonds;
    const double *v0;          // [dim][nvec] FP64 start vectors
};

struct Item {
    uint32_t inst, row0;
};

// A bond as the pass-A loop reads it from LDS: sites packed u | v << 16.
struct LdsBond {
    int32_t uv;
    float mJ4;
    double mJ2;
};
constexpr int kStageWaves = 16;   // per-wave partial slots (workgroup <= 1024 threads)
constexpr int kChunkDefault = 4;  // items a workgroup takes at a time (default)
constexpr int kWgPerCuDefault = 4; // resident workgroups per compute unit (default)

// Arrival counter, generation word and abort flag on separate 128-byte lines,
// so the polling of gen does not contend with the arrivals on count.
struct GridBar {
    unsigned count;
    unsigned pad0[31];
    unsigned gen;
    unsigned pad1[31];
    int abort;
    int pad2[31];
};

struct BatchArgs {
    const InstDesc *inst;
    const Item *items;
    int ninst, n_items, nvec, steps;
    double tol;
    GridBar *bar;
    float *r[3];
    double *partial;           // [n_items][NV]
    double *alpha, *beta;      // [npairs][steps]
    double *sigma, *cprev;     // [npairs][steps + 1]
    double *scale, *norm0;     // [npairs]
    int *stopped;              // [npairs]: steps done at breakdown, 0 while running
    int max_prefix;            // entries of the largest prefix table
    int max_bonds;             // bonds of the largest coupling list
    int chunk;                 // items a workgroup takes at a time
};

// Grid-wide barrier; returns false if the run was aborted (timeout).  One
// agent-scope release on arrival (the workgroup barrier before it orders the
// other waves' writes), relaxed polling of the generation word, and one
// agent-scope acquire fence after the wait.  Acquire loads in the polling loop
// would invalidate the caches on every iteration; measured alone, this form
// takes 8, 15 and 28 us per barrier on 256, 512 and 1024 workgroups against
// 44, 41 and 81 us with acquire polling.
__device__ bool grid_barrier(GridBar *bar, unsigned nblocks, int *lds_ok) {
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = __hip_atomic_load(&bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
        const unsigned g = __hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived = __hip_atomic_fetch_add(&bar->count, 1u, __ATOMIC_RELEASE,
                                                        __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblocks - 1) {
            __hip_atomic_store(&bar->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&bar->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long long spins = 0;
            while (ok && __hip_atomic_load(&bar->gen, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > kSpinLimit) {
                    __hip_atomic_store(&bar->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                }
                if ((spins & 1023) == 0 &&
                    __hip_atomic_load(&bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    ok = 0;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *lds_ok = ok;
    }
    __syncthreads();
    return *lds_ok != 0;
}

template <int NV>
__device__ __forceinline__ void load_row(const float *__restrict__ p, float (&v)[NV]) {
    if constexpr (NV % 4 == 0) {
#pragma unroll
        for (int q = 0; q < NV / 4; ++q) {
            const float4 t = reinterpret_cast<const float4 *>(p)[q];
            v[4 * q] = t.x;
            v[4 * q + 1] = t.y;
            v[4 * q + 2] = t.z;
            v[4 * q + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] = p[q];
    }
}

template <int NV>
__device__ __forceinline__ void store_row(float *__restrict__ p, const float (&v)[NV]) {
    if constexpr (NV % 4 == 0) {
#pragma unroll
        for (int q = 0; q < NV / 4; ++q)
            reinterpret_cast<float4 *>(p)[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2],
                                                           v[4 * q + 3]);
    } else {
#pragma unroll
        for (int q = 0; q < NV; ++q) p[q] = v[q];
    }
}

// Per-item FP64 partials of NV columns: a fixed butterfly per column inside
// each wave, then thread q < NV adds the wave sums of column q in wave order.
template <int NV>
__device__ __forceinline__ void item_partials(double (&v)[NV], double *stage, double *out) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] += __shfl_xor(v[q], off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) stage[wid * NV + q] = v[q];
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += stage[w * NV + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// Lanes per row in the two row passes: with 8 or 16 vectors a row is split
// over NV/4 lanes of 4 vectors (16 bytes) each, so the lanes of a wave read
// whole 64-byte rows together (a 64-lane load touches 16 lines, not 64).  The
// lanes of a row share its bond work (each takes every G-th bond of a batch)
// and pass the targets and coefficients around with quad permutes.
template <int NV>
constexpr int lanes_per_row() { return NV >= 8 ? NV / 4 : 1; }

// Value of lane t of this lane's group of G consecutive lanes (G = 2 or 4;
// groups never straddle a quad), by a DPP quad permute.
template <int G>
__device__ __forceinline__ uint32_t group_lane(uint32_t v, int t) {
    if constexpr (G == 4) {
        switch (t) {   // quad_perm [t, t, t, t]
            case 0: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x00, 0xf, 0xf, false);
            case 1: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x55, 0xf, 0xf, false);
            case 2: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xaa, 0xf, 0xf, false);
            default: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xff, 0xf, 0xf, false);
        }
    } else {
        switch (t) {   // quad_perm [t, t, 2 + t, 2 + t]
            case 0: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xa0, 0xf, 0xf, false);
            default: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xf5, 0xf, 0xf, false);
        }
    }
}

// item_partials when G lanes share a row: lane l holds the V = NV / G columns
// starting at (l % G) V.  A fixed butterfly over the lanes of one column group
// (offsets 32 down to G), then thread q < NV adds the wave sums of column q in
// wave order.  G = 1 is item_partials.
template <int NV, int G>
__device__ __forceinline__ void item_partials_g(double (&v)[NV / G], double *stage,
                                                double *out) {
    constexpr int V = NV / G;
#pragma unroll
    for (int off = 32; off >= G; off >>= 1) {
#pragma unroll
        for (int q = 0; q < V; ++q) v[q] += __shfl_xor(v[q], off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane < G) {
#pragma unroll
        for (int q = 0; q < V; ++q) stage[wid * NV + lane * V + q] = v[q];
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += stage[w * NV + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// Sum of column q of the item partials [first, first + count): lane l adds
// items l, l + 64, ... in order, then a fixed butterfly over the lanes.  Every
// lane of the wave returns the same value.
template <int NV>
__device__ __forceinline__ double pair_sum(const double *__restrict__ partial, uint32_t first,
                                           uint32_t count, int q) {
    const uint32_t lane = threadIdx.x & 63;
    double s = 0.0;
    for (uint32_t t = lane; t < count; t += 64) s += partial[(size_t)(first + t) * NV + q];
    return wave_sum(s);
}

template <int NV, int B>
__global__ __launch_bounds__(kBatchBlock) void batched_lanczos_kernel(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int ok_flag;
    __shared__ double sc_sigma[NV], sc_c[NV], sc_a[NV];
    // instance in LDS (pass A): the kernel writes through pointers that may
    // alias the descriptors, so uniform reads of them from global memory
    // would be vector loads per lane; LDS broadcasts are cheap
    __shared__ int s_N, s_A, s_two_s, s_nb;
    __shared__ uint32_t s_dim, s_vec_off, s_item_end;
    __shared__ uint32_t sb_dim, sb_vec_off, sb_item_end;   // pass B's instance
    uint32_t *P = reinterpret_cast<uint32_t *>(smem);
    double *F = reinterpret_cast<double *>(smem + ((a.max_prefix * 4 + 15) / 16) * 16);
    double *stage = F + 32;
    LdsBond *Bd = reinterpret_cast<LdsBond *>(stage + kStageWaves * NV);
    const unsigned nblocks = gridDim.x;
    const int npairs = a.ninst * NV;
    // per-pair reductions: one wave per (instance, vector) pair
    const int gwave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int nwaves = (int)((gridDim.x * blockDim.x) >> 6);
    const bool lane0 = (threadIdx.x & 63) == 0;
    // Workgroups take chunks of a.chunk consecutive items, chunk c going to
    // workgroup c % grid, so the grid sweeps the items roughly in order (a
    // narrow working set for the gathers).  Within a chunk, consecutive items
    // of one instance form a segment: threads add their rows' FP64
    // contributions over the segment and the workgroup reduces once per
    // segment, into the slot of the segment's first item.  All other slots
    // stay zero, so the per-pair sums over an instance's slots keep a fixed
    // order for a given grid.
    const int kChunk = a.chunk;
    const int n_chunks = (a.n_items + kChunk - 1) / kChunk;
    for (int c = blockIdx.x; c < n_chunks; c += gridDim.x) {
        const int i0 = c * kChunk, i1 = min(i0 + kChunk, a.n_items);
        for (int t = threadIdx.x; t < (i1 - i0) * NV; t += blockDim.x)
            a.partial[(size_t)i0 * NV + t] = 0.0;
    }

    // ---- init: |v0| partials per segment --------------------------------
    {
        double s[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) s[q] = 0.0;
        for (int c = blockIdx.x; c < n_chunks; c += gridDim.x) {
            const int i0 = c * kChunk, i1 = min(i0 + kChunk, a.n_items);
            int seg = i0;
            for (int it = i0; it < i1; ++it) {
                const Item itm = a.items[it];
                const InstDesc &d = a.inst[itm.inst];
                const uint32_t i = itm.row0 + threadIdx.x;
                if (i < d.dim) {
    #pragma unroll
                    for (int q = 0; q < NV; ++q) {
                        const double v = q < a.nvec ? d.v0[(size_t)i * a.nvec + q] : 0.0;
                        s[q] += v * v;
                    }
                }
                if (it + 1 == i1 || (uint32_t)(it + 1) == d.item_first + d.item_count) {
                    item_partials<NV>(s, stage, a.partial + (size_t)seg * NV);
    #pragma unroll
                    for (int q = 0; q < NV; ++q) s[q] = 0.0;
                    seg = it + 1;
                }
            }
        }
    }
    if (!grid_barrier(a.bar, nblocks, &ok_flag)) return;
    for (int p = gwave; p < npairs; p += nwaves) {
        const InstDesc &d = a.inst[p / NV];
        const int q = p % NV;
        const double s = pair_sum<NV>(a.partial, d.item_first, d.item_count, q);
        if (!lane0) continue;
        const bool live = q < a.nvec && s > 0.0;
        a.norm0[p] = sqrt(s);
        a.scale[p] = 0.0;
        a.stopped[p] = live ? 0 : -1;
        a.sigma[(size_t)p * (a.steps + 1)] = live ? 1.0 : 0.0;
        a.cprev[(size_t)p * (a.steps + 1)] = 0.0;
    }
    if (!grid_barrier(a.bar, nblocks, &ok_flag)) return;
    for (int it = blockIdx.x; it < a.n_items; it += gridDim.x) {
        const Item itm = a.items[it];
        const InstDesc &d = a.inst[itm.inst];
        const uint32_t i = itm.row0 + threadIdx.x;
        if (i < d.dim) {
            float v[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                const int p = itm.inst * NV + q;
                v[q] = (q < a.nvec && a.stopped[p] == 0)
                           ? (float)(d.v0[(size_t)i * a.nvec + q] / a.norm0[p]) : 0.0f;
            }
            store_row<NV>(a.r[0] + ((size_t)d.vec_off + i) * NV, v);
        }
    }
    if (!grid_barrier(a.bar, nblocks, &ok_flag)) return;

    // row passes: G lanes per row, this lane's V columns start at gq
    constexpr int G = lanes_per_row<NV>(), V = NV / G;
    const int gl = (int)(threadIdx.x % G), gq = gl * V;
    int loaded = -1;   // instance whose tables are in LDS
    for (int k = 0; k < a.steps; ++k) {
        const float *__restrict__ rk = a.r[k % 3];
        const float *__restrict__ rp = a.r[(k + 2) % 3];
        float *__restrict__ w = a.r[(k + 1) % 3];
        // ---- A: w = sigma H r_k - cprev r_{k-1}; alpha partials ----------
        double dacc[V];
#pragma unroll
        for (int q = 0; q < V; ++q) dacc[q] = 0.0;
        int sc_loaded = -1;
        for (int c = blockIdx.x; c < n_chunks; c += gridDim.x) {
            const int i0 = c * kChunk, i1 = min(i0 + kChunk, a.n_items);
            int seg = i0;
            for (int it = i0; it < i1; ++it) {
                const Item itm = a.items[it];
                // a new instance starts a segment; the previous segment ended with
                // a workgroup barrier, so nobody still reads what is replaced here
                if ((int)itm.inst != sc_loaded) {
                    if ((int)itm.inst != loaded) {
                        const InstDesc &d = a.inst[itm.inst];
                        const int plen = d.N * (d.A + 1) * (d.two_s + 1);
                        for (int t = threadIdx.x; t < plen; t += blockDim.x) P[t] = d.prefix[t];
                        for (int t = threadIdx.x; t < d.two_s + 2; t += blockDim.x) F[t] = d.ladder[t];
                        for (int t = threadIdx.x; t < d.nb; t += blockDim.x) {
                            const BondDev bd = d.bonds[t];
                            Bd[t] = LdsBond{bd.u | (bd.v << 16), (float)bd.mJ4, bd.mJ2};
                        }
                        if (threadIdx.x == 0) {
                            s_N = d.N;
                            s_A = d.A;
                            s_two_s = d.two_s;
                            s_nb = d.nb;
                            s_dim = d.dim;
                            s_vec_off = d.vec_off;
                            s_item_end = d.item_first + d.item_count;
                        }
                        loaded = itm.inst;
                    }
                    if (threadIdx.x < NV) {
                        const int p = itm.inst * NV + threadIdx.x;
                        sc_sigma[threadIdx.x] = a.sigma[(size_t)p * (a.steps + 1) + k];
                        sc_c[threadIdx.x] = a.cprev[(size_t)p * (a.steps + 1) + k];
                    }
                    sc_loaded = itm.inst;
                    __syncthreads();
                }
                const int iN = __builtin_amdgcn_readfirstlane(s_N);
                const int iA = __builtin_amdgcn_readfirstlane(s_A);
                const int two_s = __builtin_amdgcn_readfirstlane(s_two_s);
                const int nb = __builtin_amdgcn_readfirstlane(s_nb);
                const uint32_t dim = __builtin_amdgcn_readfirstlane(s_dim);
                const uint32_t vec_off = __builtin_amdgcn_readfirstlane(s_vec_off);
                const uint32_t item_end = __builtin_amdgcn_readfirstlane(s_item_end);
                const Prefix<uint32_t> pv{P, iA + 1, two_s + 1};
                const float *__restrict__ xr = rk + (size_t)vec_off * NV;
                // lane gl of a group decodes the group's row of sub-iteration gl,
                // so each row is decoded once; the state is passed around below
                const uint32_t i_mine = itm.row0 + gl * (kBatchBlock / G) + threadIdx.x / G;
                const uint64_t st_mine =
                    i_mine < dim ? unrank_state<uint32_t, B>(i_mine, pv, iN, iA, two_s) : 0;
                for (int sub = 0; sub < G; ++sub) {
                    const uint32_t i = itm.row0 + sub * (kBatchBlock / G) + threadIdx.x / G;
                    if (i >= dim) continue;   // the G lanes of a row leave together
                    uint64_t st = st_mine;
                    if constexpr (G > 1)
                        st = (uint64_t)group_lane<G>((uint32_t)st_mine, sub) |
                             ((uint64_t)group_lane<G>((uint32_t)(st_mine >> 32), sub) << 32);
                    float xi[V], acc[V];
                    load_row<V>(xr + (size_t)i * NV + gq, xi);
    #pragma unroll
                    for (int q = 0; q < V; ++q) acc[q] = 0.0f;
                    float diag = 0.0f;
                    // moves in batches: targets and coefficients first (a move that
                    // is not allowed reads the own row with coefficient 0), then all
                    // row loads of the batch, then the products in bond order, so
                    // kMoves row gathers are in flight together.  With G > 1 lane
                    // gl of a row finds the moves of bonds gl*BPL .. gl*BPL+BPL-1
                    // of the batch and the group shares them.
                    constexpr int kMoves = G > 1 ? 8 : 16;
                    constexpr int BPL = kMoves / 2 / G;      // bonds per lane and batch
                    for (int b0 = 0; b0 < nb; b0 += kMoves / 2) {
                        uint32_t jo[2 * BPL];
                        float co[2 * BPL];
    #pragma unroll
                        for (int t = 0; t < BPL; ++t) {
                            jo[2 * t] = jo[2 * t + 1] = i;
                            co[2 * t] = co[2 * t + 1] = 0.0f;
                            const int b = b0 + gl * BPL + t;
                            if (b < nb) {
                                const LdsBond bd = Bd[b];
                                const int u = bd.uv & 0xffff, v = bd.uv >> 16;
                                const double mJ2 = bd.mJ2;
                                const int au = digit_at<B>(st, u), av = digit_at<B>(st, v);
                                diag += bd.mJ4 * (float)((two_s - 2 * au) * (two_s - 2 * av));
                                if (au >= 1 && av < two_s) {
                                    jo[2 * t] = i + move_delta<uint32_t, B>(st, u, v, -1, pv);
                                    co[2 * t] = (float)(mJ2 * F[au] * F[av + 1]);
                                }
                                if (av >= 1 && au < two_s) {
                                    jo[2 * t + 1] = i + move_delta<uint32_t, B>(st, u, v, +1, pv);
                                    co[2 * t + 1] = (float)(mJ2 * F[av] * F[au + 1]);
                                }
                            }
                        }
                        uint32_t jm[kMoves];
                        float cm[kMoves];
                        if constexpr (G == 1) {
    #pragma unroll
                            for (int m = 0; m < kMoves; ++m) {
                                jm[m] = jo[m];
                                cm[m] = co[m];
                            }
                        } else {
    #pragma unroll
                            for (int src = 0; src < G; ++src)
    #pragma unroll
                                for (int m = 0; m < 2 * BPL; ++m) {
                                    jm[src * 2 * BPL + m] = group_lane<G>(jo[m], src);
                                    cm[src * 2 * BPL + m] = __uint_as_float(
                                        group_lane<G>(__float_as_uint(co[m]), src));
                                }
                        }
                        float xj[kMoves][V];
    #pragma unroll
                        for (int m = 0; m < kMoves; ++m)
                            load_row<V>(xr + (size_t)jm[m] * NV + gq, xj[m]);
    #pragma unroll
                        for (int m = 0; m < kMoves; ++m)
    #pragma unroll
                            for (int q = 0; q < V; ++q) acc[q] += cm[m] * xj[m][q];
                    }
                    if constexpr (G > 1) {
                        // the diagonal: each lane summed its own bonds; add the
                        // group's parts in lane order (same value in every lane)
                        const uint32_t db = __float_as_uint(diag);
                        float dsum = 0.0f;
    #pragma unroll
                        for (int src = 0; src < G; ++src)
                            dsum += __uint_as_float(group_lane<G>(db, src));
                        diag = dsum;
                    }
                    float prv[V];
                    if (k > 0) load_row<V>(rp + ((size_t)vec_off + i) * NV + gq, prv);
                    float out[V];
    #pragma unroll
                    for (int q = 0; q < V; ++q) {
                        const double hv = (double)(diag * xi[q] + acc[q]);
                        double wq = sc_sigma[gq + q] * hv;
                        if (k > 0) wq -= sc_c[gq + q] * (double)prv[q];
                        out[q] = (float)wq;
                        dacc[q] += (double)out[q] * (sc_sigma[gq + q] * (double)xi[q]);
                    }
                    store_row<V>(w + ((size_t)vec_off + i) * NV + gq, out);
                }
                if (it + 1 == i1 || (uint32_t)(it + 1) == item_end) {
                    item_partials_g<NV, G>(dacc, stage, a.partial + (size_t)seg * NV);
    #pragma unroll
                    for (int q = 0; q < V; ++q) dacc[q] = 0.0;
                    seg = it + 1;
                }
            }
        }
        if (!grid_barrier(a.bar, nblocks, &ok_flag)) return;
        // ---- A': alpha per pair --------------------------------------------
        for (int p = gwave; p < npairs; p += nwaves) {
            const InstDesc &d = a.inst[p / NV];
            const double s = pair_sum<NV>(a.partial, d.item_first, d.item_count, p % NV);
            if (lane0) a.alpha[(size_t)p * a.steps + k] = s;
        }
        if (!grid_barrier(a.bar, nblocks, &ok_flag)) return;
        // ---- B: w -= alpha sigma r_k; |w|^2 partials -----------------------
        double ss[V];
#pragma unroll
        for (int q = 0; q < V; ++q) ss[q] = 0.0;
        sc_loaded = -1;
        for (int c = blockIdx.x; c < n_chunks; c += gridDim.x) {
            const int i0 = c * kChunk, i1 = min(i0 + kChunk, a.n_items);
            int seg = i0;
            for (int it = i0; it < i1; ++it) {
                const Item itm = a.items[it];
                if ((int)itm.inst != sc_loaded) {
                    if (threadIdx.x < NV) {
                        const int p = itm.inst * NV + threadIdx.x;
                        sc_a[threadIdx.x] = a.alpha[(size_t)p * a.steps + k] *
                                            a.sigma[(size_t)p * (a.steps + 1) + k];
                    }
                    if (threadIdx.x == 0) {
                        const InstDesc &d = a.inst[itm.inst];
                        sb_dim = d.dim;
                        sb_vec_off = d.vec_off;
                        sb_item_end = d.item_first + d.item_count;
                    }
                    sc_loaded = itm.inst;
                    __syncthreads();
                }
                const uint32_t dim = __builtin_amdgcn_readfirstlane(sb_dim);
                const uint32_t vec_off = __builtin_amdgcn_readfirstlane(sb_vec_off);
                const uint32_t item_end = __builtin_amdgcn_readfirstlane(sb_item_end);
                for (int sub = 0; sub < G; ++sub) {
                    const uint32_t i = itm.row0 + sub * (kBatchBlock / G) + threadIdx.x / G;
                    if (i >= dim) continue;
                    const size_t row = ((size_t)vec_off + i) * NV + gq;
                    float wv[V], rv[V];
                    load_row<V>(w + row, wv);
                    load_row<V>(rk + row, rv);
    #pragma unroll
                    for (int q = 0; q < V; ++q) {
                        wv[q] = (float)((double)wv[q] - sc_a[gq + q] * (double)rv[q]);
                        ss[q] += (double)wv[q] * (double)wv[q];
                    }
                    store_row<V>(w + row, wv);
                }
                if (it + 1 == i1 || (uint32_t)(it + 1) == item_end) {
                    item_partials_g<NV, G>(ss, stage, a.partial + (size_t)seg * NV);
    #pragma unroll
                    for (int q = 0; q < V; ++q) ss[q] = 0.0;
                    seg = it + 1;
                }
            }
        }
        if (!grid_barrier(a.bar, nblocks, &ok_flag)) return;
        // ---- B': beta, breakdown, next sigma / cprev -----------------------
        for (int p = gwave; p < npairs; p += nwaves) {
            const InstDesc &d = a.inst[p / NV];
            const double s = pair_sum<NV>(a.partial, d.item_first, d.item_count, p % NV);
            if (!lane0) continue;
            const double b = sqrt(s);
            const size_t o = (size_t)p * (a.steps + 1);
            if (a.stopped[p] != 0) {
                a.beta[(size_t)p * a.steps + k] = 0.0;
                a.sigma[o + k + 1] = 0.0;
                a.cprev[o + k + 1] = 0.0;
                continue;
            }
            a.beta[(size_t)p * a.steps + k] = b;
            const double sc = fmax(a.scale[p], fmax(fabs(a.alpha[(size_t)p * a.steps + k]), b));
            a.scale[p] = sc;
            if (!(b > a.tol * sc)) {
                a.stopped[p] = k + 1;
                a.sigma[o + k + 1] = 0.0;
                a.cprev[o + k + 1] = 0.0;
            } else {
                a.sigma[o + k + 1] = 1.0 / b;
                a.cprev[o + k + 1] = b * a.sigma[o + k];
            }
        }
        if (!grid_barrier(a.bar, nblocks, &ok_flag)) return;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct BatchLayout {
    size_t desc, items, bar, alpha, beta, sigma, cprev, scale, norm0, stopped, partial, r0, r1,
        r2, total;
    int n_items, NV, bits;
    uint64_t rows;
};

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

static int vec_width(int nvec) {
    int NV = 1;
    while (NV < nvec) NV <<= 1;
    return NV;
}

static int batch_layout(int ninst, const hm_basis *bases, int nvec, int steps, BatchLayout *L) {
    if (ninst < 1) return fail(HM_EINVAL, "ninst must be >= 1");
    if (!bases) return fail(HM_EINVAL, "bases is null");
    if (nvec < 1 || nvec > kBatchMaxVec) return fail(HM_EINVAL, "nvec must be 1..16");
    if (steps < 1) return fail(HM_EINVAL, "steps must be >= 1");
    L->NV = vec_width(nvec);
    L->n_items = 0;
    L->rows = 0;
    // states of every instance are packed with the digit width of the
    // largest spin in the batch
    L->bits = 0;
    for (int k = 0; k < ninst; ++k) {
        if (!bases[k]) return fail(HM_EINVAL, "basis %d is null", k);
        L->bits = std::max(L->bits, bases[k]->impl.bits);
    }
    for (int k = 0; k < ninst; ++k) {
        const Basis &b = bases[k]->impl;
        if (b.N * L->bits > 64)
            return fail(HM_ERANGE,
                        "basis %d: %d sites at %d bits per digit (the batch's widest spin) "
                        "exceed 64 bits", k, b.N, L->bits);
        if (!b.idx32) return fail(HM_ERANGE, "basis %d: dimension too large for the batch", k);
        if (b.prefix_len() * 4 > kBatchPrefixLds)
            return fail(HM_ERANGE, "basis %d: prefix table exceeds the batch LDS budget", k);
        L->n_items += (int)((b.dim + kBatchBlock - 1) / kBatchBlock);
        L->rows += (uint64_t)b.dim;
    }
    if (L->rows >= ((uint64_t)1 << 32)) return fail(HM_ERANGE, "too many rows in the batch");
    const size_t npairs = (size_t)ninst * L->NV;
    size_t off = 0;
    L->desc = off; off = al256(off + sizeof(InstDesc) * ninst);
    L->items = off; off = al256(off + sizeof(Item) * L->n_items);
    L->bar = off; off = al256(off + sizeof(GridBar));
    L->alpha = off; off = al256(off + sizeof(double) * npairs * steps);
    L->beta = off; off = al256(off + sizeof(double) * npairs * steps);
    L->sigma = off; off = al256(off + sizeof(double) * npairs * (steps + 1));
    L->cprev = off; off = al256(off + sizeof(double) * npairs * (steps + 1));
    L->scale = off; off = al256(off + sizeof(double) * npairs);
    L->norm0 = off; off = al256(off + sizeof(double) * npairs);
    L->stopped = off; off = al256(off + sizeof(int) * npairs);
    L->partial = off; off = al256(off + sizeof(double) * (size_t)L->n_items * L->NV);
    const size_t vb = sizeof(float) * (size_t)L->rows * L->NV;
    L->r0 = off; off = al256(off + vb);
    L->r1 = off; off = al256(off + vb);
    L->r2 = off; off = al256(off + vb);
    L->total = off;
    return HM_OK;
}

template <int NV, int B>
static int launch_batched(BatchArgs &args, size_t lds, int wg_per_cu, hipStream_t st,
                          int *grid_out) {
    auto kern = batched_lanczos_kernel<NV, B>;
    int dev = 0, per_cu = 0;
    HM_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HM_HIP(hipGetDeviceProperties(&prop, dev));
    HM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBatchBlock, lds));
    if (per_cu < 1) return fail(HM_ERANGE, "batched kernel does not fit on a compute unit");
    // every workgroup of a cooperative launch must be resident at once
    int grid = std::min(per_cu, wg_per_cu) * prop.multiProcessorCount;
    grid = std::min(grid, std::max(args.n_items, 1));
    *grid_out = grid;
    void *params[] = {&args};
    HM_HIP(hipLaunchCooperativeKernel((const void *)kern, dim3(grid), dim3(kBatchBlock), params,
                                      (unsigned)lds, st));
    return HM_OK;
}

template <int NV>
static int dispatch_bits(int bits, BatchArgs &args, size_t lds, int wg, hipStream_t st, int *grid) {
    switch (bits) {
        case 1: return launch_batched<NV, 1>(args, lds, wg, st, grid);
        case 2: return launch_batched<NV, 2>(args, lds, wg, st, grid);
        case 3: return launch_batched<NV, 3>(args, lds, wg, st, grid);
        case 4: return launch_batched<NV, 4>(args, lds, wg, st, grid);
        default: return fail(HM_ERANGE, "batched kernel supports up to 4 bits per digit");
    }
}

__global__ void zero_bar(GridBar *bar) {
    bar->count = 0;
    bar->gen = 0;
    bar->abort = 0;
}

}  // namespace hm

using hm::fail;

extern "C" {

int hm_lanczos_batched_workspace(int32_t ninst, const hm_basis *bases, int32_t nvec,
                                 int32_t steps, size_t *bytes) {
    hm::clear_error();
    if (!bytes) return fail(HM_EINVAL, "bytes is null");
    hm::BatchLayout L;
    HM_TRY(hm::batch_layout(ninst, bases, nvec, steps, &L));
    *bytes = L.total;
    return HM_OK;
}

int hm_lanczos_batched(int32_t ninst, const hm_basis *bases, const double *const *J,
                       const double *const *d_v0, int32_t nvec, int32_t steps,
                       double breakdown_tol, int32_t chunk, int32_t wg_per_cu, void *d_work,
                       size_t work_bytes, double *alpha, double *beta, double *E0,
                       int32_t *steps_done, void *stream) {
    hm::clear_error();
    if (!J || !d_v0 || !d_work || !alpha || !beta || !E0 || !steps_done)
        return fail(HM_EINVAL, "null argument");
    if (chunk == 0) chunk = hm::kChunkDefault;
    if (wg_per_cu == 0) wg_per_cu = hm::kWgPerCuDefault;
    if (chunk < 1 || chunk > 64) return fail(HM_EINVAL, "chunk %d outside 1..64", chunk);
    if (wg_per_cu < 1 || wg_per_cu > 8)
        return fail(HM_EINVAL, "workgroups per compute unit %d outside 1..8", wg_per_cu);
    hm::BatchLayout L;
    HM_TRY(hm::batch_layout(ninst, bases, nvec, steps, &L));
    if (work_bytes < L.total)
        return fail(HM_EWORKSPACE, "workspace %zu bytes < required %zu", work_bytes, L.total);
    unsigned char *w = (unsigned char *)d_work;
    hipStream_t st = (hipStream_t)stream;
    std::vector<hm::InstDesc> desc(ninst);
    std::vector<hm::CouplingsRef> crefs(ninst);   // held until the run returns
    std::vector<hm::Item> items;
    uint32_t vec_off = 0;
    int max_prefix = 0, max_bonds = 0;
    for (int k = 0; k < ninst; ++k) {
        hm::Basis *b = &bases[k]->impl;
        if (!d_v0[k]) return fail(HM_EINVAL, "start vectors of instance %d are null", k);
        HM_TRY(hm::get_couplings(b, J[k], &crefs[k]));   // validates J, prepares the device
        const hm::Couplings *c = crefs[k].get();
        hm::InstDesc &d = desc[k];
        d.N = b->N;
        d.A = b->A;
        d.two_s = b->two_s;
        d.nb = c->nb;
        d.dim = (uint32_t)b->dim;
        d.vec_off = vec_off;
        d.item_first = (uint32_t)items.size();
        for (uint32_t r0 = 0; r0 < d.dim; r0 += hm::kBatchBlock) items.push_back({(uint32_t)k, r0});
        d.item_count = (uint32_t)items.size() - d.item_first;
        d.prefix = (const uint32_t *)b->d_prefix;
        d.ladder = b->d_ladder;
        d.bonds = c->dev;
        d.v0 = d_v0[k];
        vec_off += d.dim;
        max_prefix = std::max(max_prefix, (int)b->prefix_len());
        max_bonds = std::max(max_bonds, c->nb);
    }
    HM_HIP(hipMemcpyAsync(w + L.desc, desc.data(), sizeof(hm::InstDesc) * ninst,
                          hipMemcpyHostToDevice, st));
    HM_HIP(hipMemcpyAsync(w + L.items, items.data(), sizeof(hm::Item) * items.size(),
                          hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(hm::zero_bar, dim3(1), dim3(1), 0, st, (hm::GridBar *)(w + L.bar));
    HM_HIP(hipGetLastError());
    hm::BatchArgs a{};
    a.inst = (const hm::InstDesc *)(w + L.desc);
    a.items = (const hm::Item *)(w + L.items);
    a.ninst = ninst;
    a.n_items = L.n_items;
    a.nvec = nvec;
    a.steps = steps;
    a.tol = breakdown_tol > 0 ? breakdown_tol : 1e-6;   // FP32 vectors: FP32 noise floor
    a.bar = (hm::GridBar *)(w + L.bar);
    a.r[0] = (float *)(w + L.r0);
    a.r[1] = (float *)(w + L.r1);
    a.r[2] = (float *)(w + L.r2);
    a.partial = (double *)(w + L.partial);
    a.alpha = (double *)(w + L.alpha);
    a.beta = (double *)(w + L.beta);
    a.sigma = (double *)(w + L.sigma);
    a.cprev = (double *)(w + L.cprev);
    a.scale = (double *)(w + L.scale);
    a.norm0 = (double *)(w + L.norm0);
    a.stopped = (int *)(w + L.stopped);
    a.max_prefix = max_prefix;
    a.max_bonds = max_bonds;
    a.chunk = chunk;
    const size_t lds = ((size_t)(max_prefix * 4 + 15) / 16) * 16 + 32 * sizeof(double) +
                       (size_t)hm::kStageWaves * L.NV * sizeof(double) +
                       (size_t)max_bonds * sizeof(hm::LdsBond);
    const int bits = L.bits;
    int grid = 0, rc;
    switch (L.NV) {
        case 1: rc = hm::dispatch_bits<1>(bits, a, lds, wg_per_cu, st, &grid); break;
        case 2: rc = hm::dispatch_bits<2>(bits, a, lds, wg_per_cu, st, &grid); break;
        case 4: rc = hm::dispatch_bits<4>(bits, a, lds, wg_per_cu, st, &grid); break;
        case 8: rc = hm::dispatch_bits<8>(bits, a, lds, wg_per_cu, st, &grid); break;
        default: rc = hm::dispatch_bits<16>(bits, a, lds, wg_per_cu, st, &grid); break;
    }
    if (rc != HM_OK) return rc;
    HM_HIP(hipStreamSynchronize(st));
    hm::GridBar bar;
    HM_HIP(hipMemcpy(&bar, w + L.bar, sizeof bar, hipMemcpyDeviceToHost));
    if (bar.abort) return fail(HM_EDEVICE, "batched kernel: grid barrier timed out");
    const size_t npairs = (size_t)ninst * L.NV;
    std::vector<double> al(npairs * steps), be(npairs * steps);
    std::vector<int> stop(npairs);
    HM_HIP(hipMemcpy(al.data(), w + L.alpha, sizeof(double) * al.size(), hipMemcpyDeviceToHost));
    HM_HIP(hipMemcpy(be.data(), w + L.beta, sizeof(double) * be.size(), hipMemcpyDeviceToHost));
    HM_HIP(hipMemcpy(stop.data(), w + L.stopped, sizeof(int) * npairs, hipMemcpyDeviceToHost));
    for (int k = 0; k < ninst; ++k)
        for (int q = 0; q < nvec; ++q) {
            const size_t p = (size_t)k * L.NV + q, o = ((size_t)k * nvec + q) * steps;
            if (stop[p] < 0) return fail(HM_EINVAL, "start vector %d of instance %d is zero", q, k);
            const int done = stop[p] > 0 ? stop[p] : steps;
            for (int s = 0; s < steps; ++s) {
                alpha[o + s] = s < done ? al[p * steps + s] : 0.0;
                beta[o + s] = s < done ? be[p * steps + s] : 0.0;
            }
            steps_done[k * nvec + q] = done;
            HM_TRY(hm_tridiag_lowest(done, alpha + o, beta + o, &E0[k * nvec + q], nullptr));
        }
    return HM_OK;
}

}  // extern "C"
