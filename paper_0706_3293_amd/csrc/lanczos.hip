// Lanczos three-term recurrence on the GPU (Paige's ordering), the
// ground-state recompute pass and the host tridiagonal eigensolver.
//
// Step k (0-based) with v_k = sigma_k r_k kept as a raw vector r_k and a
// device scalar sigma_k:
//   pass A  w = sigma_k (H r_k) - cprev_k r_{k-1}      [fused in the H x kernel]
//           alpha partials  <w, v_k>                   [same kernel, FP64]
//   finish  alpha_k = sum of partials                  [one workgroup, fixed order]
//   pass B  w -= alpha_k v_k,  partials of |w|^2       [FP64 arithmetic]
//   [reorth twice: h = V^T w, w -= V h]
//   finish  beta_k = |w|; breakdown test; sigma_{k+1} = 1/beta_k,
//           cprev_{k+1} = beta_k sigma_k
// The raw buffers rotate (r_{k+1} is w), so the 1/beta normalization never
// costs a vector pass.  All reductions are per-workgroup partials summed in a
// fixed order: two runs with the same inputs give the same bits, which the
// recompute pass relies on.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "device_common.h"
#include "hm_internal.h"
#include "hx_row.h"

namespace hm {

int launch_hx_generic(const Basis *b, const Couplings *c, int dtype, const HxPass &p,
                      hipStream_t st);
int hx_generic_grid(const Basis *b);
int launch_hx_half(const Basis *b, const Couplings *c, int dtype, const HxPass &p,
                   hipStream_t st);
int hx_half_grid(const Basis *b);
bool half_supported(const Basis *b);
int half_prepare_tables(Basis *b, const Couplings *c);
bool half_fits(const Basis *b, const Couplings *c);

// 0 = automatic (the spin-1/2 block kernel when it applies to the basis and
// its neighbour table fits the budget, else the generic digit kernel),
// 1 = generic, 2 = block kernel (-1 if it does not apply).
int choose_kernel(const Basis *b, const Couplings *c, int requested) {
    if (requested == 1) return 1;
    const bool ok = c ? half_fits(b, c) : half_supported(b);
    if (requested == 2) return ok ? 2 : -1;
    return ok ? 2 : 1;
}

int hx_partial_count(const Basis *b, int kernel) {
    return kernel == 2 ? hx_half_grid(b) : hx_generic_grid(b);
}

int launch_hx(const Basis *b, const Couplings *c, int dtype, int kernel, const HxPass &p,
              hipStream_t st) {
    if (kernel == 2) return launch_hx_half(b, c, dtype, p, st);
    return launch_hx_generic(b, c, dtype, p, st);
}

// Device-side scalars of one Lanczos run.
struct LzDev {
    int stopped;     // steps done when a breakdown ended the run; 0 while running
    int bad_start;   // 1 if |v0| == 0
    double tol;
    double scale;    // running max(|alpha_j|, beta_j)
    double norm0;    // |v0|
    double psi_norm;
    unsigned ticket; // workgroups of the current fused pass B that are done
};

// One-workgroup run (below): automatic choice without reorthogonalization up
// to kSmallAutoWork (rows x bonds) of row work per step, accepted when asked
// for explicitly up to kSmallMaxDim rows.
constexpr int64_t kSmallAutoWork = 16384;
constexpr int64_t kSmallMaxDim = 1 << 20;

struct Layout {
    size_t lz, alpha, beta, sigma, cprev, coef, hcoef, partial, bpart, r0, r1, r2, V, states,
        total;
    int grid_vec, grid_b, nparts;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int vec_grid(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    g = std::min<int64_t>(g, kMaxGrid);
    g = std::max<int64_t>(g, 1);
    if (g >= kXcds) g -= g % kXcds;
    return (int)g;
}

// Workgroups of pass B: about 8 16-byte vectors per thread, so that long
// vectors run on many more workgroups than fit at once and the dispatcher
// keeps every CU busy to the end (601 M FP32 rows: 1.51 ms on 2048
// workgroups, 1.36 ms on 65536).
constexpr int64_t kMaxGridB = 65536;
static int pass_b_grid(int64_t n, size_t es) {
    const int64_t per = (int64_t)(16 / es) * kBlock * 8;
    int64_t g = std::min<int64_t>((n + per - 1) / per, kMaxGridB);
    g = std::max<int64_t>(g, vec_grid(n));
    if (g >= kXcds) g -= g % kXcds;
    return (int)g;
}

// Workspace layout; the partial-sum area holds one entry per workgroup of
// pass B and of whichever H x kernel may run (kMaxGrid, or the block kernel's grid when its
// schedule asks for more), so the layout does not depend on the kernel choice.
static Layout layout(const Basis *b, int steps, int prec, int reorth) {
    Layout L{};
    const size_t es = prec == HM_PREC_F64 ? 8 : 4;
    L.grid_vec = vec_grid(b->dim);
    L.grid_b = pass_b_grid(b->dim, es);
    L.nparts = std::max({kMaxGrid, L.grid_b, half_supported(b) ? hx_half_grid(b) : 0});
    size_t partial_len = (size_t)L.nparts;
    if (reorth) partial_len = std::max(partial_len, (size_t)L.grid_vec * (size_t)steps);
    size_t off = 0;
    L.lz = off; off = align256(off + sizeof(LzDev));
    L.alpha = off; off = align256(off + sizeof(double) * steps);
    L.beta = off; off = align256(off + sizeof(double) * steps);
    L.sigma = off; off = align256(off + sizeof(double) * (steps + 1));
    L.cprev = off; off = align256(off + sizeof(double) * (steps + 1));
    L.coef = off; off = align256(off + sizeof(double) * steps);
    L.hcoef = off; off = align256(off + sizeof(double) * (steps + 1));
    L.partial = off; off = align256(off + sizeof(double) * partial_len);
    L.bpart = off; off = align256(off + sizeof(double) * kMaxGrid);
    L.r0 = off; off = align256(off + es * (size_t)b->dim);
    L.r1 = off; off = align256(off + es * (size_t)b->dim);
    L.r2 = off; off = align256(off + es * (size_t)b->dim);
    L.V = off;
    if (reorth) off = align256(off + es * (size_t)b->dim * (size_t)steps);
    // decoded states of the one-workgroup run (any basis it may take)
    L.states = off;
    if (b->dim <= kSmallMaxDim) off = align256(off + sizeof(uint64_t) * (size_t)b->dim);
    L.total = off;
    return L;
}

// ---------------------------------------------------------------------------
// Vector kernels.  Each workgroup owns one contiguous slice of rows (XCD-aware
// order) and writes one FP64 partial.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void sumsq_kernel(const T *__restrict__ x, int64_t n,
                                                       double *__restrict__ partial,
                                                       const int *__restrict__ stopped) {
    if (stopped && *stopped) return;
    __shared__ double red[16];
    int64_t first, last;
    block_rows<int64_t>(xcd_logical_block(blockIdx.x, gridDim.x), gridDim.x, n, first, last);
    double s = 0.0;
    for (int64_t i = first + threadIdx.x; i < last; i += blockDim.x) {
        const double v = (double)x[i];
        s += v * v;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Sum of n partials in a fixed order by one workgroup: thread t adds
// partials t, t + blockDim, t + 2 blockDim, ... in that order, then the wave
// and workgroup sums combine the threads in a fixed order.
__device__ double fixed_sum(const double *__restrict__ partial, int n, double *red) {
    // 16 loads in flight per thread before their additions (large grids of
    // the H x pass write up to 2^20 partials; their loads are served from
    // beyond L2, since other XCDs wrote them)
    constexpr int U = 16;
    const int stride = blockDim.x;
    double s = 0.0;
    int t = threadIdx.x;
    for (; t + (U - 1) * stride < n; t += U * stride) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = partial[t + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) s += v[u];
    }
    for (; t < n; t += stride) s += partial[t];
    return block_sum(s, red);
}

// Threads of the finish that sums the H x pass's partials (one per workgroup
// of that pass, up to 2^20): 16 waves, the most block_sum combines.
constexpr int kFinishBlock = 1024;

__global__ __launch_bounds__(kBlock) void finish_init(LzDev *lz, const double *partial, int n,
                                                      double *sigma, double *cprev,
                                                      double tol) {
    __shared__ double red[16];
    const double s = fixed_sum(partial, n, red);
    if (threadIdx.x == 0) {
        lz->stopped = 0;
        lz->tol = tol;
        lz->scale = 0.0;
        lz->norm0 = sqrt(s);
        lz->bad_start = !(s > 0.0);
        lz->psi_norm = 0.0;
        lz->ticket = 0;
        sigma[0] = 1.0;
        cprev[0] = 0.0;
        if (lz->bad_start) lz->stopped = -1;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void init_write(const double *__restrict__ v0,
                                                     T *__restrict__ r, int64_t n,
                                                     const LzDev *__restrict__ lz) {
    if (lz->stopped) return;
    const double inv = 1.0 / lz->norm0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        r[i] = (T)(v0[i] * inv);
}

__global__ __launch_bounds__(kFinishBlock) void finish_alpha(LzDev *lz, const double *partial,
                                                             int n, double *alpha, int k) {
    if (lz->stopped) return;
    __shared__ double red[16];
    const double s = fixed_sum(partial, n, red);
    if (threadIdx.x == 0) alpha[k] = s;
}

// 16-byte vector type of an element type.
template <typename T> struct VecOf;
template <> struct VecOf<float> { using type = float4; };
template <> struct VecOf<double> { using type = double2; };

// w -= alpha_k sigma_k r_k (FP64 arithmetic, one rounding), partial |w|^2.
template <typename T>
__global__ __launch_bounds__(kBlock) void pass_b(T *__restrict__ w, const T *__restrict__ r,
                                                 int64_t n, const LzDev *__restrict__ lz,
                                                 const double *__restrict__ alpha,
                                                 const double *__restrict__ sigma, int k,
                                                 double *__restrict__ partial) {
    if (lz->stopped) return;
    __shared__ double red[16];
    const double a = alpha[k] * sigma[k];
    int64_t first, last;
    block_rows<int64_t>(xcd_logical_block(blockIdx.x, gridDim.x), gridDim.x, n, first, last);
    // 16-byte vector loads and stores over the aligned middle of the range
    // (the buffers start on 256-byte boundaries), single elements at its ends
    constexpr int V = 16 / sizeof(T);
    using Vec = typename VecOf<T>::type;
    const int64_t m0 = std::min(last, (first + V - 1) / V * V);
    const int64_t m1 = std::max(m0, last / V * V);
    double s = 0.0;
    for (int64_t i = first + threadIdx.x; i < m0; i += blockDim.x) {
        const T wi = (T)((double)w[i] - a * (double)r[i]);
        w[i] = wi;
        s += (double)wi * (double)wi;
    }
    Vec *wv = reinterpret_cast<Vec *>(w);
    const Vec *rv = reinterpret_cast<const Vec *>(r);
#pragma unroll 2
    for (int64_t j = m0 / V + threadIdx.x; j < m1 / V; j += blockDim.x) {
        Vec wj = wv[j];
        const Vec rj = rv[j];
        T *we = reinterpret_cast<T *>(&wj);
        const T *re = reinterpret_cast<const T *>(&rj);
#pragma unroll
        for (int e = 0; e < V; ++e) {
            we[e] = (T)((double)we[e] - a * (double)re[e]);
            s += (double)we[e] * (double)we[e];
        }
        wv[j] = wj;
    }
    for (int64_t i = m1 + threadIdx.x; i < last; i += blockDim.x) {
        const T wi = (T)((double)w[i] - a * (double)r[i]);
        w[i] = wi;
        s += (double)wi * (double)wi;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kFinishBlock) void finish_beta(LzDev *lz, const double *partial,
                                                            int n, const double *alpha,
                                                            double *beta, double *sigma,
                                                            double *cprev, int k) {
    if (lz->stopped) return;
    __shared__ double red[16];
    const double s = fixed_sum(partial, n, red);
    if (threadIdx.x == 0) {
        const double b = sqrt(s);
        beta[k] = b;
        const double sc = fmax(lz->scale, fmax(fabs(alpha[k]), b));
        lz->scale = sc;
        if (!(b > lz->tol * sc)) {
            lz->stopped = k + 1;
        } else {
            sigma[k + 1] = 1.0 / b;
            cprev[k + 1] = b * sigma[k];
        }
    }
}

// Pass B with the one-workgroup finishes folded in, for small grids (a few
// dozen workgroups), where launches dominate a step.  Every workgroup sums
// the H x partials (alpha_k) in the same fixed order, so all use the same
// alpha, and applies w -= alpha_k sigma_k r_k.
//   MODE 0: nothing more (reorthogonalization follows, then sumsq_kernel and
//           finish_beta);
//   MODE 2: each workgroup writes its |w|^2 partial to bpart and takes a
//           device-scope ticket; the last one to arrive sums bpart in a fixed
//           order and does what finish_beta does, then resets the ticket for
//           the next step.
// On large grids both cost more than they save (every workgroup re-reads all
// H x partials, and the tickets are one contended atomic per workgroup), so
// there the step keeps finish_alpha, pass_b and finish_beta.
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void pass_b_fused(
    T *__restrict__ w, const T *__restrict__ r, int64_t n, LzDev *lz,
    const double *__restrict__ hx_partial, int n_hx, double *alpha, double *beta, double *sigma,
    double *cprev, int k, double *bpart) {
    if (lz->stopped) return;
    __shared__ double red[16];
    __shared__ double s_alpha;
    __shared__ int s_last;
    const double a_sum = fixed_sum(hx_partial, n_hx, red);
    if (threadIdx.x == 0) {
        s_alpha = a_sum;
        if (blockIdx.x == 0) alpha[k] = a_sum;
    }
    __syncthreads();
    const double al = s_alpha;
    const double a = al * sigma[k];
    int64_t first, last;
    block_rows<int64_t>(xcd_logical_block(blockIdx.x, gridDim.x), gridDim.x, n, first, last);
    double s = 0.0;
    for (int64_t i = first + threadIdx.x; i < last; i += blockDim.x) {
        const T wi = (T)((double)w[i] - a * (double)r[i]);
        w[i] = wi;
        s += (double)wi * (double)wi;
    }
    if constexpr (MODE == 2) {
        s = block_sum(s, red);
        if (threadIdx.x == 0) {
            bpart[blockIdx.x] = s;
            // the release orders the partial before the ticket; the last
            // workgroup acquires every partial before summing them
            const unsigned t = __hip_atomic_fetch_add(&lz->ticket, 1u, __ATOMIC_RELEASE,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            s_last = t == gridDim.x - 1;
            if (s_last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (!s_last) return;
        const double b2 = fixed_sum(bpart, gridDim.x, red);
        if (threadIdx.x == 0) {
            lz->ticket = 0;
            const double b = sqrt(b2);
            beta[k] = b;
            const double sc = fmax(lz->scale, fmax(fabs(al), b));
            lz->scale = sc;
            if (!(b > lz->tol * sc)) {
                lz->stopped = k + 1;
            } else {
                sigma[k + 1] = 1.0 / b;
                cprev[k + 1] = b * sigma[k];
            }
        }
    }
}

// Reorthogonalization: partial[j * G + blk] = sum_i V[j][i] w_i over the slice.
template <typename T>
__global__ __launch_bounds__(kBlock) void reorth_dots(const T *__restrict__ V,
                                                      const T *__restrict__ w, int64_t n,
                                                      int nv, double *__restrict__ partial,
                                                      const LzDev *__restrict__ lz) {
    if (lz->stopped) return;
    __shared__ double red[16];
    const int j = blockIdx.y;
    int64_t first, last;
    block_rows<int64_t>(xcd_logical_block(blockIdx.x, gridDim.x), gridDim.x, n, first, last);
    double s = 0.0;
    const T *Vj = V + (size_t)j * (size_t)n;
    for (int64_t i = first + threadIdx.x; i < last; i += blockDim.x)
        s += (double)Vj[i] * (double)w[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[(size_t)j * gridDim.x + blockIdx.x] = s;
}

// h_j = sum of the G partials of coefficient j: one wave per j (blockIdx.x),
// lanes over the partials, a fixed butterfly.
__global__ __launch_bounds__(64) void reorth_finish(const double *partial, int G, double *h,
                                                    const LzDev *lz) {
    if (lz->stopped) return;
    const int j = blockIdx.x;
    double s = 0.0;
    for (int t = threadIdx.x; t < G; t += 64) s += partial[(size_t)j * G + t];
    s = wave_sum(s);
    if (threadIdx.x == 0) h[j] = s;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void reorth_update(const T *__restrict__ V,
                                                        T *__restrict__ w, int64_t n, int nv,
                                                        const double *__restrict__ h,
                                                        const LzDev *__restrict__ lz) {
    if (lz->stopped) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double acc = (double)w[i];
        for (int j = 0; j < nv; ++j) acc -= h[j] * (double)V[(size_t)j * (size_t)n + i];
        w[i] = (T)acc;
    }
}

__global__ __launch_bounds__(kBlock) void finish_psi_norm(LzDev *lz, const double *partial,
                                                          int n) {
    __shared__ double red[16];
    const double s = fixed_sum(partial, n, red);
    if (threadIdx.x == 0) lz->psi_norm = sqrt(s);
}

__global__ __launch_bounds__(kBlock) void scale_psi(double *__restrict__ psi, int64_t n,
                                                    const LzDev *__restrict__ lz) {
    const double nrm = lz->psi_norm;
    if (!(nrm > 0.0)) return;
    const double inv = 1.0 / nrm;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        psi[i] *= inv;
}

// Ground-state accumulation psi += c_k v_k = c_k sigma_k r_k in FP64.  Kept out
// of the H x kernel so both Lanczos passes run the same recurrence kernels.
template <typename T>
__global__ __launch_bounds__(kBlock) void psi_axpy(double *__restrict__ psi,
                                                   const T *__restrict__ r, int64_t n,
                                                   const double *__restrict__ coef,
                                                   const double *__restrict__ sigma,
                                                   const LzDev *__restrict__ lz) {
    if (lz->stopped) return;
    const double a = coef[0] * sigma[0];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        psi[i] += a * (double)r[i];
}

__global__ void zero_f64(double *__restrict__ x, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = 0.0;
}

// ---------------------------------------------------------------------------
// Small problems: the whole run in one workgroup.
//
// For a few thousand rows a step is little work, but the multi-kernel step
// costs two launches (ten with full reorthogonalization).  Here one
// workgroup of 1024 threads runs every step in a single launch: thread t owns
// rows t, t + 1024, ... (the generic row of hx_row.h, on states decoded once
// at the start and kept in the workspace), reductions are fixed
// trees (block_sum, wave_sum), and workgroup barriers order the passes, so a
// run is reproducible and the recompute pass repeats it bit for bit.  The
// recurrence is the same (Paige's ordering, the same breakdown test); v_k is
// stored normalized.  One compute unit does all the row work, so the run pays
// off only while that work stays below the launch costs it saves.  Measured
// against directly launched steps, without reorthogonalization: faster at 70
// rows x 8 bonds (0.46 vs 0.65 ms, 60 steps), 924 x 12 (1.4 vs 1.7 ms, 120
// steps) and 1107 x 7 (1.2 vs 1.7 ms, 100 steps); slower at 3432 x 14 (5.2
// vs 2.7 ms, 150 steps) and 2024 x 48 (5.4 ms, 150 steps).  With
// reorthogonalization, whose k-term sums run on this one workgroup, it is
// slower already at 924 rows (7.7 vs 5.3 ms).
// ---------------------------------------------------------------------------
constexpr int kSmallBlock = 1024;

template <typename T, typename I>
struct SmallArgs {
    const I *prefix;
    const double *ladder;
    const BondDev *bonds;
    int nb, N, A, two_s, steps, reorth;
    I dim;
    double tol;
    const double *v0;
    T *buf[3];
    T *V;                    // [steps][dim] normalized v_j (full reorthogonalization)
    uint64_t *states;        // [dim] decoded states, filled at the start of the run
    double *alpha, *beta, *hc;
    LzDev *lz;
    const double *coef;      // recompute pass: c_k, else nullptr
    double *psi;
};

__device__ __forceinline__ double block_bcast(double v, double *red, double *slot) {
    v = block_sum(v, red);
    if (threadIdx.x == 0) *slot = v;
    __syncthreads();
    const double r = *slot;
    __syncthreads();
    return r;
}

template <typename T, typename I, int B>
__global__ __launch_bounds__(kSmallBlock) void lanczos_small_kernel(const SmallArgs<T, I> a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[16];
    __shared__ double slot;
    const int plen = a.N * (a.A + 1) * (a.two_s + 1);
    I *P = reinterpret_cast<I *>(smem);
    T *F = reinterpret_cast<T *>(smem + ((plen * sizeof(I) + 15) / 16) * 16);
    for (int t = threadIdx.x; t < plen; t += blockDim.x) P[t] = a.prefix[t];
    for (int t = threadIdx.x; t < a.two_s + 2; t += blockDim.x) F[t] = (T)a.ladder[t];
    __syncthreads();
    const Prefix<I> pv{P, a.A + 1, a.two_s + 1};
    const I n = a.dim;
    const I tid = threadIdx.x, nt = blockDim.x;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nwv = blockDim.x >> 6;

    double s = 0.0;
    for (I i = tid; i < n; i += nt) s += a.v0[i] * a.v0[i];
    s = block_bcast(s, red, &slot);
    if (threadIdx.x == 0) {
        a.lz->tol = a.tol;
        a.lz->norm0 = sqrt(s);
        a.lz->bad_start = !(s > 0.0);
        a.lz->stopped = a.lz->bad_start ? -1 : 0;
        a.lz->psi_norm = 0.0;
    }
    if (!(s > 0.0)) return;
    const double inv0 = 1.0 / sqrt(s);
    for (I i = tid; i < n; i += nt) {
        const T v = (T)(a.v0[i] * inv0);
        a.buf[0][i] = v;
        if (a.reorth) a.V[i] = v;
        if (a.psi) a.psi[i] = 0.0;
        a.states[i] = unrank_state<I, B>(i, pv, a.N, a.A, a.two_s);
    }
    __syncthreads();
    double beta_prev = 0.0, scale = 0.0;
    int stopped = 0;
    for (int k = 0; k < a.steps; ++k) {
        const T *__restrict__ vk = a.buf[k % 3];
        const T *__restrict__ vp = a.buf[(k + 2) % 3];
        T *__restrict__ w = a.buf[(k + 1) % 3];
        // w = H v_k - beta_{k-1} v_{k-1};  alpha_k = <w, v_k>
        double dot = 0.0;
        for (I i = tid; i < n; i += nt) {
            const uint64_t st = a.states[i];
            const T xi = vk[i];
            const T hv = row_hx<T, I, B>(st, i, xi, vk, a.bonds, a.nb, a.two_s, pv, F);
            double wi = (double)hv;
            if (k > 0) wi -= beta_prev * (double)vp[i];
            const T wt = (T)wi;
            w[i] = wt;
            dot += (double)wt * (double)xi;
            if (a.psi) a.psi[i] += a.coef[k] * (double)xi;
        }
        const double alpha = block_bcast(dot, red, &slot);
        // w -= alpha_k v_k (rows of this thread only)
        double ss = 0.0;
        for (I i = tid; i < n; i += nt) {
            const T wi = (T)((double)w[i] - alpha * (double)vk[i]);
            w[i] = wi;
            ss += (double)wi * (double)wi;
        }
        if (a.reorth) {
            __syncthreads();
            for (int rep = 0; rep < 2; ++rep) {
                // h_j = <V_j, w>: one wave per j, lanes over rows, fixed tree
                for (int j = wid; j <= k; j += nwv) {
                    const T *__restrict__ Vj = a.V + (size_t)j * (size_t)n;
                    double d = 0.0;
                    for (I i = lane; i < n; i += 64) d += (double)Vj[i] * (double)w[i];
                    d = wave_sum(d);
                    if (lane == 0) a.hc[j] = d;
                }
                __syncthreads();
                for (I i = tid; i < n; i += nt) {
                    double acc = (double)w[i];
                    for (int j = 0; j <= k; ++j) acc -= a.hc[j] * (double)a.V[(size_t)j * n + i];
                    w[i] = (T)acc;
                }
                __syncthreads();
            }
            ss = 0.0;
            for (I i = tid; i < n; i += nt) ss += (double)w[i] * (double)w[i];
        }
        const double beta = sqrt(block_bcast(ss, red, &slot));
        scale = fmax(scale, fmax(fabs(alpha), beta));
        if (threadIdx.x == 0) {
            a.alpha[k] = alpha;
            a.beta[k] = beta;
            a.lz->scale = scale;
        }
        if (!(beta > a.tol * scale)) {
            stopped = k + 1;
            break;
        }
        const double binv = 1.0 / beta;
        for (I i = tid; i < n; i += nt) {
            const T v = (T)((double)w[i] * binv);
            w[i] = v;
            if (a.reorth && k + 1 < a.steps) a.V[(size_t)(k + 1) * n + i] = v;
        }
        beta_prev = beta;
        __syncthreads();
    }
    if (threadIdx.x == 0) a.lz->stopped = stopped;
    if (a.psi) {
        __syncthreads();
        double q = 0.0;
        for (I i = tid; i < n; i += nt) q += a.psi[i] * a.psi[i];
        const double nrm = sqrt(block_bcast(q, red, &slot));
        if (threadIdx.x == 0) a.lz->psi_norm = nrm;
        if (nrm > 0.0)
            for (I i = tid; i < n; i += nt) a.psi[i] /= nrm;
    }
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
static thread_local bool g_timing = false;
static thread_local double g_hx_ms = 0.0, g_loop_ms = 0.0;
static thread_local int g_hx_launches = 0;

struct Run {
    Basis *b;
    const Couplings *c;
    int steps, prec, reorth, kernel, use_graph, small;
    double tol;
    Layout L;
    unsigned char *w;
    hipStream_t st;
    const double *v0;
    const double *coef_host;   // ritz pass: c_k (host), else nullptr
    double *psi;               // ritz pass output, else nullptr
};

// Largest grids (pass B and the H x partials) for the fused pass B.
constexpr int kFusedMaxGrid = 64;

template <typename T>
static int enqueue_steps(Run &R, int k0, int k1, std::vector<hipEvent_t> *ev) {
    Basis *b = R.b;
    const int64_t n = b->dim;
    LzDev *lz = (LzDev *)(R.w + R.L.lz);
    double *alpha = (double *)(R.w + R.L.alpha), *beta = (double *)(R.w + R.L.beta);
    double *sigma = (double *)(R.w + R.L.sigma), *cprev = (double *)(R.w + R.L.cprev);
    double *coef = (double *)(R.w + R.L.coef), *hc = (double *)(R.w + R.L.hcoef);
    double *partial = (double *)(R.w + R.L.partial), *bpart = (double *)(R.w + R.L.bpart);
    T *buf[3] = {(T *)(R.w + R.L.r0), (T *)(R.w + R.L.r1), (T *)(R.w + R.L.r2)};
    T *V = (T *)(R.w + R.L.V);
    const int G = R.L.grid_vec, Gb = R.L.grid_b;
    const int Ghx = hx_partial_count(b, R.kernel);
    const int dtype = R.prec == HM_PREC_F64 ? HM_F64 : HM_F32;
    for (int k = k0; k < k1; ++k) {
        T *rk = buf[k % 3], *rprev = buf[(k + 2) % 3], *wn = buf[(k + 1) % 3];
        HxPass p;
        p.x = rk;
        p.y = wn;
        p.p = k > 0 ? rprev : nullptr;
        p.sigma = sigma + k;
        p.cprev = cprev + k;
        p.partial = partial;
        p.store = R.reorth ? (void *)(V + (size_t)k * (size_t)n) : nullptr;
        p.stopped = &lz->stopped;
        if (ev) HM_HIP(hipEventRecord((*ev)[2 * k], R.st));
        HM_TRY(launch_hx(b, R.c, dtype, R.kernel, p, R.st));
        if (ev) HM_HIP(hipEventRecord((*ev)[2 * k + 1], R.st));
        if (R.psi)
            hipLaunchKernelGGL(psi_axpy<T>, dim3(G), dim3(kBlock), 0, R.st, R.psi, rk, n,
                               coef + k, sigma + k, lz);
        const bool small = G <= kFusedMaxGrid && Ghx <= kFusedMaxGrid;
        if (small && !R.reorth) {
            // pass B with both finishes: two launches per step in all
            hipLaunchKernelGGL((pass_b_fused<T, 2>), dim3(G), dim3(kBlock), 0, R.st, wn, rk, n,
                               lz, partial, Ghx, alpha, beta, sigma, cprev, k, bpart);
            continue;
        }
        if (small) {
            hipLaunchKernelGGL((pass_b_fused<T, 0>), dim3(G), dim3(kBlock), 0, R.st, wn, rk, n,
                               lz, partial, Ghx, alpha, beta, sigma, cprev, k, bpart);
        } else {
            hipLaunchKernelGGL(finish_alpha, dim3(1), dim3(kFinishBlock), 0, R.st, lz, partial, Ghx,
                               alpha, k);
            hipLaunchKernelGGL(pass_b<T>, dim3(Gb), dim3(kBlock), 0, R.st, wn, rk, n, lz, alpha,
                               sigma, k, partial);
        }
        if (!R.reorth) {
            hipLaunchKernelGGL(finish_beta, dim3(1), dim3(kFinishBlock), 0, R.st, lz, partial, Gb,
                               alpha, beta, sigma, cprev, k);
            continue;
        }
        // with full reorthogonalization beta is the norm after it
        for (int rep = 0; rep < 2; ++rep) {
            hipLaunchKernelGGL(reorth_dots<T>, dim3(G, k + 1), dim3(kBlock), 0, R.st, V, wn, n,
                               k + 1, partial, lz);
            hipLaunchKernelGGL(reorth_finish, dim3(k + 1), dim3(64), 0, R.st, partial, G, hc,
                               lz);
            hipLaunchKernelGGL(reorth_update<T>, dim3(G), dim3(kBlock), 0, R.st, V, wn, n,
                               k + 1, hc, lz);
        }
        hipLaunchKernelGGL(sumsq_kernel<T>, dim3(G), dim3(kBlock), 0, R.st, wn, n, partial,
                           &lz->stopped);
        hipLaunchKernelGGL(finish_beta, dim3(1), dim3(kFinishBlock), 0, R.st, lz, partial, G, alpha,
                           beta, sigma, cprev, k);
    }
    HM_HIP(hipGetLastError());
    return HM_OK;
}

// Waits for the run and copies its results to the host.
static int collect(const Run &R, double *alpha_h, double *beta_h, int *steps_done) {
    HM_HIP(hipGetLastError());
    HM_HIP(hipStreamSynchronize(R.st));
    LzDev hlz;
    HM_HIP(hipMemcpy(&hlz, R.w + R.L.lz, sizeof hlz, hipMemcpyDeviceToHost));
    if (hlz.bad_start) return fail(HM_EINVAL, "start vector has zero norm");
    const int done = hlz.stopped > 0 ? hlz.stopped : R.steps;
    if (alpha_h)
        HM_HIP(hipMemcpy(alpha_h, R.w + R.L.alpha, sizeof(double) * done, hipMemcpyDeviceToHost));
    if (beta_h)
        HM_HIP(hipMemcpy(beta_h, R.w + R.L.beta, sizeof(double) * done, hipMemcpyDeviceToHost));
    if (alpha_h) std::fill(alpha_h + done, alpha_h + R.steps, 0.0);
    if (beta_h) std::fill(beta_h + done, beta_h + R.steps, 0.0);
    *steps_done = done;
    return HM_OK;
}

template <typename T, typename I, int B>
static void launch_small_b(const Run &R) {
    const Basis *b = R.b;
    SmallArgs<T, I> a{};
    a.prefix = (const I *)b->d_prefix;
    a.ladder = b->d_ladder;
    a.bonds = R.c->dev;
    a.nb = R.c->nb;
    a.N = b->N;
    a.A = b->A;
    a.two_s = b->two_s;
    a.steps = R.steps;
    a.reorth = R.reorth;
    a.dim = (I)b->dim;
    a.tol = R.tol;
    a.v0 = R.v0;
    a.buf[0] = (T *)(R.w + R.L.r0);
    a.buf[1] = (T *)(R.w + R.L.r1);
    a.buf[2] = (T *)(R.w + R.L.r2);
    a.V = (T *)(R.w + R.L.V);
    a.states = (uint64_t *)(R.w + R.L.states);
    a.alpha = (double *)(R.w + R.L.alpha);
    a.beta = (double *)(R.w + R.L.beta);
    a.hc = (double *)(R.w + R.L.hcoef);
    a.lz = (LzDev *)(R.w + R.L.lz);
    a.coef = R.psi ? (const double *)(R.w + R.L.coef) : nullptr;
    a.psi = R.psi;
    const size_t lds = ((prefix_bytes(b) + 15) / 16) * 16 + (b->two_s + 2) * sizeof(double);
    hipLaunchKernelGGL((lanczos_small_kernel<T, I, B>), dim3(1), dim3(kSmallBlock), lds, R.st,
                       a);
}

template <typename T>
static int launch_small(const Run &R) {
    HM_TRY(check_lds(R.b));
    if (!R.b->idx32) return fail(HM_ERANGE, "the one-workgroup run needs 32-bit prefix tables");
    switch (R.b->bits) {
        case 1: launch_small_b<T, uint32_t, 1>(R); break;
        case 2: launch_small_b<T, uint32_t, 2>(R); break;
        case 3: launch_small_b<T, uint32_t, 3>(R); break;
        case 4: launch_small_b<T, uint32_t, 4>(R); break;
        case 5: launch_small_b<T, uint32_t, 5>(R); break;
        case 6: launch_small_b<T, uint32_t, 6>(R); break;
        case 7: launch_small_b<T, uint32_t, 7>(R); break;
        case 8: launch_small_b<T, uint32_t, 8>(R); break;
        default: return fail(HM_ERANGE, "bits per digit %d unsupported", R.b->bits);
    }
    HM_HIP(hipGetLastError());
    return HM_OK;
}

// The instantiated graph of the whole step loop for this run.  A capture
// bakes in the kernels and every argument of the step loop: the coupling list
// (by its serial number), the workspace address, the number of steps, the
// precision, reorthogonalization, the H x kernel and the ground-state output
// (the recompute pass), and through the basis handle its schedule and tables.
// The start vector, the breakdown tolerance and the recompute coefficients
// are not part of it: the initialization runs before the graph and leaves
// them in the workspace.  A handle keeps kGraphCacheEntries graphs, least
// recently used first out.
template <typename T>
static int step_graph(Run &R, hipGraphExec_t *out) {
    Basis *b = R.b;
    const std::vector<uint64_t> key = {R.c->serial, (uint64_t)(uintptr_t)R.w,
                                       (uint64_t)R.steps, (uint64_t)R.prec, (uint64_t)R.reorth,
                                       (uint64_t)R.kernel, (uint64_t)(uintptr_t)R.psi,
                                       (uint64_t)sizeof(T)};
    {
        std::lock_guard<std::mutex> lock(b->mu);
        for (auto it = b->graphs.begin(); it != b->graphs.end(); ++it)
            if (it->key == key) {
                b->graphs.splice(b->graphs.begin(), b->graphs, it);
                *out = b->graphs.front().exec;
                return HM_OK;
            }
    }
    hipGraph_t graph = nullptr;
    HM_HIP(hipStreamBeginCapture(R.st, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_steps<T>(R, 0, R.steps, nullptr);
    hipError_t e = hipStreamEndCapture(R.st, &graph);
    if (rc != HM_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(HM_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(HM_EDEVICE, "graph instantiation: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lock(b->mu);
    while (b->graphs.size() >= kGraphCacheEntries) {
        // no launch of it can be pending when it is dropped: the run that
        // used it synchronized its stream before returning
        if (b->graphs.back().exec) (void)hipGraphExecDestroy(b->graphs.back().exec);
        b->graphs.pop_back();
    }
    b->graphs.push_front(Basis::Graph{key, exec});
    *out = exec;
    return HM_OK;
}

template <typename T>
static int run_lanczos(Run &R, double *alpha_h, double *beta_h, int *steps_done) {
    Basis *b = R.b;
    const int64_t n = b->dim;
    LzDev *lz = (LzDev *)(R.w + R.L.lz);
    double *partial = (double *)(R.w + R.L.partial);
    double *sigma = (double *)(R.w + R.L.sigma), *cprev = (double *)(R.w + R.L.cprev);
    T *r0 = (T *)(R.w + R.L.r0);
    const int G = R.L.grid_vec;
    if (R.psi) {
        HM_HIP(hipMemcpyAsync(R.w + R.L.coef, R.coef_host, sizeof(double) * R.steps,
                              hipMemcpyHostToDevice, R.st));
        if (!R.small) hipLaunchKernelGGL(zero_f64, dim3(G), dim3(kBlock), 0, R.st, R.psi, n);
    }
    if (R.small) {
        HM_TRY(launch_small<T>(R));
        return collect(R, alpha_h, beta_h, steps_done);
    }
    hipLaunchKernelGGL(sumsq_kernel<double>, dim3(G), dim3(kBlock), 0, R.st, R.v0, n, partial,
                       (const int *)nullptr);
    hipLaunchKernelGGL(finish_init, dim3(1), dim3(kBlock), 0, R.st, lz, partial, G, sigma,
                       cprev, R.tol);
    hipLaunchKernelGGL(init_write<T>, dim3(G), dim3(kBlock), 0, R.st, R.v0, r0, n, lz);
    HM_HIP(hipGetLastError());

    const bool timing = g_timing;
    // timing events, destroyed on every return path
    struct Events {
        std::vector<hipEvent_t> e;
        ~Events() {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } evs;
    std::vector<hipEvent_t> ev;
    hipEvent_t lo = nullptr, hi = nullptr;
    if (timing) {
        evs.e.assign(2 * (size_t)R.steps + 2, nullptr);
        for (auto &e : evs.e) HM_HIP(hipEventCreate(&e));
        ev.assign(evs.e.begin(), evs.e.begin() + 2 * (size_t)R.steps);
        lo = evs.e[2 * (size_t)R.steps];
        hi = evs.e[2 * (size_t)R.steps + 1];
        HM_HIP(hipEventRecord(lo, R.st));
    }
    int rc = HM_OK;
    if (R.use_graph && !timing) {
        // the step loop as one graph, captured and instantiated on the first
        // call with this key and replayed by later calls
        hipGraphExec_t exec = nullptr;
        HM_TRY(step_graph<T>(R, &exec));
        HM_HIP(hipGraphLaunch(exec, R.st));
    } else {
        rc = enqueue_steps<T>(R, 0, R.steps, timing ? &ev : nullptr);
        if (rc != HM_OK) return rc;
    }
    if (R.psi) {
        hipLaunchKernelGGL(sumsq_kernel<double>, dim3(G), dim3(kBlock), 0, R.st, R.psi, n,
                           partial, (const int *)nullptr);
        hipLaunchKernelGGL(finish_psi_norm, dim3(1), dim3(kBlock), 0, R.st, lz, partial, G);
        hipLaunchKernelGGL(scale_psi, dim3(G), dim3(kBlock), 0, R.st, R.psi, n, lz);
    }
    if (timing) HM_HIP(hipEventRecord(hi, R.st));
    HM_TRY(collect(R, alpha_h, beta_h, steps_done));
    const int done = *steps_done;
    if (timing) {
        double hx = 0.0;
        for (int k = 0; k < done; ++k) {
            float ms = 0.f;
            HM_HIP(hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]));
            hx += ms;
        }
        float loop = 0.f;
        HM_HIP(hipEventElapsedTime(&loop, lo, hi));
        g_hx_ms = hx;
        g_hx_launches = done;
        g_loop_ms = loop;
    }
    return HM_OK;
}

static int check_opts(const Basis *b, const hm_lanczos_opts *o) {
    if (!o) return fail(HM_EINVAL, "opts is null");
    if (o->precision != HM_PREC_F64 && o->precision != HM_PREC_F32_MIXED)
        return fail(HM_EINVAL, "unknown precision %d", o->precision);
    if (o->kernel < 0 || o->kernel > 3) return fail(HM_EINVAL, "unknown kernel %d", o->kernel);
    if (o->kernel == 3 && b->dim > kSmallMaxDim)
        return fail(HM_ERANGE, "the one-workgroup run takes at most %lld rows",
                    (long long)kSmallMaxDim);
    if (o->kernel != 3 && choose_kernel(b, nullptr, o->kernel) < 0)
        return fail(HM_EINVAL, "spin-1/2 block kernel not applicable to this basis");
    return HM_OK;
}

static int run_common(hm_basis h, const double *J, const double *d_v0, int32_t steps,
                      const hm_lanczos_opts *o, void *d_work, size_t work_bytes,
                      const double *coef, double *d_psi, double *alpha, double *beta,
                      int32_t *steps_done, void *stream) {
    if (!h || !d_v0 || !d_work || !steps_done) return fail(HM_EINVAL, "null argument");
    if (steps < 1) return fail(HM_EINVAL, "steps must be >= 1");
    Basis *b = &h->impl;
    HM_TRY(check_opts(b, o));
    CouplingsRef cref;
    HM_TRY(get_couplings(b, J, &cref));
    const Couplings *c = cref.get();
    const bool small = o->kernel == 3 || (o->kernel == 0 && !g_timing && !o->full_reorth &&
                                          b->dim * (int64_t)std::max(c->nb, 1) <= kSmallAutoWork);
    const int kernel = small ? 1 : choose_kernel(b, c, o->kernel);
    if (kernel < 0) return fail(HM_ERANGE, "block kernel tables too large for these couplings");
    if (kernel == 2) HM_TRY(half_prepare_tables(b, c));
    Run R{};
    R.small = small ? 1 : 0;
    R.b = b;
    R.c = c;
    R.steps = steps;
    R.prec = o->precision;
    R.reorth = o->full_reorth ? 1 : 0;
    R.kernel = kernel;
    R.use_graph = o->use_graph ? 1 : 0;
    R.tol = o->breakdown_tol > 0 ? o->breakdown_tol
                                 : (R.prec == HM_PREC_F64 ? 1e-12 : 1e-6);
    R.L = layout(b, steps, R.prec, R.reorth);
    if (work_bytes < R.L.total)
        return fail(HM_EWORKSPACE, "workspace %zu bytes < required %zu", work_bytes, R.L.total);
    R.w = (unsigned char *)d_work;
    R.v0 = d_v0;
    R.coef_host = coef;
    R.psi = d_psi;
    hipStream_t st = (hipStream_t)stream;
    hipStream_t own = nullptr;
    if (R.use_graph && st == nullptr) {
        // the null stream cannot be captured; a blocking stream orders
        // itself after earlier null-stream work
        HM_HIP(hipStreamCreate(&own));
        st = own;
    }
    R.st = st;
    int done = 0;
    int rc = R.prec == HM_PREC_F64 ? run_lanczos<double>(R, alpha, beta, &done)
                                   : run_lanczos<float>(R, alpha, beta, &done);
    if (own) (void)hipStreamDestroy(own);
    if (rc != HM_OK) return rc;
    *steps_done = done;
    return HM_OK;
}

// Lowest eigenvalue of the symmetric tridiagonal T by bisection on the Sturm
// count, then its eigenvector by inverse iteration.
static int sturm_count(int k, const double *a, const double *b, double x) {
    int neg = 0;
    double q = 1.0;
    for (int i = 0; i < k; ++i) {
        const double bb = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
        q = (a[i] - x) - (i > 0 ? bb / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) ++neg;
    }
    return neg;
}

static double lowest_eigenvalue(int k, const double *a, const double *b) {
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    const double span = std::max(std::fabs(lo), std::fabs(hi));
    lo -= 1e-12 * span + 1e-300;
    hi += 1e-12 * span + 1e-300;
    for (int it = 0; it < 2000; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(k, a, b, mid) >= 1) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

static void inverse_iteration(int k, const double *a, const double *b, double lam,
                              double *x) {
    // LU of (T - lam I) with partial pivoting for a tridiagonal matrix.
    double norm = 0.0;
    for (int i = 0; i < k; ++i)
        norm = std::max(norm, std::fabs(a[i]) + (i > 0 ? std::fabs(b[i - 1]) : 0.0) +
                                  (i + 1 < k ? std::fabs(b[i]) : 0.0));
    const double tiny = std::max(norm, 1e-300) * 1e-15;
    std::vector<double> d(k), du(k), du2(k), dl(k);
    std::vector<int> piv(k);
    for (int i = 0; i < k; ++i) {
        d[i] = a[i] - lam;
        du[i] = i + 1 < k ? b[i] : 0.0;
        dl[i] = i + 1 < k ? b[i] : 0.0;
        du2[i] = 0.0;
    }
    for (int i = 0; i + 1 < k; ++i) {
        if (std::fabs(d[i]) >= std::fabs(dl[i])) {
            piv[i] = 0;
            if (d[i] == 0.0) d[i] = tiny;
            const double f = dl[i] / d[i];
            dl[i] = f;
            d[i + 1] -= f * du[i];
        } else {
            piv[i] = 1;
            const double f = d[i] / dl[i];
            d[i] = dl[i];
            dl[i] = f;
            const double t = du[i];
            du[i] = d[i + 1];
            d[i + 1] = t - f * d[i + 1];
            if (i + 2 < k) {
                du2[i] = du[i + 1];
                du[i + 1] = -f * du[i + 1];
            }
        }
    }
    for (int i = 0; i < k; ++i)
        if (std::fabs(d[i]) < tiny) d[i] = d[i] < 0 ? -tiny : tiny;
    for (int i = 0; i < k; ++i) x[i] = 1.0 / std::sqrt((double)k) * (1.0 + 0.01 * ((i * 7919) % 13));
    for (int rep = 0; rep < 3; ++rep) {
        // forward: apply L^{-1} with the recorded row swaps
        for (int i = 0; i + 1 < k; ++i) {
            if (piv[i] == 0) {
                x[i + 1] -= dl[i] * x[i];
            } else {
                const double t = x[i];
                x[i] = x[i + 1];
                x[i + 1] = t - dl[i] * x[i + 1];
            }
        }
        // backward: U x = y
        for (int i = k - 1; i >= 0; --i) {
            double s = x[i];
            if (i + 1 < k) s -= du[i] * x[i + 1];
            if (i + 2 < k) s -= du2[i] * x[i + 2];
            x[i] = s / d[i];
        }
        double nrm = 0.0;
        for (int i = 0; i < k; ++i) nrm += x[i] * x[i];
        nrm = std::sqrt(nrm);
        for (int i = 0; i < k; ++i) x[i] /= nrm;
    }
    int first = 0;
    while (first < k && std::fabs(x[first]) < 1e-300) ++first;
    if (first < k && x[first] < 0)
        for (int i = 0; i < k; ++i) x[i] = -x[i];
}

}  // namespace hm

using hm::fail;

extern "C" {

int hm_tridiag_lowest(int32_t k, const double *alpha, const double *beta, double *eval,
                      double *evec) {
    hm::clear_error();
    if (k < 1 || !alpha || !eval || (k > 1 && !beta)) return fail(HM_EINVAL, "bad arguments");
    for (int i = 0; i < k; ++i)
        if (!std::isfinite(alpha[i]) || (i + 1 < k && !std::isfinite(beta[i])))
            return fail(HM_EINVAL, "non-finite tridiagonal entry");
    const double lam = hm::lowest_eigenvalue(k, alpha, beta);
    *eval = lam;
    if (evec) {
        if (k == 1) evec[0] = 1.0;
        else hm::inverse_iteration(k, alpha, beta, lam, evec);
    }
    return HM_OK;
}

int hm_lanczos_workspace(hm_basis h, int32_t steps, const hm_lanczos_opts *o, size_t *bytes) {
    hm::clear_error();
    if (!h || !bytes) return fail(HM_EINVAL, "null argument");
    if (steps < 1) return fail(HM_EINVAL, "steps must be >= 1");
    HM_TRY(hm::check_opts(&h->impl, o));
    *bytes = hm::layout(&h->impl, steps, o->precision, o->full_reorth ? 1 : 0).total;
    return HM_OK;
}

int hm_lanczos(hm_basis h, const double *J, const double *d_v0, int32_t steps,
               const hm_lanczos_opts *o, void *d_work, size_t work_bytes, double *alpha,
               double *beta, double *E0, int32_t *steps_done, void *stream) {
    hm::clear_error();
    if (!alpha || !beta || !E0) return fail(HM_EINVAL, "null output");
    int done = 0;
    HM_TRY(hm::run_common(h, J, d_v0, steps, o, d_work, work_bytes, nullptr, nullptr, alpha,
                          beta, &done, stream));
    *steps_done = done;
    return hm_tridiag_lowest(done, alpha, beta, E0, nullptr);
}

int hm_lanczos_ritz(hm_basis h, const double *J, const double *d_v0, int32_t steps_done,
                    const double *c, const hm_lanczos_opts *o, void *d_work,
                    size_t work_bytes, double *d_psi, double *alpha_out, double *beta_out,
                    void *stream) {
    hm::clear_error();
    if (!c || !d_psi) return fail(HM_EINVAL, "null argument");
    int done = 0;
    HM_TRY(hm::run_common(h, J, d_v0, steps_done, o, d_work, work_bytes, c, d_psi, alpha_out,
                          beta_out, &done, stream));
    if (done != steps_done)
        return fail(HM_EINVAL, "recompute stopped after %d of %d steps", done, steps_done);
    return HM_OK;
}

int hm_set_timing(int32_t enable) {
    hm::g_timing = enable != 0;
    return HM_OK;
}

int hm_last_timing(double *hx_ms, int32_t *hx_launches, double *loop_ms) {
    if (hx_ms) *hx_ms = hm::g_hx_ms;
    if (hx_launches) *hx_launches = hm::g_hx_launches;
    if (loop_ms) *loop_ms = hm::g_loop_ms;
    return HM_OK;
}

}  // extern "C"
