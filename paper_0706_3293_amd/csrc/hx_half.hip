// Spin-1/2 block kernel for the row-gather H x (Sec. 4, Eq. (E-4-b)).
//
// For s = 1/2 a basis state is an N-bit word with A set bits (a_u = 1 on the
// set bits), and the order of Eq. (E-3-a) restricted to H(M) is the order of
// the words' values.  The encoding sum of Sec. 3.2 then reduces to
// sum_t C(c_t, t) over the set-bit positions c_1 < c_2 < ... (P[k][A_k][1] =
// D(k-1, A_k) = C(k-1, A_k)).  Split a word into its low K bits L and high
// N-K bits h: the index is Off(h) + rankL(L), where rankL is the position of L
// among the K-bit words with the same number of set bits, and Off(h) depends
// on h only.  So the rows with one high part h form a contiguous block of
// C(K, A - popcount(h)) rows, ordered like the low words.
//
// Work item = (a group of R high words with the same popcount, a chunk of 64
// low words of their class).  Lane r owns the low word L of rank r and the R
// rows (h_m, L), m = 0..R-1:
//   * bonds inside the low word: flip test and rankL(L') (LDS table) are done
//     once per lane and reused for the R rows; target Off(h_m) + rankL(L');
//   * bonds inside the high word: flip and target block are the same for the
//     whole wavefront and the low word is unchanged, so the 64 lanes gather 64
//     consecutive entries of x at Off(h_m') + r: coalesced;
//   * bonds with one site in each word: the high bit is wave-uniform, the low
//     bit decides per lane, target Off(h_m') + rankL(L').
// Target block offsets of the high and straddling bonds depend on h and the
// bond only; they are tabulated per (basis, couplings).
// y_i = shift x_i + sum over flippable bonds of (-J/2)(x_j - x_i), with
// shift = -sum_b J_b / 4 (s = 1/2: m_u m_v = +-1/4 and every allowed ladder
// term has matrix element -J/2).  A bond that cannot flip gathers x_i itself
// and so adds zero; this keeps eight gathers in flight without branches.
// Each row is written by one lane; workgroups are persistent, and the eight
// XCDs take turns on runs of consecutive items so that they sweep x together.
#include <algorithm>
#include <type_traits>
#include <vector>

#include "device_common.h"
#include "hm_internal.h"

namespace hm {

constexpr int kHalfMaxK = 14;
constexpr int kHalfMaxHighBits = 24;
constexpr int kGroup = 8;
constexpr uint32_t kNoHigh = 0xFFFFFFFFu;      // padding slot of a high-word group
constexpr size_t kMaxNeighbourBytes = (size_t)8 << 30;
constexpr int64_t kMaxHalfGrid = 1 << 20;   // workgroups (and FP64 partials) of one launch

// Persistent sweep over the items (grid a multiple of 8; workgroup b runs on
// XCD b % 8): the XCDs take turns on runs of kSweepRun consecutive items, so
// all eight work in the same region of x at any time and gathers that reach
// far share the Infinity Cache, while a run keeps neighbouring blocks within
// one XCD's L2.  Local index l of XCD x8 (its waves stride through l
// together) maps to item (l / run) * 8 run + x8 run + l % run.
constexpr uint32_t kSweepRun = 64;

__device__ __forceinline__ uint32_t sweep_item(uint32_t l, uint32_t x8) {
    return (l / kSweepRun) * (kXcds * kSweepRun) + x8 * kSweepRun + l % kSweepRun;
}

// Eight bonds of one group, structure-of-arrays so one group is fetched with
// a few wide scalar loads.
//   low group:        m1 = bits u, v of the low word
//   high group:       m1 = bits u-K, v-K of the high word
//   straddling group: m1 = bit u of the low word, m2 = bit v-K of the high word
// Padding entries have m1 = m2 = 0 and coefficient 0; they never flip.
struct BondGroup {
    uint32_t m1[kGroup];
    uint32_t m2[kGroup];
    float c32[kGroup];      // -J/2 rounded to FP32
    uint32_t pad[kGroup];
    double c64[kGroup];     // -J/2
};

// Per-basis tables of the block kernel.
struct HalfTables {
    int K = 0, block = 256, R = 1, C = 0;   // C > 0: staged blocks of 64 C entries
    int ipw = 0;                            // items per wave that size the grid (0: default)
    int64_t n_items = 0, n_groups = 0;
    std::vector<uint64_t> off_host;
    uint16_t *d_rankL = nullptr, *d_unrankL = nullptr;
    void *d_off = nullptr;            // uint32 or uint64 per high word
    uint32_t *d_hgroups = nullptr;    // n_groups x R high words
    uint32_t *d_items = nullptr;      // (group << 8) | chunk
    int class_start[kHalfMaxK + 2] = {0};
    int class_size[kHalfMaxK + 2] = {0};
};

static void free_half(void *p) {
    auto *t = (HalfTables *)p;
    if (!t) return;
    if (t->d_rankL) (void)hipFree(t->d_rankL);
    if (t->d_unrankL) (void)hipFree(t->d_unrankL);
    if (t->d_off) (void)hipFree(t->d_off);
    if (t->d_hgroups) (void)hipFree(t->d_hgroups);
    if (t->d_items) (void)hipFree(t->d_items);
    delete t;
}

// Bonds of one coupling list regrouped for a given K, plus the neighbour
// table: for every high word h a row of (nHg + nSg) * 8 block offsets.  Its
// high-word part is compacted: first the target blocks of the high-word bonds
// that flip for h, in bond order (hcnt[h] of them, their bond slots in hidx),
// then the own block up to the next multiple of 8, paired with a bond of
// coefficient 0; a bond that cannot flip would only add c (x_i - x_i) = 0,
// so the compacted rows give the same sums with fewer loads.  The straddling
// part holds Off(h ^ m2) per bond in group order.  (Cached in the Couplings
// object of the basis.)
struct HalfBonds {
    int K = -1, nLg = 0, nHg = 0, nSg = 0;
    int nL = 0, nS = 0;           // low-word and straddling bonds (slots in use)
    BondGroup *groups = nullptr;
    void *nbr = nullptr;
    uint32_t *hcnt = nullptr;     // flipping high-word bonds per high word
    uint16_t *hidx = nullptr;     // their bond slots, nHg * 8 per high word
};

template <typename I>
struct HalfArgs {
    const uint16_t *rankL, *unrankL;
    const I *off;
    const I *nbr;
    const uint32_t *hcnt;
    const uint16_t *hidx;
    const uint32_t *hgroups;
    const uint32_t *items;
    const BondGroup *groups;
    uint32_t n_items;
    int K, A, nLg, nHg, nSg, width;
    int nL, nS;
    double shift;
    int class_start[kHalfMaxK + 2];
    int class_size[kHalfMaxK + 2];
};

// Element at a byte offset from a wave-uniform base pointer.
template <typename T>
__device__ __forceinline__ T load_at(const T *__restrict__ base, uint32_t byte_off) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}

// Visits slots [0, n) of a run of 8-slot groups (n wave-uniform) in pieces
// of at most MaxW (8 or 4) slots: pieces of MaxW, then at most one piece of
// 4 and pieces of 2, each inside one group; f(std::integral_constant<int, W>,
// first slot).  The slots after n up to the next even number are padding (a
// bond that never flips, or the own block with coefficient 0), so every
// piece gives the sums of the slots in use, in slot order, with at most one
// padding slot instead of up to seven.  Narrower pieces keep fewer loads in
// flight per wave but need fewer registers, so more waves fit.
template <int MaxW, typename F>
__device__ __forceinline__ void for_pieces(int n, F &&f) {
    static_assert(MaxW == kGroup || MaxW == 4, "pieces of 8 or 4 slots");
    int k = 0;
    for (; k + MaxW <= n; k += MaxW) f(std::integral_constant<int, MaxW>{}, k);
    if (MaxW == kGroup && n - k >= 4) {
        f(std::integral_constant<int, 4>{}, k);
        k += 4;
    }
    for (; k < n; k += 2) f(std::integral_constant<int, 2>{}, k);
}

template <typename T> __device__ __forceinline__ T coef(const BondGroup &g, int q);
template <> __device__ __forceinline__ float coef<float>(const BondGroup &g, int q) {
    return g.c32[q];
}
template <> __device__ __forceinline__ double coef<double>(const BondGroup &g, int q) {
    return g.c64[q];
}

template <typename T, typename I, int R, bool DOT, bool STORE>
__global__ __launch_bounds__(256) void hx_half_kernel(
    const HalfArgs<I> g, const T *__restrict__ x, T *__restrict__ y, const T *__restrict__ prev,
    const double *__restrict__ sigma_p, const double *__restrict__ cprev_p,
    double *__restrict__ partial, T *__restrict__ store, const int *__restrict__ stopped) {
    if (stopped && *stopped) return;
    extern __shared__ __align__(16) uint16_t lds16[];
    __shared__ double red[16];
    const int nlow = 1 << g.K;
    uint16_t *rankL = lds16;
    uint16_t *unrankL = lds16 + nlow;
    for (int t = threadIdx.x; t < nlow; t += blockDim.x) {
        rankL[t] = g.rankL[t];
        unrankL[t] = g.unrankL[t];
    }
    __syncthreads();

    const double sigma = sigma_p ? *sigma_p : 1.0;
    const double cprev = cprev_p ? *cprev_p : 0.0;
    const T shift = (T)g.shift;
    const int lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;
    uint32_t stride = gridDim.x * nw, wl, x8 = 0;
    const bool by_xcd = gridDim.x % kXcds == 0;
    if (by_xcd) {
        x8 = blockIdx.x % kXcds;
        stride = (gridDim.x / kXcds) * nw;
        wl = (blockIdx.x / kXcds) * nw + (threadIdx.x >> 6);
    } else {
        wl = blockIdx.x * nw + (threadIdx.x >> 6);
    }
    wl = __builtin_amdgcn_readfirstlane(wl);
    x8 = __builtin_amdgcn_readfirstlane(x8);
    stride = __builtin_amdgcn_readfirstlane(stride);
    const BondGroup *__restrict__ gl = g.groups;
    const BondGroup *__restrict__ gh = g.groups + g.nLg;
    const BondGroup *__restrict__ gs = g.groups + g.nLg + g.nHg;
    // widest slot piece: 4 in FP32 (fewer registers, more waves: N=32 R=4
    // pass 15.2 -> 14.6 ms, N=36 H x 267 -> 260 ms), 8 in FP64 (R=1 28.7 ms
    // with pieces of 8, 31.9 ms with pieces of 4)
    constexpr int kW = sizeof(T) == 4 ? 4 : kGroup;
    double dot = 0.0;
    for (uint32_t l = wl;; l += stride) {
        const uint32_t it = by_xcd ? sweep_item(l, x8) : l;
        if (it >= g.n_items) break;
        const uint32_t item = g.items[it];
        const uint32_t *__restrict__ hg = g.hgroups + (size_t)(item >> 8) * R;
        uint32_t hs[R];
        bool valid[R];
#pragma unroll
        for (int m = 0; m < R; ++m) hs[m] = hg[m];
#pragma unroll
        for (int m = 0; m < R; ++m) {
            valid[m] = hs[m] != kNoHigh;
            if (!valid[m]) hs[m] = hs[0];          // padding slots shadow slot 0
        }
        const int aL = g.A - __popc(hs[0]);
        const int S = g.class_size[aL];
        const int r0 = (int)(item & 255u) * 64 + lane;
        const bool live = r0 < S;
        const int r = live ? r0 : 0;              // dead lanes shadow row 0 of the block
        const uint32_t L = unrankL[g.class_start[aL] + r];
        I off[R];
        const I *__restrict__ nb[R];
        T xi[R], acc[R];
        // offsets inside a block are byte offsets from a wave-uniform block
        // base, so loads take the scalar-base + 32-bit-offset address form
        const uint32_t r_bytes = (uint32_t)r * (uint32_t)sizeof(T);
#pragma unroll
        for (int m = 0; m < R; ++m) {
            off[m] = g.off[hs[m]];
            nb[m] = g.nbr + (size_t)hs[m] * g.width;
            xi[m] = load_at(x + off[m], r_bytes);
            acc[m] = 0;
        }
        // bonds inside the low word: the test and rankL(L ^ m) once per lane
        for_pieces<kW>(g.nL, [&](auto Wc, int k) {
            constexpr int W = decltype(Wc)::value;
            const BondGroup &G = gl[k / kGroup];
            const int q0 = W == kGroup ? 0 : k % kGroup;
            uint32_t mk[W], idx[W];
#pragma unroll
            for (int q = 0; q < W; ++q) mk[q] = G.m1[q0 + q];
#pragma unroll
            for (int q = 0; q < W; ++q) idx[q] = rankL[L ^ mk[q]];
#pragma unroll
            for (int q = 0; q < W; ++q)
                idx[q] = __popc(L & mk[q]) == 1 ? idx[q] * (uint32_t)sizeof(T) : r_bytes;
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const T *__restrict__ xb = x + off[m];
                T xj[W];
#pragma unroll
                for (int q = 0; q < W; ++q) xj[q] = load_at(xb, idx[q]);
#pragma unroll
                for (int q = 0; q < W; ++q) acc[m] += coef<T>(G, q0 + q) * (xj[q] - xi[m]);
            }
        });
        // bonds inside the high word that flip for h_m (compacted rows of the
        // table): target block, same low word, coalesced gathers.  Up to 4
        // rows per lane go through their rows of the table together, up to
        // the longest (shorter rows continue with their own block and
        // coefficient 0), so that R groups of loads are in flight at once;
        // with 8 rows per lane that costs too many registers, and the rows
        // go one after another.  The sums are the same either way.
        if constexpr (R <= 4) {
            const uint16_t *__restrict__ bi[R];
            int nmax = 0;
#pragma unroll
            for (int m = 0; m < R; ++m) {
                nmax = max(nmax, (int)g.hcnt[hs[m]]);
                bi[m] = g.hidx + (size_t)hs[m] * (g.nHg * kGroup);
            }
            for_pieces<kW>(nmax, [&](auto Wc, int k) {
                constexpr int W = decltype(Wc)::value;
                T xj[R][W];
#pragma unroll
                for (int m = 0; m < R; ++m)
#pragma unroll
                    for (int q = 0; q < W; ++q) xj[m][q] = load_at(x + nb[m][k + q], r_bytes);
#pragma unroll
                for (int m = 0; m < R; ++m)
#pragma unroll
                    for (int q = 0; q < W; ++q) {
                        const uint32_t b = bi[m][k + q];
                        acc[m] += coef<T>(gh[b >> 3], b & 7) * (xj[m][q] - xi[m]);
                    }
            });
        } else {
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const int nf = (int)g.hcnt[hs[m]];
                const uint16_t *__restrict__ bi = g.hidx + (size_t)hs[m] * (g.nHg * kGroup);
                for_pieces<kW>(nf, [&](auto Wc, int k) {
                    constexpr int W = decltype(Wc)::value;
                    T xj[W];
#pragma unroll
                    for (int q = 0; q < W; ++q) xj[q] = load_at(x + nb[m][k + q], r_bytes);
#pragma unroll
                    for (int q = 0; q < W; ++q) {
                        const uint32_t b = bi[k + q];
                        acc[m] += coef<T>(gh[b >> 3], b & 7) * (xj[q] - xi[m]);
                    }
                });
            }
        }
        // bonds with one site in each word: uniform high bit, per-lane low bit
        for_pieces<kW>(g.nS, [&](auto Wc, int k) {
            constexpr int W = decltype(Wc)::value;
            const BondGroup &G = gs[k / kGroup];
            const int q0 = W == kGroup ? 0 : k % kGroup;
            uint32_t ml[W], lb[W], rk[W];
#pragma unroll
            for (int q = 0; q < W; ++q) ml[q] = G.m1[q0 + q];
#pragma unroll
            for (int q = 0; q < W; ++q) {
                rk[q] = rankL[L ^ ml[q]];
                lb[q] = L & ml[q];
            }
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const I *__restrict__ nbs = nb[m] + g.nHg * kGroup + k;
                const I own = off[m] + (I)r;
                T xj[W];
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    // the low-bit value that differs from the high bit;
                    // padding entries (ml = 0) get an impossible value
                    const uint32_t want =
                        ml[q] == 0 ? 1u : ((hs[m] & G.m2[q0 + q]) ? 0u : ml[q]);
                    xj[q] = x[lb[q] == want ? nbs[q] + (I)rk[q] : own];
                }
#pragma unroll
                for (int q = 0; q < W; ++q) acc[m] += coef<T>(G, q0 + q) * (xj[q] - xi[m]);
            }
        });
#pragma unroll
        for (int m = 0; m < R; ++m) {
            if (live && valid[m]) {
                const I row = off[m] + (I)r;
                const T hv = shift * xi[m] + acc[m];
                double w = sigma * (double)hv;
                if (prev) w -= cprev * (double)prev[row];
                const T wt = (T)w;
                y[row] = wt;
                if constexpr (DOT) dot += (double)wt * (sigma * (double)xi[m]);
                if constexpr (STORE) store[row] = (T)(sigma * (double)xi[m]);
            }
        }
    }
    if constexpr (DOT) {
        const double s = block_sum(dot, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// Read-only tables seen through the constant address space.
template <typename T>
using Const = const __attribute__((address_space(4))) T;
template <typename T>
__device__ __forceinline__ const Const<T> *as_const(const T *p) {
    return (const Const<T> *)p;
}
template <typename T> __device__ __forceinline__ T coefc(const Const<BondGroup> &g, int q);
template <> __device__ __forceinline__ float coefc<float>(const Const<BondGroup> &g, int q) {
    return g.c32[q];
}
template <> __device__ __forceinline__ double coefc<double>(const Const<BondGroup> &g, int q) {
    return g.c64[q];
}

// Staged variant.  Work item = one group of R high words of one popcount
// class with ALL rows of their blocks: the block size S = C(K, aL) is at most
// 64 C, and lane r owns the low words of ranks r, r + 64, ..., r + 64 (C - 1).
// The wave first copies the R blocks of x into its private LDS slice (the
// loads it needs anyway for x_i), so the gathers of the bonds inside the low
// word, which scatter over the block, read LDS instead of going through the
// vector memory pipeline; high-word and straddling bonds gather from global
// memory as in hx_half_kernel (coalesced for high-word bonds).  Same
// arithmetic per row as hx_half_kernel: acc accumulates the
// bonds in the same order, so both kernels give bitwise equal results.
// Shared state of one wave of the staged kernel.
template <typename T, typename I>
struct StagedWave {
    const uint16_t *rankL, *unrankL;
    T *xs;                              // this wave's LDS slice
    const Const<BondGroup> *gl, *gh, *gs;
    const Const<I> *nbr;
    const Const<uint32_t> *hcnt;
    const Const<uint16_t> *hidx;
    const T *x;
    T *y;
    const T *prev;
    T *store;
    double sigma, cprev;
    T shift;
    int lane;
};

// One item (R blocks of class size S) with J live 64-row slices per block
// (J = ceil(S / 64) rounded up to a power of two, J <= C).
template <typename T, typename I, int R, int C, int J, bool DOT, bool STORE>
__device__ __forceinline__ void staged_item(const HalfArgs<I> &g, const StagedWave<T, I> &w,
                                            const uint32_t (&hs)[R], const bool (&valid)[R],
                                            const I (&off)[R], int S, int cs, double &dot) {
    constexpr int kSlice = 64 * C;
    uint32_t L[J], rb[J];
    bool live[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int r0 = w.lane + 64 * j;
        live[j] = r0 < S;
        const int r = live[j] ? r0 : 0;            // dead lanes shadow row 0
        rb[j] = (uint32_t)r;
        L[j] = w.unrankL[cs + r];
    }
    const Const<I> *nb[R];
    T xi[R][J], acc[R][J];
#pragma unroll
    for (int m = 0; m < R; ++m) {
        nb[m] = w.nbr + (size_t)hs[m] * g.width;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            xi[m][j] = load_at(w.x + off[m], rb[j] * (uint32_t)sizeof(T));
            acc[m][j] = 0;
        }
    }
    // stage this item's blocks.  The slice is private to the wave and a
    // wave's LDS accesses complete in program order, so the previous item's
    // reads are done and the writes below are seen by the reads after them;
    // the wave barrier keeps the compiler from moving LDS accesses across.
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int m = 0; m < R; ++m)
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (live[j]) w.xs[m * kSlice + rb[j]] = xi[m][j];
    __builtin_amdgcn_wave_barrier();
    // Widest piece of each slot list.  Pieces of 8 keep more loads in flight
    // per wave, pieces of 4 need fewer registers, so more waves fit; measured
    // on the N=32 pass A of a Lanczos step (FP32 89 VGPRs, 5 waves per SIMD,
    // 9.75 ms against 10.39 ms with pieces of 8 at 117 VGPRs; FP64 96 VGPRs,
    // 17.09 against 17.83 ms).
    constexpr int kLowW = sizeof(T) == 4 ? 4 : kGroup, kHighW = 4, kStrW = 4;
    // bonds inside the low word: LDS gathers
    for_pieces<kLowW>(g.nL, [&](auto Wc, int k) {
        constexpr int W = decltype(Wc)::value;
        const Const<BondGroup> &G = w.gl[k / kGroup];
        const int q0 = W == kGroup ? 0 : k % kGroup;
        uint32_t mk[W];
#pragma unroll
        for (int q = 0; q < W; ++q) mk[q] = G.m1[q0 + q];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            uint32_t idx[W];
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const uint32_t t2 = w.rankL[L[j] ^ mk[q]];
                idx[q] = __popc(L[j] & mk[q]) == 1 ? t2 : rb[j];
            }
#pragma unroll
            for (int m = 0; m < R; ++m) {
                T xj[W];
#pragma unroll
                for (int q = 0; q < W; ++q) xj[q] = w.xs[m * kSlice + idx[q]];
#pragma unroll
                for (int q = 0; q < W; ++q)
                    acc[m][j] += coefc<T>(G, q0 + q) * (xj[q] - xi[m][j]);
            }
        }
    });
    // bonds inside the high word that flip for h_m (compacted rows of the
    // table): coalesced global gathers
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int nf = (int)w.hcnt[hs[m]];
        const Const<uint16_t> *bi = w.hidx + (size_t)hs[m] * (g.nHg * kGroup);
        for_pieces<kHighW>(nf, [&](auto Wc, int k) {
            constexpr int W = decltype(Wc)::value;
            I o[W];
            T c[W];
#pragma unroll
            for (int q = 0; q < W; ++q) {
                o[q] = nb[m][k + q];
                const uint32_t b = bi[k + q];
                c[q] = coefc<T>(w.gh[b >> 3], b & 7);
            }
#pragma unroll
            for (int j = 0; j < J; ++j) {
                T xj[W];
#pragma unroll
                for (int q = 0; q < W; ++q)
                    xj[q] = load_at(w.x + o[q], rb[j] * (uint32_t)sizeof(T));
#pragma unroll
                for (int q = 0; q < W; ++q) acc[m][j] += c[q] * (xj[q] - xi[m][j]);
            }
        });
    }
    // bonds with one site in each word: uniform high bit, per-lane low bit
    auto straddle = [&](auto Wc, int k) {
        constexpr int W = decltype(Wc)::value;
        const Const<BondGroup> &G = w.gs[k / kGroup];
        const int q0 = W == kGroup ? 0 : k % kGroup;
        uint32_t ml[W];
#pragma unroll
        for (int q = 0; q < W; ++q) ml[q] = G.m1[q0 + q];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            uint32_t rk[W], lb[W];
#pragma unroll
            for (int q = 0; q < W; ++q) {
                rk[q] = w.rankL[L[j] ^ ml[q]];
                lb[q] = L[j] & ml[q];
            }
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const Const<I> *nbs = nb[m] + g.nHg * kGroup + k;
                const I own = off[m] + (I)rb[j];
                T xj[W];
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const uint32_t want =
                        ml[q] == 0 ? 1u : ((hs[m] & G.m2[q0 + q]) ? 0u : ml[q]);
                    xj[q] = w.x[lb[q] == want ? nbs[q] + (I)rk[q] : own];
                }
#pragma unroll
                for (int q = 0; q < W; ++q)
                    acc[m][j] += coefc<T>(G, q0 + q) * (xj[q] - xi[m][j]);
            }
        }
    };
    for_pieces<kStrW>(g.nS, straddle);
#pragma unroll
    for (int m = 0; m < R; ++m) {
#pragma unroll
        for (int j = 0; j < J; ++j) {
            if (live[j] && valid[m]) {
                const I row = off[m] + (I)rb[j];
                const T hv = w.shift * xi[m][j] + acc[m][j];
                double v = w.sigma * (double)hv;
                if (w.prev) v -= w.cprev * (double)w.prev[row];
                const T vt = (T)v;
                w.y[row] = vt;
                if constexpr (DOT) dot += (double)vt * (w.sigma * (double)xi[m][j]);
                if constexpr (STORE) w.store[row] = (T)(w.sigma * (double)xi[m][j]);
            }
        }
    }
}

template <typename T, typename I, int R, int C, bool DOT, bool STORE>
__global__ __launch_bounds__(256) void hx_half_staged_kernel(
    const HalfArgs<I> g, const T *__restrict__ x, T *__restrict__ y, const T *__restrict__ prev,
    const double *__restrict__ sigma_p, const double *__restrict__ cprev_p,
    double *__restrict__ partial, T *__restrict__ store, const int *__restrict__ stopped) {
    if (stopped && *stopped) return;
    extern __shared__ __align__(16) uint16_t lds16[];
    __shared__ double red[16];
    const int nlow = 1 << g.K;
    uint16_t *rankL = lds16;
    uint16_t *unrankL = lds16 + nlow;
    for (int t = threadIdx.x; t < nlow; t += blockDim.x) {
        rankL[t] = g.rankL[t];
        unrankL[t] = g.unrankL[t];
    }
    __syncthreads();

    StagedWave<T, I> w;
    w.rankL = rankL;
    w.unrankL = unrankL;
    w.xs = reinterpret_cast<T *>(lds16 + 2 * nlow) + (size_t)(threadIdx.x >> 6) * (R * 64 * C);
    // the tables are read-only for the whole launch: reading them through
    // the constant address space lets wave-uniform reads be scalar loads even
    // though the wave writes LDS in between
    w.gl = as_const(g.groups);
    w.gh = w.gl + g.nLg;
    w.gs = w.gl + g.nLg + g.nHg;
    w.nbr = as_const(g.nbr);
    w.hcnt = as_const(g.hcnt);
    w.hidx = as_const(g.hidx);
    w.x = x;
    w.y = y;
    w.prev = prev;
    w.store = store;
    w.sigma = sigma_p ? *sigma_p : 1.0;
    w.cprev = cprev_p ? *cprev_p : 0.0;
    w.shift = (T)g.shift;
    w.lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;
    uint32_t stride = gridDim.x * nw, wl, x8 = 0;
    const bool by_xcd = gridDim.x % kXcds == 0;
    if (by_xcd) {
        x8 = blockIdx.x % kXcds;
        stride = (gridDim.x / kXcds) * nw;
        wl = (blockIdx.x / kXcds) * nw + (threadIdx.x >> 6);
    } else {
        wl = blockIdx.x * nw + (threadIdx.x >> 6);
    }
    wl = __builtin_amdgcn_readfirstlane(wl);
    x8 = __builtin_amdgcn_readfirstlane(x8);
    stride = __builtin_amdgcn_readfirstlane(stride);
    const Const<uint32_t> *hgroups = as_const(g.hgroups);
    const Const<I> *offs = as_const(g.off);
    double dot = 0.0;
    for (uint32_t l = wl;; l += stride) {
        const uint32_t it = by_xcd ? sweep_item(l, x8) : l;
        if (it >= g.n_items) break;
        const Const<uint32_t> *hg = hgroups + (size_t)it * R;
        uint32_t hs[R];
        bool valid[R];
        I off[R];
#pragma unroll
        for (int m = 0; m < R; ++m) hs[m] = hg[m];
#pragma unroll
        for (int m = 0; m < R; ++m) {
            valid[m] = hs[m] != kNoHigh;
            if (!valid[m]) hs[m] = hs[0];
            off[m] = offs[hs[m]];
        }
        const int aL = g.A - __popc(hs[0]);
        const int S = g.class_size[aL];
        const int cs = g.class_start[aL];
        // live 64-row slices, rounded up to a power of two (wave-uniform)
        const int nj = (S + 63) >> 6;
        if (C >= 8 && nj > 4)
            staged_item<T, I, R, C, (C >= 8 ? 8 : 1), DOT, STORE>(g, w, hs, valid, off, S, cs, dot);
        else if (C >= 4 && nj > 2)
            staged_item<T, I, R, C, (C >= 4 ? 4 : 1), DOT, STORE>(g, w, hs, valid, off, S, cs, dot);
        else if (C >= 2 && nj > 1)
            staged_item<T, I, R, C, 2, DOT, STORE>(g, w, hs, valid, off, S, cs, dot);
        else
            staged_item<T, I, R, C, 1, DOT, STORE>(g, w, hs, valid, off, S, cs, dot);
    }
    if constexpr (DOT) {
        const double s = block_sum(dot, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
// Defaults measured on MI355X (one FP32 H x of J1-J2 rings): K = 13 beats 14
// at N = 32 (14.5 vs 19.4 ms) and N = 36 (283 vs 365 ms).
static int default_low_bits(int N) {
    int K = N <= 30 ? std::min(N, 12) : (N <= 36 ? 13 : 14);
    if (N - K > kHalfMaxHighBits) K = N - kHalfMaxHighBits;
    return K;
}

static int low_bits_of(const Basis *b) { return b->half_K > 0 ? b->half_K : default_low_bits(b->N); }
static int block_of(const Basis *b) { return b->half_block > 0 ? b->half_block : 256; }
static int rows_of(const Basis *b) {
    if (b->half_R > 0) return b->half_R;
    return b->dim >= ((int64_t)1 << 22) ? 4 : 1;
}

bool half_supported(const Basis *b) {
    if (b->two_s != 1) return false;
    const int K = low_bits_of(b);
    return K <= kHalfMaxK && K <= b->N && b->N - K <= kHalfMaxHighBits;
}

static int64_t binom(int n, int k) {
    if (k < 0 || k > n) return 0;
    int64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// Number of (high-word group, 64-row chunk) items, from the block sizes.
static int64_t item_count(const Basis *b) {
    const int K = low_bits_of(b), nh = b->N - K, R = rows_of(b);
    int64_t n = 0;
    for (int ph = 0; ph <= nh; ++ph) {
        const int aL = b->A - ph;
        if (aL < 0 || aL > K) continue;
        n += ((binom(nh, ph) + R - 1) / R) * ((binom(K, aL) + 63) / 64);
    }
    return n;
}

// Staged blocks: entries per lane (C) for a block of up to C(K, K/2) rows,
// 0 if the largest block does not fit 8 per lane.
static int staged_entries(int K) {
    const int64_t smax = binom(K, K / 2);
    return smax <= 128 ? 2 : (smax <= 256 ? 4 : (smax <= 512 ? 8 : 0));
}

static bool staged_possible(const Basis *b) {
    const int C = staged_entries(low_bits_of(b)), R = rows_of(b);
    return C > 0 && b->idx32 && R <= (C == 8 ? 2 : 4);
}

// Whether the staged work split runs (a function of the basis and its
// schedule only, so workspace sizes can be computed before the tables).
static bool staged_of(const Basis *b) {
    if (b->half_staging == 1) return false;
    if (b->half_staging == 2) return true;
    return false;
}

// Number of high-word groups (work items of the staged split).
static int64_t group_count(const Basis *b) {
    const int K = low_bits_of(b), nh = b->N - K, R = rows_of(b);
    int64_t n = 0;
    for (int ph = 0; ph <= nh; ++ph) {
        const int aL = b->A - ph;
        if (aL < 0 || aL > K) continue;
        n += (binom(nh, ph) + R - 1) / R;
    }
    return n;
}

// Workgroups for n_items work items: by default one item per wave up to
// kMaxGrid workgroups (then the persistent waves take several each); with
// ipw > 0 about ipw items per wave, up to kMaxHalfGrid workgroups.  A grid
// larger than the resident workgroups leaves the balancing of unequal items
// (blocks of 1 to 252 rows in the staged split) to the hardware dispatcher.
static int grid_for_items(int64_t n_items, int block, int ipw) {
    const int nw = block / 64;
    int64_t g;
    if (ipw > 0) {
        g = (n_items + (int64_t)nw * ipw - 1) / ((int64_t)nw * ipw);
        g = std::min<int64_t>(g, kMaxHalfGrid);
    } else {
        g = (n_items + nw - 1) / nw;
        g = std::min<int64_t>(g, kMaxGrid);
    }
    g = std::max<int64_t>(g, 1);
    if (g >= kXcds) g -= g % kXcds;
    return (int)g;
}

// Workgroups of the block kernel (= FP64 partial sums it writes).
int hx_half_grid(const Basis *b) {
    return grid_for_items(staged_of(b) ? group_count(b) : item_count(b), block_of(b), b->half_ipw);
}

static hipError_t upload(void **dst, const void *src, size_t bytes) {
    hipError_t e = hipMalloc(dst, bytes);
    if (e == hipSuccess) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    return e;
}

static int half_prepare(Basis *b, HalfTables **out) {
    std::lock_guard<std::mutex> lock(b->mu);
    HM_TRY(device_prepare(b));
    if (b->half_tables) {
        *out = (HalfTables *)b->half_tables;
        return HM_OK;
    }
    const int N = b->N, A = b->A;
    const int K = low_bits_of(b), R = rows_of(b);
    if (K > kHalfMaxK || N - K > kHalfMaxHighBits || K < 1 || K > N)
        return fail(HM_EINVAL, "block kernel: low bits K=%d unsupported for N=%d", K, N);
    if (staged_of(b) && !staged_possible(b))
        return fail(HM_EINVAL,
                    "staged block kernel needs C(K, K/2) <= 512, 32-bit indices and at most "
                    "4 rows per lane (2 when K = 11); K=%d, R=%d", K, R);
    auto *t = new HalfTables;
    t->K = K;
    t->R = R;
    t->block = block_of(b);
    t->C = staged_of(b) ? staged_entries(K) : 0;
    t->ipw = b->half_ipw;
    const int nlow = 1 << K;
    std::vector<uint16_t> rankL(nlow), unrankL(nlow);
    std::vector<int> fill(K + 1, 0);
    for (int a = 0, s = 0; a <= K; ++a) {
        t->class_start[a] = s;
        t->class_size[a] = (int)binom(K, a);
        s += t->class_size[a];
    }
    for (int L = 0; L < nlow; ++L) {   // ascending values: colex order per class
        const int a = __builtin_popcount((unsigned)L);
        rankL[L] = (uint16_t)fill[a];
        unrankL[t->class_start[a] + fill[a]] = (uint16_t)L;
        ++fill[a];
    }
    const int nh = N - K;
    const int64_t nhigh = (int64_t)1 << nh;
    t->off_host.assign(nhigh, 0);
    std::vector<std::vector<uint32_t>> by_class(nh + 1);
    int64_t expect = 0;
    for (int64_t h = 0; h < nhigh; ++h) {
        const int ph = __builtin_popcountll((unsigned long long)h);
        const int aL = A - ph;
        if (aL < 0 || aL > K) continue;
        uint64_t o = 0;
        int t_idx = aL;
        for (int q = 0; q < nh; ++q)
            if ((h >> q) & 1) o += (uint64_t)binom(K + q, ++t_idx);
        if ((int64_t)o != expect) {
            free_half(t);
            return fail(HM_EINVAL, "internal: block offsets out of order at h=%lld", (long long)h);
        }
        t->off_host[h] = o;
        expect += t->class_size[aL];
        by_class[ph].push_back((uint32_t)h);
    }
    if (expect != b->dim) {
        free_half(t);
        return fail(HM_EINVAL, "internal: block sizes sum to %lld, dim %lld", (long long)expect,
                    (long long)b->dim);
    }
    // groups of R high words of one popcount class, ordered by the offset of
    // their first block so the sweep follows memory order
    struct Grp { uint64_t key; int ph; size_t start; };
    std::vector<Grp> grps;
    for (int ph = 0; ph <= nh; ++ph)
        for (size_t s = 0; s < by_class[ph].size(); s += R)
            grps.push_back({t->off_host[by_class[ph][s]], ph, s});
    std::sort(grps.begin(), grps.end(), [](const Grp &a, const Grp &b) { return a.key < b.key; });
    std::vector<uint32_t> hgroups, items;
    hgroups.reserve(grps.size() * R);
    for (size_t gi = 0; gi < grps.size(); ++gi) {
        const auto &cls = by_class[grps[gi].ph];
        for (int m = 0; m < R; ++m) {
            const size_t s = grps[gi].start + m;
            hgroups.push_back(s < cls.size() ? cls[s] : kNoHigh);
        }
        const int S = t->class_size[A - grps[gi].ph];
        for (int c = 0; c * 64 < S; ++c) items.push_back(((uint32_t)gi << 8) | (uint32_t)c);
    }
    if ((int64_t)items.size() != item_count(b) || grps.size() >= ((size_t)1 << 24)) {
        free_half(t);
        return fail(HM_EINVAL, "internal: %zu items, expected %lld", items.size(),
                    (long long)item_count(b));
    }
    t->n_items = (int64_t)items.size();
    t->n_groups = (int64_t)grps.size();
    hipError_t e = upload((void **)&t->d_rankL, rankL.data(), nlow * sizeof(uint16_t));
    if (e == hipSuccess) e = upload((void **)&t->d_unrankL, unrankL.data(), nlow * sizeof(uint16_t));
    if (e == hipSuccess) {
        if (b->idx32) {
            std::vector<uint32_t> o32(t->off_host.begin(), t->off_host.end());
            e = upload(&t->d_off, o32.data(), o32.size() * sizeof(uint32_t));
        } else {
            e = upload(&t->d_off, t->off_host.data(), t->off_host.size() * sizeof(uint64_t));
        }
    }
    if (e == hipSuccess)
        e = upload((void **)&t->d_hgroups, hgroups.data(), hgroups.size() * sizeof(uint32_t));
    if (e == hipSuccess) e = upload((void **)&t->d_items, items.data(), items.size() * sizeof(uint32_t));
    if (e != hipSuccess) {
        free_half(t);
        return fail(HM_EDEVICE, "block kernel tables: %s", hipGetErrorString(e));
    }
    b->half_tables = t;
    b->half_tables_free = free_half;
    *out = t;
    return HM_OK;
}

static void free_half_bonds(void *p) {
    auto *hb = (HalfBonds *)p;
    if (!hb) return;
    if (hb->groups) (void)hipFree(hb->groups);
    if (hb->nbr) (void)hipFree(hb->nbr);
    if (hb->hcnt) (void)hipFree(hb->hcnt);
    if (hb->hidx) (void)hipFree(hb->hidx);
    delete hb;
}

struct Flat {
    uint32_t m1 = 0, m2 = 0;
    double c = 0.0;
};

static void to_groups(const std::vector<Flat> &v, std::vector<BondGroup> &out) {
    for (size_t i = 0; i < v.size(); i += kGroup) {
        BondGroup G{};
        for (int q = 0; q < kGroup && i + q < v.size(); ++q) {
            G.m1[q] = v[i + q].m1;
            G.m2[q] = v[i + q].m2;
            G.c64[q] = v[i + q].c;
            G.c32[q] = (float)v[i + q].c;
        }
        out.push_back(G);
    }
}

static size_t neighbour_bytes(const Basis *b, const Couplings *c, int K) {
    int nH = 0, nS = 0;
    for (const BondDev &bd : c->host) {
        if (bd.u >= K) ++nH;
        else if (bd.v >= K) ++nS;
    }
    const size_t width = (size_t)((nH + kGroup - 1) / kGroup + (nS + kGroup - 1) / kGroup) * kGroup;
    const size_t hwidth = (size_t)((nH + kGroup - 1) / kGroup) * kGroup;
    return ((size_t)1 << (b->N - K)) *
           (width * (b->idx32 ? 4 : 8) + hwidth * sizeof(uint16_t) + sizeof(uint32_t));
}

static int half_bonds(Basis *b, const Couplings *c, const HalfTables *t,
                      const HalfBonds **out) {
    const int K = t->K;
    std::lock_guard<std::mutex> lock(b->mu);
    auto *cc = const_cast<Couplings *>(c);
    if (cc->half && ((HalfBonds *)cc->half)->K == K) {
        *out = (const HalfBonds *)cc->half;
        return HM_OK;
    }
    if (neighbour_bytes(b, c, K) > kMaxNeighbourBytes)
        return fail(HM_ERANGE, "block kernel neighbour table would exceed %zu bytes",
                    kMaxNeighbourBytes);
    std::vector<Flat> lo, hi, st;
    for (const BondDev &bd : c->host) {
        Flat f;
        f.c = bd.mJ2;
        if (bd.v < K) {
            f.m1 = (1u << bd.u) | (1u << bd.v);
            lo.push_back(f);
        } else if (bd.u >= K) {
            f.m1 = (1u << (bd.u - K)) | (1u << (bd.v - K));
            hi.push_back(f);
        } else {
            f.m1 = 1u << bd.u;
            f.m2 = 1u << (bd.v - K);
            st.push_back(f);
        }
    }
    std::vector<BondGroup> groups;
    to_groups(lo, groups);
    const int nLg = (int)groups.size();
    to_groups(hi, groups);
    const int nHg = (int)groups.size() - nLg;
    to_groups(st, groups);
    const int nSg = (int)groups.size() - nLg - nHg;
    groups.push_back(BondGroup{});    // all coefficients 0: the padding of compacted rows
    const int width = (nHg + nSg) * kGroup, hwidth = nHg * kGroup;
    const uint16_t zero_slot = (uint16_t)((nHg + nSg) * kGroup);   // relative to the high groups
    const int64_t nhigh = (int64_t)1 << (b->N - K);
    // neighbour table: compacted high-word part (target blocks of the bonds
    // that flip, then the own block), straddling part Off(h ^ m2)
    std::vector<uint64_t> nbr((size_t)nhigh * width, 0);
    std::vector<uint32_t> hcnt((size_t)nhigh, 0);
    std::vector<uint16_t> hidx((size_t)nhigh * hwidth, zero_slot);
    for (int64_t h = 0; h < nhigh; ++h) {
        const int aL = b->A - __builtin_popcountll((unsigned long long)h);
        if (aL < 0 || aL > K) continue;
        uint64_t *row = &nbr[(size_t)h * width];
        uint16_t *irow = &hidx[(size_t)h * hwidth];
        int n = 0;
        for (int k = 0; k < nHg; ++k)
            for (int q = 0; q < kGroup; ++q) {
                const uint32_t m = groups[nLg + k].m1[q];
                if (__builtin_popcountll((unsigned long long)(h & m)) == 1) {
                    row[n] = t->off_host[h ^ m];
                    irow[n] = (uint16_t)(k * kGroup + q);
                    ++n;
                }
            }
        hcnt[h] = (uint32_t)n;
        for (int s2 = n; s2 < hwidth; ++s2) row[s2] = t->off_host[h];
        for (int k = 0; k < nSg; ++k)
            for (int q = 0; q < kGroup; ++q)
                row[(nHg + k) * kGroup + q] = t->off_host[h ^ groups[nLg + nHg + k].m2[q]];
    }
    auto *hb = new HalfBonds;
    hb->K = K;
    hb->nLg = nLg;
    hb->nHg = nHg;
    hb->nSg = nSg;
    hb->nL = (int)lo.size();
    hb->nS = (int)st.size();
    hipError_t e = hipSuccess;
    if (!groups.empty()) e = upload((void **)&hb->groups, groups.data(), groups.size() * sizeof(BondGroup));
    if (e == hipSuccess && !nbr.empty()) {
        if (b->idx32) {
            std::vector<uint32_t> n32(nbr.begin(), nbr.end());
            e = upload(&hb->nbr, n32.data(), n32.size() * sizeof(uint32_t));
        } else {
            e = upload(&hb->nbr, nbr.data(), nbr.size() * sizeof(uint64_t));
        }
    }
    if (e == hipSuccess) e = upload((void **)&hb->hcnt, hcnt.data(), hcnt.size() * sizeof(uint32_t));
    if (e == hipSuccess && !hidx.empty())
        e = upload((void **)&hb->hidx, hidx.data(), hidx.size() * sizeof(uint16_t));
    if (e != hipSuccess) {
        free_half_bonds(hb);
        return fail(HM_EDEVICE, "block kernel bonds: %s", hipGetErrorString(e));
    }
    if (cc->half && cc->half_free) cc->half_free(cc->half);
    cc->half = hb;
    cc->half_free = free_half_bonds;
    *out = hb;
    return HM_OK;
}

template <typename T, typename I, int R>
static void launch_r(const HalfTables *t, const HalfArgs<I> &g, const HxPass &p, hipStream_t st) {
    const int grid = grid_for_items(t->n_items, t->block, t->ipw);
    const size_t lds = 2 * sizeof(uint16_t) * ((size_t)1 << t->K);
    const T *x = (const T *)p.x;
    T *y = (T *)p.y;
    const T *pr = (const T *)p.p;
    T *store = (T *)p.store;
#define HM_LAUNCH(D, S)                                                                     \
    hipLaunchKernelGGL((hx_half_kernel<T, I, R, D, S>), dim3(grid), dim3(t->block), lds, st, \
                       g, x, y, pr, p.sigma, p.cprev, p.partial, store, p.stopped)
    const bool dot = p.partial != nullptr, sto = store != nullptr;
    if (!dot && !sto) HM_LAUNCH(false, false);
    else if (dot && !sto) HM_LAUNCH(true, false);
    else if (!dot && sto) HM_LAUNCH(false, true);
    else HM_LAUNCH(true, true);
#undef HM_LAUNCH
}

template <typename T, int R, int C>
static void launch_staged(const HalfTables *t, const HalfArgs<uint32_t> &g, const HxPass &p,
                          hipStream_t st) {
    const int grid = grid_for_items(t->n_groups, t->block, t->ipw);
    const size_t lds = 2 * sizeof(uint16_t) * ((size_t)1 << t->K) +
                       (size_t)(t->block / 64) * R * 64 * C * sizeof(T);
    const T *x = (const T *)p.x;
    T *y = (T *)p.y;
    const T *pr = (const T *)p.p;
    T *store = (T *)p.store;
#define HM_LAUNCH(D, S)                                                                    \
    hipLaunchKernelGGL((hx_half_staged_kernel<T, uint32_t, R, C, D, S>), dim3(grid),       \
                       dim3(t->block), lds, st, g, x, y, pr, p.sigma, p.cprev, p.partial, \
                       store, p.stopped)
    const bool dot = p.partial != nullptr, sto = store != nullptr;
    if (!dot && !sto) HM_LAUNCH(false, false);
    else if (dot && !sto) HM_LAUNCH(true, false);
    else if (!dot && sto) HM_LAUNCH(false, true);
    else HM_LAUNCH(true, true);
#undef HM_LAUNCH
}

template <typename T>
static void launch_staged_t(const HalfTables *t, HalfArgs<uint32_t> g, const HxPass &p,
                            hipStream_t st) {
    g.n_items = (uint32_t)t->n_groups;
    if (t->C == 2) {
        if (t->R == 1) launch_staged<T, 1, 2>(t, g, p, st);
        else if (t->R == 2) launch_staged<T, 2, 2>(t, g, p, st);
        else launch_staged<T, 4, 2>(t, g, p, st);
    } else if (t->C == 4) {
        if (t->R == 1) launch_staged<T, 1, 4>(t, g, p, st);
        else if (t->R == 2) launch_staged<T, 2, 4>(t, g, p, st);
        else launch_staged<T, 4, 4>(t, g, p, st);
    } else {
        if (t->R == 1) launch_staged<T, 1, 8>(t, g, p, st);
        else launch_staged<T, 2, 8>(t, g, p, st);
    }
}

template <typename T, typename I>
static void launch_t(const HalfTables *t, const HalfBonds *hb, const Basis *b, double shift,
                     const HxPass &p, hipStream_t st) {
    HalfArgs<I> g{};
    g.rankL = t->d_rankL;
    g.unrankL = t->d_unrankL;
    g.off = (const I *)t->d_off;
    g.nbr = (const I *)hb->nbr;
    g.hcnt = hb->hcnt;
    g.hidx = hb->hidx;
    g.hgroups = t->d_hgroups;
    g.items = t->d_items;
    g.groups = hb->groups;
    g.n_items = (uint32_t)t->n_items;
    g.K = t->K;
    g.A = b->A;
    g.nLg = hb->nLg;
    g.nHg = hb->nHg;
    g.nSg = hb->nSg;
    g.nL = hb->nL;
    g.nS = hb->nS;
    g.width = (hb->nHg + hb->nSg) * kGroup;
    g.shift = shift;
    for (int a = 0; a <= kHalfMaxK + 1; ++a) {
        g.class_start[a] = t->class_start[a];
        g.class_size[a] = t->class_size[a];
    }
    if constexpr (sizeof(I) == 4) {
        if (t->C > 0) {
            launch_staged_t<T>(t, g, p, st);
            return;
        }
    }
    switch (t->R) {
        case 1: launch_r<T, I, 1>(t, g, p, st); break;
        case 2: launch_r<T, I, 2>(t, g, p, st); break;
        case 4: launch_r<T, I, 4>(t, g, p, st); break;
        default: launch_r<T, I, 8>(t, g, p, st); break;
    }
}

// Builds the tables and the regrouped bonds (also ahead of a graph capture:
// no allocation may happen while a stream is capturing).
int half_prepare_tables(Basis *b, const Couplings *c) {
    HalfTables *t = nullptr;
    HM_TRY(half_prepare(b, &t));
    const HalfBonds *hb = nullptr;
    return half_bonds(b, c, t, &hb);
}

// Whether the block kernel can run these couplings (neighbour table budget).
bool half_fits(const Basis *b, const Couplings *c) {
    return half_supported(b) && neighbour_bytes(b, c, low_bits_of(b)) <= kMaxNeighbourBytes;
}

int launch_hx_half(const Basis *cb, const Couplings *c, int dtype, const HxPass &p,
                   hipStream_t st) {
    Basis *b = const_cast<Basis *>(cb);
    HalfTables *t = nullptr;
    HM_TRY(half_prepare(b, &t));
    const HalfBonds *hb = nullptr;
    HM_TRY(half_bonds(b, c, t, &hb));
    if (dtype == HM_F64) {
        if (b->idx32) launch_t<double, uint32_t>(t, hb, b, c->diag_shift, p, st);
        else launch_t<double, uint64_t>(t, hb, b, c->diag_shift, p, st);
    } else {
        if (b->idx32) launch_t<float, uint32_t>(t, hb, b, c->diag_shift, p, st);
        else launch_t<float, uint64_t>(t, hb, b, c->diag_shift, p, st);
    }
    HM_HIP(hipGetLastError());
    return HM_OK;
}

}  // namespace hm
