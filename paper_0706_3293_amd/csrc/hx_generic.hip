// Row-gather H x for any spin s (Sec. 4, Eq. (E-4-b)), and the device
// encoding/decoding entry points (Sec. 3.1, 3.2).
//
// One GPU lane owns one output row i: it decodes |i>, adds the diagonal
// element, and for every bond whose ladder term does not annihilate |i> it
// computes the target index j from the change of the encoding sum and
// gathers x_j.  Only y_i is written, so there are no write conflicts and no
// atomics.  The prefix table and the ladder factors are staged in LDS; the
// bond list is read with wave-uniform (scalar) loads.
#include "device_common.h"
#include "hm_internal.h"
#include "hx_row.h"

namespace hm {

template <typename T, typename I, int B, bool DOT, bool STORE, bool TAB>
__global__ __launch_bounds__(kBlock) void hx_generic_kernel(
    const I *__restrict__ gprefix, const double *__restrict__ gladder,
    const BondDev *__restrict__ bonds, int nb, int N, int A, int two_s, I dim,
    const T *__restrict__ x, T *__restrict__ y, const T *__restrict__ prev,
    const double *__restrict__ sigma_p, const double *__restrict__ cprev_p,
    double *__restrict__ partial, T *__restrict__ store, const int *__restrict__ stopped) {
    if (stopped && *stopped) return;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[16];
    const int plen = N * (A + 1) * (two_s + 1);
    I *P = reinterpret_cast<I *>(smem);
    const size_t pbytes = ((plen * sizeof(I) + 15) / 16) * 16;
    T *F = reinterpret_cast<T *>(smem + pbytes);
    // TAB: this lane's column of the per-site term positions (row_hx_tab)
    const size_t fbytes = (((size_t)two_s + 2) * sizeof(double) + 15) / 16 * 16;
    uint16_t *sb = reinterpret_cast<uint16_t *>(smem + pbytes + fbytes) + threadIdx.x;
    for (int t = threadIdx.x; t < plen; t += blockDim.x) P[t] = gprefix[t];
    for (int t = threadIdx.x; t < two_s + 2; t += blockDim.x) F[t] = (T)gladder[t];
    __syncthreads();
    const Prefix<I> pv{P, A + 1, two_s + 1};

    const double sigma = sigma_p ? *sigma_p : 1.0;
    const double cprev = cprev_p ? *cprev_p : 0.0;
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    I first, last;
    block_rows<I>(lb, gridDim.x, dim, first, last);
    double dot = 0.0;
    for (I row = first + threadIdx.x; row < last; row += blockDim.x) {
        const uint64_t st = unrank_state<I, B>(row, pv, N, A, two_s);
        const T xi = x[row];
        T hv;
        if constexpr (TAB)
            hv = row_hx_tab<T, I, B>(st, row, xi, x, bonds, nb, N, two_s, pv, F, sb, blockDim.x);
        else
            hv = row_hx<T, I, B>(st, row, xi, x, bonds, nb, two_s, pv, F);
        double w = sigma * (double)hv;
        if (prev) w -= cprev * (double)prev[row];
        const T wt = (T)w;
        y[row] = wt;
        if constexpr (DOT) dot += (double)wt * (sigma * (double)xi);
        if constexpr (STORE) store[row] = (T)(sigma * (double)xi);
    }
    if constexpr (DOT) {
        const double s = block_sum(dot, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

template <typename I, int B>
__global__ __launch_bounds__(kBlock) void unrank_kernel(const I *__restrict__ gprefix, int N,
                                                        int A, int two_s, int64_t dim,
                                                        const int64_t *__restrict__ idx,
                                                        int64_t n, uint64_t *__restrict__ out) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int plen = N * (A + 1) * (two_s + 1);
    I *P = reinterpret_cast<I *>(smem);
    for (int t = threadIdx.x; t < plen; t += blockDim.x) P[t] = gprefix[t];
    __syncthreads();
    const Prefix<I> pv{P, A + 1, two_s + 1};
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx[t];
        out[t] = (i < 0 || i >= dim) ? ~0ull : unrank_state<I, B>((I)i, pv, N, A, two_s);
    }
}

template <typename I, int B>
__global__ __launch_bounds__(kBlock) void rank_kernel(const I *__restrict__ gprefix, int N,
                                                      int A, int two_s,
                                                      const uint64_t *__restrict__ states,
                                                      int64_t n, int64_t *__restrict__ out) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int plen = N * (A + 1) * (two_s + 1);
    I *P = reinterpret_cast<I *>(smem);
    for (int t = threadIdx.x; t < plen; t += blockDim.x) P[t] = gprefix[t];
    __syncthreads();
    const Prefix<I> pv{P, A + 1, two_s + 1};
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t st = states[t];
        bool ok = N * B == 64 || (st >> (N * B)) == 0;
        int sum = 0;
        for (int u = 0; u < N; ++u) {
            const int a = digit_at<B>(st, u);
            ok = ok && a <= two_s;
            sum += a;
        }
        ok = ok && sum == A;
        out[t] = ok ? (int64_t)rank_state<I, B>(st, pv, N, A) : (int64_t)-1;
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
size_t prefix_bytes(const Basis *b) {
    return b->prefix_len() * (b->idx32 ? sizeof(uint32_t) : sizeof(uint64_t));
}

int check_lds(const Basis *b) {
    if (prefix_bytes(b) + 16 + (b->two_s + 2) * sizeof(double) > kMaxPrefixLds)
        return fail(HM_ERANGE, "prefix table (%zu bytes) exceeds the LDS budget",
                    prefix_bytes(b));
    return HM_OK;
}

int generic_grid(int64_t rows) {
    int64_t g = (rows + kBlock - 1) / kBlock;
    if (g > kMaxGrid) g = kMaxGrid;
    if (g < 1) g = 1;
    if (g >= kXcds) g -= g % kXcds;   // a multiple of 8 enables the XCD mapping
    return (int)g;
}

int hx_generic_grid(const Basis *b) { return generic_grid(b->dim); }

// LDS a workgroup of the generic kernel may take with the term positions.
constexpr size_t kMaxGenericLds = 64 * 1024;

template <typename T, typename I, int B>
static void launch_hx_t(const Basis *b, const Couplings *c, const HxPass &p, int grid,
                        size_t lds, hipStream_t st) {
    const I *pref = (const I *)b->d_prefix;
    const T *x = (const T *)p.x;
    T *y = (T *)p.y;
    const T *pr = (const T *)p.p;
    T *store = (T *)p.store;
    const bool dot = p.partial != nullptr, sto = store != nullptr;
    // tabulated term positions (row_hx_tab) for s >= 1: N x 256 x 2 bytes of
    // LDS beside the prefix table, and positions that fit 16 bits.  Measured
    // (one FP32 H x): s = 1, N = 16 ring 0.284 -> 0.268 ms; s = 2, N = 12
    // ring 0.924 -> 0.826 ms; for s = 1/2 it was slower (N = 28 J1-J2 ring
    // 4.56 -> 5.04 ms), where the digit walks are single popcounts.
    const size_t lds_tab = lds + (size_t)b->N * kBlock * sizeof(uint16_t);
    const bool tab = b->two_s >= 2 && lds_tab <= kMaxGenericLds && b->prefix_len() <= 65535;
#define HM_LAUNCH(D, S, TB)                                                                 \
    hipLaunchKernelGGL((hx_generic_kernel<T, I, B, D, S, TB>), dim3(grid), dim3(kBlock),    \
                       TB ? lds_tab : lds, st, pref, b->d_ladder, c->dev, c->nb, b->N, b->A, \
                       b->two_s, (I)b->dim, x, y, pr, p.sigma, p.cprev, p.partial, store,  \
                       p.stopped)
    if (tab) {
        if (!dot && !sto) HM_LAUNCH(false, false, true);
        else if (dot && !sto) HM_LAUNCH(true, false, true);
        else if (!dot && sto) HM_LAUNCH(false, true, true);
        else HM_LAUNCH(true, true, true);
    } else {
        if (!dot && !sto) HM_LAUNCH(false, false, false);
        else if (dot && !sto) HM_LAUNCH(true, false, false);
        else if (!dot && sto) HM_LAUNCH(false, true, false);
        else HM_LAUNCH(true, true, false);
    }
#undef HM_LAUNCH
}

template <typename T, typename I>
static int dispatch_bits(const Basis *b, const Couplings *c, const HxPass &p, int grid,
                         size_t lds, hipStream_t st) {
    switch (b->bits) {
        case 1: launch_hx_t<T, I, 1>(b, c, p, grid, lds, st); break;
        case 2: launch_hx_t<T, I, 2>(b, c, p, grid, lds, st); break;
        case 3: launch_hx_t<T, I, 3>(b, c, p, grid, lds, st); break;
        case 4: launch_hx_t<T, I, 4>(b, c, p, grid, lds, st); break;
        case 5: launch_hx_t<T, I, 5>(b, c, p, grid, lds, st); break;
        case 6: launch_hx_t<T, I, 6>(b, c, p, grid, lds, st); break;
        case 7: launch_hx_t<T, I, 7>(b, c, p, grid, lds, st); break;
        case 8: launch_hx_t<T, I, 8>(b, c, p, grid, lds, st); break;
        default: return fail(HM_ERANGE, "bits per digit %d unsupported", b->bits);
    }
    return HM_OK;
}

int launch_hx_generic(const Basis *b, const Couplings *c, int dtype, const HxPass &p,
                      hipStream_t st) {
    HM_TRY(check_lds(b));
    const int grid = generic_grid(b->dim);
    // prefix table, then the 2s + 2 ladder factors (room for doubles)
    const size_t lds = ((prefix_bytes(b) + 15) / 16) * 16 +
                       (((size_t)b->two_s + 2) * sizeof(double) + 15) / 16 * 16;
    int rc;
    if (dtype == HM_F64)
        rc = b->idx32 ? dispatch_bits<double, uint32_t>(b, c, p, grid, lds, st)
                      : dispatch_bits<double, uint64_t>(b, c, p, grid, lds, st);
    else
        rc = b->idx32 ? dispatch_bits<float, uint32_t>(b, c, p, grid, lds, st)
                      : dispatch_bits<float, uint64_t>(b, c, p, grid, lds, st);
    HM_TRY(rc);
    HM_HIP(hipGetLastError());
    return HM_OK;
}

template <typename I, int B>
static void launch_codec(const Basis *b, bool un, const int64_t *d_idx, const uint64_t *d_st,
                         int64_t n, uint64_t *o_st, int64_t *o_idx, hipStream_t st) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    const size_t lds = prefix_bytes(b);
    if (un)
        hipLaunchKernelGGL((unrank_kernel<I, B>), dim3((int)g), dim3(kBlock), lds, st,
                           (const I *)b->d_prefix, b->N, b->A, b->two_s, b->dim, d_idx, n,
                           o_st);
    else
        hipLaunchKernelGGL((rank_kernel<I, B>), dim3((int)g), dim3(kBlock), lds, st,
                           (const I *)b->d_prefix, b->N, b->A, b->two_s, d_st, n, o_idx);
}

template <typename I>
static int codec_bits(const Basis *b, bool un, const int64_t *d_idx, const uint64_t *d_st,
                      int64_t n, uint64_t *o_st, int64_t *o_idx, hipStream_t st) {
    switch (b->bits) {
        case 1: launch_codec<I, 1>(b, un, d_idx, d_st, n, o_st, o_idx, st); break;
        case 2: launch_codec<I, 2>(b, un, d_idx, d_st, n, o_st, o_idx, st); break;
        case 3: launch_codec<I, 3>(b, un, d_idx, d_st, n, o_st, o_idx, st); break;
        case 4: launch_codec<I, 4>(b, un, d_idx, d_st, n, o_st, o_idx, st); break;
        case 5: launch_codec<I, 5>(b, un, d_idx, d_st, n, o_st, o_idx, st); break;
        case 6: launch_codec<I, 6>(b, un, d_idx, d_st, n, o_st, o_idx, st); break;
        case 7: launch_codec<I, 7>(b, un, d_idx, d_st, n, o_st, o_idx, st); break;
        case 8: launch_codec<I, 8>(b, un, d_idx, d_st, n, o_st, o_idx, st); break;
        default: return fail(HM_ERANGE, "bits per digit %d unsupported", b->bits);
    }
    return HM_OK;
}

int launch_unrank(const Basis *b, const int64_t *d_idx, int64_t n, uint64_t *d_state,
                  hipStream_t st) {
    HM_TRY(check_lds(b));
    HM_TRY(b->idx32 ? codec_bits<uint32_t>(b, true, d_idx, nullptr, n, d_state, nullptr, st)
                    : codec_bits<uint64_t>(b, true, d_idx, nullptr, n, d_state, nullptr, st));
    HM_HIP(hipGetLastError());
    return HM_OK;
}

int launch_rank(const Basis *b, const uint64_t *d_state, int64_t n, int64_t *d_idx,
                hipStream_t st) {
    HM_TRY(check_lds(b));
    HM_TRY(b->idx32 ? codec_bits<uint32_t>(b, false, nullptr, d_state, n, nullptr, d_idx, st)
                    : codec_bits<uint64_t>(b, false, nullptr, d_state, n, nullptr, d_idx, st));
    HM_HIP(hipGetLastError());
    return HM_OK;
}

}  // namespace hm
