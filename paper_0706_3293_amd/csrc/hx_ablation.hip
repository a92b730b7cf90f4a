// Ablations of two of the paper's design choices for H x, kept for
// measurement (hm_apply_kernel kernels 3 and 4); neither is on the Lanczos
// path.
//
//  * Successor sweep (Sec. 3.1): each lane decodes only the first row of a run
//    of kRun consecutive rows and steps to the next rows with the successor
//    operation (one ball moved one box up, the lower boxes refilled from the
//    left) instead of decoding every row.  The per-row arithmetic is the
//    generic kernel's (row_hx), so y is bitwise identical; what changes is the
//    decode cost and the memory pattern (a lane walks its own run, so the
//    lanes of a wave touch rows kRun apart).
//  * Column scatter (Sec. 4): the loop order the paper rejects because of
//    write conflicts.  The source row j is outer: lane j adds H_ij x_j into
//    every y_i its state reaches, with hardware floating-point atomic adds
//    after y has been cleared.  Each y_i then receives its terms in a
//    run-dependent order.
#include "device_common.h"
#include "hm_internal.h"
#include "hx_row.h"

namespace hm {

constexpr int kRun = 16;

// Next basis state in the order of the encoding (Sec. 3.1): find the first
// box k (from site 1) that holds a ball while box k+1 has room, move one ball
// from k to k+1, and refill boxes 1..k from the left with the balls they held,
// at most 2s per box.  Returns false for the last state.
template <int B>
__device__ __forceinline__ bool successor_state(uint64_t &st, int N, int two_s) {
    int carry = 0;   // balls in the boxes below k
    for (int k = 0; k + 1 < N; ++k) {
        const int ak = digit_at<B>(st, k);
        if (ak >= 1 && digit_at<B>(st, k + 1) < two_s) {
            int balls = carry + ak - 1;
            const int nbits = (k + 1) * B;        // < N B <= 64
            uint64_t ns = (st >> nbits) << nbits;
            ns += (uint64_t)1 << nbits;
            for (int t = 0; balls > 0; ++t) {
                const int f = balls < two_s ? balls : two_s;
                ns |= (uint64_t)f << (t * B);
                balls -= f;
            }
            st = ns;
            return true;
        }
        carry += ak;
    }
    return false;
}

template <typename T, typename I>
__device__ __forceinline__ void load_tables(const I *__restrict__ gprefix,
                                            const double *__restrict__ gladder, int plen,
                                            int two_s, I *P, T *F) {
    for (int t = threadIdx.x; t < plen; t += blockDim.x) P[t] = gprefix[t];
    for (int t = threadIdx.x; t < two_s + 2; t += blockDim.x) F[t] = (T)gladder[t];
    __syncthreads();
}

template <typename T, typename I, int B>
__global__ __launch_bounds__(kBlock) void hx_successor_kernel(
    const I *__restrict__ gprefix, const double *__restrict__ gladder,
    const BondDev *__restrict__ bonds, int nb, int N, int A, int two_s, I dim,
    const T *__restrict__ x, T *__restrict__ y) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int plen = N * (A + 1) * (two_s + 1);
    I *P = reinterpret_cast<I *>(smem);
    T *F = reinterpret_cast<T *>(smem + ((plen * sizeof(I) + 15) / 16) * 16);
    load_tables<T, I>(gprefix, gladder, plen, two_s, P, F);
    const Prefix<I> pv{P, A + 1, two_s + 1};
    const uint64_t nruns = ((uint64_t)dim + kRun - 1) / kRun;
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < nruns;
         q += (uint64_t)gridDim.x * blockDim.x) {
        I row = (I)(q * kRun);
        const I end = (I)((q + 1) * kRun < (uint64_t)dim ? (q + 1) * kRun : (uint64_t)dim);
        uint64_t st = unrank_state<I, B>(row, pv, N, A, two_s);
        for (;;) {
            y[row] = row_hx<T, I, B>(st, row, x[row], x, bonds, nb, two_s, pv, F);
            if (++row >= end) break;
            successor_state<B>(st, N, two_s);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void fill_zero(T *__restrict__ y, int64_t n) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        y[t] = (T)0;
}

template <typename T, typename I, int B>
__global__ __launch_bounds__(kBlock) void hx_scatter_kernel(
    const I *__restrict__ gprefix, const double *__restrict__ gladder,
    const BondDev *__restrict__ bonds, int nb, int N, int A, int two_s, I dim,
    const T *__restrict__ x, T *__restrict__ y) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int plen = N * (A + 1) * (two_s + 1);
    I *P = reinterpret_cast<I *>(smem);
    T *F = reinterpret_cast<T *>(smem + ((plen * sizeof(I) + 15) / 16) * 16);
    load_tables<T, I>(gprefix, gladder, plen, two_s, P, F);
    const Prefix<I> pv{P, A + 1, two_s + 1};
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < (uint64_t)dim;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const I j = (I)t;
        const uint64_t st = unrank_state<I, B>(j, pv, N, A, two_s);
        const T xj = x[j];
        T diag = 0;
        for (int b = 0; b < nb; ++b) {
            const int u = bonds[b].u, v = bonds[b].v;
            const T mJ4 = (T)bonds[b].mJ4, mJ2 = (T)bonds[b].mJ2;
            const int au = digit_at<B>(st, u), av = digit_at<B>(st, v);
            diag += mJ4 * (T)((two_s - 2 * au) * (two_s - 2 * av));
            if (au >= 1 && av < two_s) {
                const I i = j + move_delta<I, B>(st, u, v, -1, pv);
                unsafeAtomicAdd(&y[i], (mJ2 * F[au] * F[av + 1]) * xj);
            }
            if (av >= 1 && au < two_s) {
                const I i = j + move_delta<I, B>(st, u, v, +1, pv);
                unsafeAtomicAdd(&y[i], (mJ2 * F[av] * F[au + 1]) * xj);
            }
        }
        unsafeAtomicAdd(&y[j], diag * xj);
    }
}

template <typename T, typename I, int B>
static void launch_ablation_t(const Basis *b, const Couplings *c, int kernel, const void *x,
                              void *y, hipStream_t st) {
    const int grid = generic_grid(kernel == 3 ? (b->dim + kRun - 1) / kRun : b->dim);
    const size_t lds = ((prefix_bytes(b) + 15) / 16) * 16 + (b->two_s + 2) * sizeof(double);
    const I *pref = (const I *)b->d_prefix;
    if (kernel == 3) {
        hipLaunchKernelGGL((hx_successor_kernel<T, I, B>), dim3(grid), dim3(kBlock), lds, st,
                           pref, b->d_ladder, c->dev, c->nb, b->N, b->A, b->two_s, (I)b->dim,
                           (const T *)x, (T *)y);
    } else {
        hipLaunchKernelGGL((fill_zero<T>), dim3(generic_grid(b->dim)), dim3(kBlock), 0, st,
                           (T *)y, (int64_t)b->dim);
        hipLaunchKernelGGL((hx_scatter_kernel<T, I, B>), dim3(grid), dim3(kBlock), lds, st,
                           pref, b->d_ladder, c->dev, c->nb, b->N, b->A, b->two_s, (I)b->dim,
                           (const T *)x, (T *)y);
    }
}

template <typename T, typename I>
static int ablation_bits(const Basis *b, const Couplings *c, int kernel, const void *x, void *y,
                         hipStream_t st) {
    switch (b->bits) {
        case 1: launch_ablation_t<T, I, 1>(b, c, kernel, x, y, st); break;
        case 2: launch_ablation_t<T, I, 2>(b, c, kernel, x, y, st); break;
        case 3: launch_ablation_t<T, I, 3>(b, c, kernel, x, y, st); break;
        case 4: launch_ablation_t<T, I, 4>(b, c, kernel, x, y, st); break;
        default: return fail(HM_ERANGE, "ablation kernels support up to 4 bits per digit");
    }
    return HM_OK;
}

int launch_hx_ablation(const Basis *b, const Couplings *c, int dtype, int kernel,
                       const void *x, void *y, hipStream_t st) {
    if (kernel != 3 && kernel != 4) return fail(HM_EINVAL, "ablation kernel must be 3 or 4");
    HM_TRY(check_lds(b));
    int rc;
    if (dtype == HM_F64)
        rc = b->idx32 ? ablation_bits<double, uint32_t>(b, c, kernel, x, y, st)
                      : ablation_bits<double, uint64_t>(b, c, kernel, x, y, st);
    else
        rc = b->idx32 ? ablation_bits<float, uint32_t>(b, c, kernel, x, y, st)
                      : ablation_bits<float, uint64_t>(b, c, kernel, x, y, st);
    HM_TRY(rc);
    HM_HIP(hipGetLastError());
    return HM_OK;
}

}  // namespace hm
