// Block Lanczos on H(M): several lowest eigenpairs at once, degenerate ones
// included, from p start vectors (the multi-vector product H X the batched
// path uses, here in FP64 on one instance).
//
// The paper's recurrence is the single-vector Lanczos method (Secs. 1, 4); its
// block form replaces the scalars alpha_k, beta_k by p x p blocks:
//   V_0 R_0 = X0                      (QR of the start block)
//   W = H V_k - V_{k-1} B_{k-1}^T
//   A_k = V_k^T W;   W -= V_k A_k
//   twice:  W -= sum_{j<=k} V_j (V_j^T W)      (full reorthogonalization)
//   V_{k+1} B_k = W                   (QR; B_k upper triangular)
// and the eigenvalues of the block tridiagonal matrix with diagonal blocks
// A_k and sub-diagonal blocks B_k approximate the lowest eigenvalues of H.
//
// Blocks are stored row-interleaved, [dim][p] FP64, so one decode of a basis
// state serves all p columns and a gathered row is p contiguous doubles.  The
// QR is Cholesky QR applied twice (the second pass restores orthogonality to
// rounding level); the p x p Cholesky factorizations run on the host.  Block
// dot products V^T W are per-workgroup partials summed in a fixed order, so a
// run is reproducible.
#include <algorithm>
#include <cmath>
#include <vector>

#include "device_common.h"
#include "hm_internal.h"
#include "hx_row.h"

namespace hm {

constexpr int kDotBlock = 256;
constexpr int kDotGrid = 256;

template <int P>
__device__ __forceinline__ void load_drow(const double *__restrict__ p, double (&v)[P]) {
    if constexpr (P % 2 == 0) {
#pragma unroll
        for (int q = 0; q < P / 2; ++q) {
            const double2 t = reinterpret_cast<const double2 *>(p)[q];
            v[2 * q] = t.x;
            v[2 * q + 1] = t.y;
        }
    } else {
        v[0] = p[0];
    }
}

// Y = H X for a [dim][P] block (generic digits, any s).
template <typename I, int B, int P>
__global__ __launch_bounds__(kBlock) void block_hx_kernel(
    const I *__restrict__ gprefix, const double *__restrict__ gladder,
    const BondDev *__restrict__ bonds, int nb, int N, int A, int two_s, I dim,
    const double *__restrict__ X, double *__restrict__ Y) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int plen = N * (A + 1) * (two_s + 1);
    I *Pt = reinterpret_cast<I *>(smem);
    double *F = reinterpret_cast<double *>(smem + ((plen * sizeof(I) + 15) / 16) * 16);
    for (int t = threadIdx.x; t < plen; t += blockDim.x) Pt[t] = gprefix[t];
    for (int t = threadIdx.x; t < two_s + 2; t += blockDim.x) F[t] = gladder[t];
    __syncthreads();
    const Prefix<I> pv{Pt, A + 1, two_s + 1};
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    I first, last;
    block_rows<I>(lb, gridDim.x, dim, first, last);
    for (I row = first + threadIdx.x; row < last; row += blockDim.x) {
        const uint64_t st = unrank_state<I, B>(row, pv, N, A, two_s);
        double xi[P], acc[P];
        load_drow<P>(X + (size_t)row * P, xi);
        double diag = 0.0;
#pragma unroll
        for (int q = 0; q < P; ++q) acc[q] = 0.0;
        for (int b = 0; b < nb; ++b) {
            const int u = bonds[b].u, v = bonds[b].v;
            const double mJ2 = bonds[b].mJ2;
            const int au = digit_at<B>(st, u), av = digit_at<B>(st, v);
            diag += bonds[b].mJ4 * (double)((two_s - 2 * au) * (two_s - 2 * av));
            if (au >= 1 && av < two_s) {
                const I j = row + move_delta<I, B>(st, u, v, -1, pv);
                const double c = mJ2 * F[au] * F[av + 1];
                double xj[P];
                load_drow<P>(X + (size_t)j * P, xj);
#pragma unroll
                for (int q = 0; q < P; ++q) acc[q] += c * xj[q];
            }
            if (av >= 1 && au < two_s) {
                const I j = row + move_delta<I, B>(st, u, v, +1, pv);
                const double c = mJ2 * F[av] * F[au + 1];
                double xj[P];
                load_drow<P>(X + (size_t)j * P, xj);
#pragma unroll
                for (int q = 0; q < P; ++q) acc[q] += c * xj[q];
            }
        }
#pragma unroll
        for (int q = 0; q < P; ++q) Y[(size_t)row * P + q] = diag * xi[q] + acc[q];
    }
}

// Per-workgroup partials of X_j^T W for the blocks j = blockIdx.y (X_j at
// X + j * dim * P): thread t of a group handles the pair (t / P, t % P); the
// 256 / P^2 groups take interleaved rows and are added in group order.
template <int P>
__global__ __launch_bounds__(kDotBlock) void block_dots_kernel(const double *__restrict__ X,
                                                               const double *__restrict__ W,
                                                               int64_t dim,
                                                               double *__restrict__ partial) {
    constexpr int PP = P * P, G = kDotBlock / PP;
    __shared__ double red[kDotBlock];
    const double *__restrict__ Xj = X + (size_t)blockIdx.y * dim * P;
    const int t = threadIdx.x % PP, g = threadIdx.x / PP;
    const int r = t / P, c = t % P;
    double s = 0.0;
    if (g < G) {
        const int64_t per = (dim + gridDim.x - 1) / gridDim.x;
        const int64_t lo = per * blockIdx.x, hi = std::min<int64_t>(lo + per, dim);
        for (int64_t row = lo + g; row < hi; row += G) s += Xj[row * P + r] * W[row * P + c];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < PP) {
        double acc = 0.0;
        for (int q = 0; q < G; ++q) acc += red[q * PP + threadIdx.x];
        partial[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * PP + threadIdx.x] = acc;
    }
}

// The same dots for P <= 4, JC blocks per workgroup: a thread keeps the P
// entries of W of its row in registers and adds the outer products with the
// rows of JC consecutive blocks, so each entry of W and X_j is loaded once per
// chunk (the kernel above loads each P times and W once per block).  Sums
// in a fixed order: per thread over its rows, a butterfly per wave, the waves
// in order.
constexpr int kDotChunk = 4;

template <int P>
__global__ __launch_bounds__(kDotBlock) void block_dots_chunk_kernel(
    const double *__restrict__ X, const double *__restrict__ W, int64_t dim, int nblk,
    double *__restrict__ partial) {
    constexpr int PP = P * P, JC = kDotChunk;
    __shared__ double stage[(kDotBlock / 64) * JC * PP];
    const int j0 = blockIdx.y * JC;
    double acc[JC][PP];
#pragma unroll
    for (int jj = 0; jj < JC; ++jj)
#pragma unroll
        for (int q = 0; q < PP; ++q) acc[jj][q] = 0.0;
    const int64_t per = (dim + gridDim.x - 1) / gridDim.x;
    const int64_t lo = per * blockIdx.x, hi = std::min<int64_t>(lo + per, dim);
    for (int64_t row = lo + threadIdx.x; row < hi; row += blockDim.x) {
        double w[P];
        load_drow<P>(W + row * P, w);
#pragma unroll
        for (int jj = 0; jj < JC; ++jj) {
            if (j0 + jj >= nblk) break;
            double xv[P];
            load_drow<P>(X + ((size_t)(j0 + jj) * dim + row) * P, xv);
#pragma unroll
            for (int r = 0; r < P; ++r)
#pragma unroll
                for (int c = 0; c < P; ++c) acc[jj][r * P + c] += xv[r] * w[c];
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int jj = 0; jj < JC; ++jj)
#pragma unroll
        for (int q = 0; q < PP; ++q) {
            const double v = wave_sum(acc[jj][q]);
            if (lane == 0) stage[(wid * JC + jj) * PP + q] = v;
        }
    __syncthreads();
    for (int t = threadIdx.x; t < JC * PP; t += blockDim.x) {
        const int jj = t / PP, q = t % PP;
        if (j0 + jj >= nblk) continue;
        double v = 0.0;
        for (int w8 = 0; w8 < (int)(blockDim.x >> 6); ++w8) v += stage[(w8 * JC + jj) * PP + q];
        partial[((size_t)(j0 + jj) * gridDim.x + blockIdx.x) * PP + q] = v;
    }
}

// out[j][pp] = sum over workgroups in order of partial[j][w][pp].
__global__ void block_dots_finish(const double *__restrict__ partial, int nparts, int PP,
                                  double *__restrict__ out) {
    const int j = blockIdx.x, pp = threadIdx.x;
    if (pp >= PP) return;
    double s = 0.0;
    for (int w = 0; w < nparts; ++w) s += partial[((size_t)j * nparts + w) * PP + pp];
    out[(size_t)j * PP + pp] = s;
}

// W[row][c] -= sum_{j < nblk} sum_r X_j[row][r] M_j[r][c]
template <int P>
__global__ __launch_bounds__(kBlock) void block_update_kernel(const double *__restrict__ X,
                                                              const double *__restrict__ M,
                                                              int nblk, int64_t dim,
                                                              double *__restrict__ W) {
    for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < dim;
         row += (int64_t)gridDim.x * blockDim.x) {
        double w[P];
        load_drow<P>(W + row * P, w);
        for (int j = 0; j < nblk; ++j) {
            double x[P];
            load_drow<P>(X + ((size_t)j * dim + row) * P, x);
            const double *__restrict__ Mj = M + (size_t)j * P * P;
#pragma unroll
            for (int r = 0; r < P; ++r)
#pragma unroll
                for (int c = 0; c < P; ++c) w[c] -= x[r] * Mj[r * P + c];
        }
#pragma unroll
        for (int c = 0; c < P; ++c) W[row * P + c] = w[c];
    }
}

// W[row] <- W[row] R^{-1} for the upper triangular R (row-vector solve)
template <int P>
__global__ __launch_bounds__(kBlock) void block_trsm_kernel(const double *__restrict__ R,
                                                            int64_t dim,
                                                            double *__restrict__ W) {
    for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < dim;
         row += (int64_t)gridDim.x * blockDim.x) {
        double w[P];
        load_drow<P>(W + row * P, w);
#pragma unroll
        for (int c = 0; c < P; ++c) {
            double v = w[c];
#pragma unroll
            for (int r = 0; r < c; ++r) v -= w[r] * R[r * P + c];
            w[c] = v / R[c * P + c];
        }
#pragma unroll
        for (int c = 0; c < P; ++c) W[row * P + c] = w[c];
    }
}

struct BlockLayout {
    size_t V, Wtmp, partial, dots, mats, total;
};

static size_t al256b(size_t x) { return (x + 255) & ~(size_t)255; }

static int block_layout(const Basis *b, int p, int steps, BlockLayout *L) {
    if (p != 1 && p != 2 && p != 4 && p != 8 && p != 16)
        return fail(HM_EINVAL, "block size p must be 1, 2, 4, 8 or 16");
    if (steps < 1) return fail(HM_EINVAL, "steps must be >= 1");
    const size_t blk = (size_t)b->dim * p * sizeof(double);
    size_t off = 0;
    L->V = off; off = al256b(off + blk * (size_t)(steps + 1));
    L->Wtmp = off; off = al256b(off + blk);
    L->partial = off; off = al256b(off + sizeof(double) * (size_t)(steps + 1) * kDotGrid * p * p);
    L->dots = off; off = al256b(off + sizeof(double) * (size_t)(steps + 1) * p * p);
    L->mats = off; off = al256b(off + sizeof(double) * (size_t)(steps + 1) * p * p);
    L->total = off;
    return HM_OK;
}

// Upper Cholesky factor R (G = R^T R) of a p x p symmetric matrix; false if
// a pivot is not above tol * (largest diagonal entry).
static bool cholesky_upper(const std::vector<double> &G, int p, double tol,
                           std::vector<double> &R) {
    R.assign((size_t)p * p, 0.0);
    double dmax = 0.0;
    for (int i = 0; i < p; ++i) dmax = std::max(dmax, G[(size_t)i * p + i]);
    if (!(dmax > 0.0)) return false;
    for (int i = 0; i < p; ++i) {
        double d = G[(size_t)i * p + i];
        for (int k = 0; k < i; ++k) d -= R[(size_t)k * p + i] * R[(size_t)k * p + i];
        if (!(d > tol * dmax)) return false;
        const double rii = std::sqrt(d);
        R[(size_t)i * p + i] = rii;
        for (int j = i + 1; j < p; ++j) {
            double s = G[(size_t)i * p + j];
            for (int k = 0; k < i; ++k) s -= R[(size_t)k * p + i] * R[(size_t)k * p + j];
            R[(size_t)i * p + j] = s / rii;
        }
    }
    return true;
}

namespace {

struct BlockRun {
    const Basis *b;
    const Couplings *c;
    int p, steps;
    unsigned char *w;
    BlockLayout L;
    hipStream_t st;
    double *V(int k) const { return (double *)(w + L.V) + (size_t)k * b->dim * p; }
    double *Wt() const { return (double *)(w + L.Wtmp); }
    double *partial() const { return (double *)(w + L.partial); }
    double *dots() const { return (double *)(w + L.dots); }
    double *mats() const { return (double *)(w + L.mats); }
};

template <int P>
int dots(const BlockRun &R, const double *X, int nblk, const double *W, std::vector<double> &out) {
    if constexpr (P <= 4)
        hipLaunchKernelGGL((block_dots_chunk_kernel<P>), dim3(kDotGrid, (nblk + kDotChunk - 1) / kDotChunk),
                           dim3(kDotBlock), 0, R.st, X, W, (int64_t)R.b->dim, nblk, R.partial());
    else
        hipLaunchKernelGGL((block_dots_kernel<P>), dim3(kDotGrid, nblk), dim3(kDotBlock), 0, R.st,
                           X, W, (int64_t)R.b->dim, R.partial());
    hipLaunchKernelGGL(block_dots_finish, dim3(nblk), dim3(P * P), 0, R.st, R.partial(),
                       kDotGrid, P * P, R.dots());
    HM_HIP(hipGetLastError());
    out.resize((size_t)nblk * P * P);
    HM_HIP(hipMemcpyAsync(out.data(), R.dots(), sizeof(double) * out.size(),
                          hipMemcpyDeviceToHost, R.st));
    HM_HIP(hipStreamSynchronize(R.st));
    return HM_OK;
}

template <int P>
int update(const BlockRun &R, const double *X, int nblk, const std::vector<double> &M, double *W) {
    HM_HIP(hipMemcpyAsync(R.mats(), M.data(), sizeof(double) * M.size(), hipMemcpyHostToDevice,
                          R.st));
    hipLaunchKernelGGL((block_update_kernel<P>), dim3(generic_grid(R.b->dim)), dim3(kBlock), 0,
                       R.st, X, R.mats(), nblk, (int64_t)R.b->dim, W);
    HM_HIP(hipGetLastError());
    return HM_OK;
}

// Cholesky QR applied twice to W in place; Rout = R2 R1.  Returns HM_ERANGE
// (not an error for the caller: breakdown) if W is numerically rank deficient
// or its largest squared column norm is at most `floor2`.
template <int P>
int cholqr2(const BlockRun &R, double *W, double tol, double floor2, std::vector<double> &Rout) {
    std::vector<double> G, R1, R2;
    for (int pass = 0; pass < 2; ++pass) {
        HM_TRY(dots<P>(R, W, 1, W, G));
        if (pass == 0) {
            double dmax = 0.0;
            for (int i = 0; i < P; ++i) dmax = std::max(dmax, G[(size_t)i * P + i]);
            if (!(dmax > floor2)) return HM_ERANGE;
        }
        for (int i = 0; i < P; ++i)   // symmetrize the rounding of the two triangles
            for (int j = i + 1; j < P; ++j)
                G[(size_t)i * P + j] = G[(size_t)j * P + i] =
                    0.5 * (G[(size_t)i * P + j] + G[(size_t)j * P + i]);
        std::vector<double> &Rk = pass == 0 ? R1 : R2;
        if (!cholesky_upper(G, P, pass == 0 ? tol : 1e-14, Rk)) return HM_ERANGE;
        HM_HIP(hipMemcpyAsync(R.mats(), Rk.data(), sizeof(double) * P * P,
                              hipMemcpyHostToDevice, R.st));
        hipLaunchKernelGGL((block_trsm_kernel<P>), dim3(generic_grid(R.b->dim)), dim3(kBlock), 0,
                           R.st, R.mats(), (int64_t)R.b->dim, W);
        HM_HIP(hipGetLastError());
    }
    Rout.assign((size_t)P * P, 0.0);
    for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) {
            double s = 0.0;
            for (int k = 0; k < P; ++k) s += R2[(size_t)i * P + k] * R1[(size_t)k * P + j];
            Rout[(size_t)i * P + j] = s;
        }
    return HM_OK;
}

template <typename I, int Bb, int P>
int run_block(BlockRun &R, const double *X0, double *Aout, double *Bout, int *done) {
    const Basis *b = R.b;
    const size_t blk = (size_t)b->dim * P * sizeof(double);
    const size_t lds = ((prefix_bytes(b) + 15) / 16) * 16 + (b->two_s + 2) * sizeof(double);
    const int grid = generic_grid(b->dim);
    const double tol = 1e-12;
    // V_0 R_0 = X0
    HM_HIP(hipMemcpyAsync(R.V(0), X0, blk, hipMemcpyDeviceToDevice, R.st));
    std::vector<double> Rq, Ak, C, Bprev;
    double scale = 0.0;   // running max |entry| of the A and B blocks
    int rc = cholqr2<P>(R, R.V(0), tol, 0.0, Rq);
    if (rc == HM_ERANGE) return fail(HM_EINVAL, "start block is rank deficient");
    HM_TRY(rc);
    *done = 0;
    for (int k = 0; k < R.steps; ++k) {
        double *W = R.V(k + 1);
        hipLaunchKernelGGL((block_hx_kernel<I, Bb, P>), dim3(grid), dim3(kBlock), lds, R.st,
                           (const I *)b->d_prefix, b->d_ladder, R.c->dev, R.c->nb, b->N, b->A,
                           b->two_s, (I)b->dim, R.V(k), W);
        HM_HIP(hipGetLastError());
        if (k > 0) {   // W -= V_{k-1} B_{k-1}^T
            std::vector<double> Bt((size_t)P * P);
            for (int i = 0; i < P; ++i)
                for (int j = 0; j < P; ++j) Bt[(size_t)i * P + j] = Bprev[(size_t)j * P + i];
            HM_TRY(update<P>(R, R.V(k - 1), 1, Bt, W));
        }
        HM_TRY(dots<P>(R, R.V(k), 1, W, Ak));
        HM_TRY(update<P>(R, R.V(k), 1, Ak, W));
        for (int i = 0; i < P; ++i)
            for (int j = 0; j < P; ++j) {
                const double a = 0.5 * (Ak[(size_t)i * P + j] + Ak[(size_t)j * P + i]);
                Aout[((size_t)k * P + i) * P + j] = a;
                scale = std::max(scale, std::fabs(a));
            }
        for (int pass = 0; pass < 2; ++pass) {
            HM_TRY(dots<P>(R, R.V(0), k + 1, W, C));
            HM_TRY(update<P>(R, R.V(0), k + 1, C, W));
        }
        *done = k + 1;
        if (k + 1 == R.steps) break;
        // breakdown when what is left of W is at rounding level of the
        // recurrence's scale: the block Krylov space is exhausted
        rc = cholqr2<P>(R, W, tol, (1e-12 * scale) * (1e-12 * scale), Bprev);
        if (rc == HM_ERANGE) break;
        HM_TRY(rc);
        for (size_t t = 0; t < (size_t)P * P; ++t) {
            Bout[(size_t)k * P * P + t] = Bprev[t];
            scale = std::max(scale, std::fabs(Bprev[t]));
        }
    }
    HM_HIP(hipStreamSynchronize(R.st));
    return HM_OK;
}

template <typename I, int Bb>
int dispatch_p(BlockRun &R, const double *X0, double *A, double *B, int *done) {
    switch (R.p) {
        case 1: return run_block<I, Bb, 1>(R, X0, A, B, done);
        case 2: return run_block<I, Bb, 2>(R, X0, A, B, done);
        case 4: return run_block<I, Bb, 4>(R, X0, A, B, done);
        case 8: return run_block<I, Bb, 8>(R, X0, A, B, done);
        default: return run_block<I, Bb, 16>(R, X0, A, B, done);
    }
}

template <typename I>
int dispatch_bits(BlockRun &R, const double *X0, double *A, double *B, int *done) {
    switch (R.b->bits) {
        case 1: return dispatch_p<I, 1>(R, X0, A, B, done);
        case 2: return dispatch_p<I, 2>(R, X0, A, B, done);
        case 3: return dispatch_p<I, 3>(R, X0, A, B, done);
        case 4: return dispatch_p<I, 4>(R, X0, A, B, done);
        default: return fail(HM_ERANGE, "block Lanczos supports up to 4 bits per digit");
    }
}

}  // namespace
}  // namespace hm

using hm::fail;

extern "C" {

int hm_block_lanczos_workspace(hm_basis h, int32_t p, int32_t steps, size_t *bytes) {
    hm::clear_error();
    if (!h || !bytes) return fail(HM_EINVAL, "null argument");
    hm::BlockLayout L;
    HM_TRY(hm::block_layout(&h->impl, p, steps, &L));
    *bytes = L.total;
    return HM_OK;
}

int hm_block_lanczos(hm_basis h, const double *J, const double *d_X0, int32_t p, int32_t steps,
                     void *d_work, size_t work_bytes, double *A, double *B, int32_t *steps_done,
                     void *stream) {
    hm::clear_error();
    if (!h || !J || !d_X0 || !d_work || !A || !B || !steps_done)
        return fail(HM_EINVAL, "null argument");
    hm::Basis *b = &h->impl;
    hm::BlockLayout L;
    HM_TRY(hm::block_layout(b, p, steps, &L));
    if (work_bytes < L.total)
        return fail(HM_EWORKSPACE, "workspace %zu bytes < required %zu", work_bytes, L.total);
    if (b->dim < p) return fail(HM_EINVAL, "block size p=%d exceeds the dimension", p);
    HM_TRY(hm::check_lds(b));
    hm::CouplingsRef cref;
    HM_TRY(hm::get_couplings(b, J, &cref));
    const hm::Couplings *c = cref.get();
    std::fill(A, A + (size_t)steps * p * p, 0.0);
    std::fill(B, B + (size_t)steps * p * p, 0.0);
    hm::BlockRun R{b, c, p, steps, (unsigned char *)d_work, L, (hipStream_t)stream};
    int done = 0;
    const int rc = b->idx32 ? hm::dispatch_bits<uint32_t>(R, d_X0, A, B, &done)
                            : hm::dispatch_bits<uint64_t>(R, d_X0, A, B, &done);
    *steps_done = done;
    return rc;
}

}  // extern "C"
