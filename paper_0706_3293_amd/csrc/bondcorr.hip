// Bond correlations <psi| s(u).s(v) |psi> for a list of bonds: the backward
// kernel of the ground-state energy (dE0/dJ_uv = -<s(u).s(v)>).
//
// Rows are visited in the gather form of Eq. (E-4-b): the lane that owns row
// i decodes |i>, and for every bond adds psi_i times the row i of s(u).s(v)
// applied to psi (diagonal m_u m_v psi_i plus the two ladder terms, each
// 1/2 * ladder factors * psi_j).  Per-bond sums are reduced wave by wave in a
// fixed butterfly order into per-wave LDS slots, then per workgroup, then
// over workgroups by a single workgroup: no atomics, bitwise reproducible.
#include <cstring>
#include <mutex>
#include <vector>

#include "device_common.h"
#include "hm_internal.h"

namespace hm {

constexpr int kCorrMaxBonds = 1024;
constexpr int kCorrBlock = 256;

template <typename I, int B>
__global__ __launch_bounds__(kCorrBlock) void bond_corr_kernel(
    const I *__restrict__ gprefix, const double *__restrict__ gladder,
    const int32_t *__restrict__ uv, int nb, int N, int A, int two_s, I dim,
    const double *__restrict__ psi, double *__restrict__ partial) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int plen = N * (A + 1) * (two_s + 1);
    const int nwaves = blockDim.x >> 6;
    I *P = reinterpret_cast<I *>(smem);
    size_t off = ((plen * sizeof(I) + 15) / 16) * 16;
    double *F = reinterpret_cast<double *>(smem + off);
    off += ((two_s + 2) * sizeof(double) + 15) / 16 * 16;
    double *acc = reinterpret_cast<double *>(smem + off);   // [nwaves][nb]
    for (int t = threadIdx.x; t < plen; t += blockDim.x) P[t] = gprefix[t];
    for (int t = threadIdx.x; t < two_s + 2; t += blockDim.x) F[t] = gladder[t];
    for (int t = threadIdx.x; t < nwaves * nb; t += blockDim.x) acc[t] = 0.0;
    __syncthreads();
    const Prefix<I> pv{P, A + 1, two_s + 1};
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    I first, last;
    block_rows<I>(xcd_logical_block(blockIdx.x, gridDim.x), gridDim.x, dim, first, last);
    // every lane runs the same number of iterations so the wave reductions
    // below see all 64 lanes; lanes past `last` contribute zero
    const I span = last - first;
    const I iters = (span + blockDim.x - 1) / blockDim.x;
    for (I it = 0; it < iters; ++it) {
        const I row = first + it * blockDim.x + threadIdx.x;
        const bool live = row < last;
        const uint64_t st = live ? unrank_state<I, B>(row, pv, N, A, two_s) : 0;
        const double pi = live ? psi[row] : 0.0;
        for (int b = 0; b < nb; ++b) {
            const int u = uv[2 * b], v = uv[2 * b + 1];
            double c = 0.0;
            if (live) {
                const int au = digit_at<B>(st, u), av = digit_at<B>(st, v);
                double s = 0.25 * (double)((two_s - 2 * au) * (two_s - 2 * av)) * pi;
                if (au >= 1 && av < two_s)
                    s += 0.5 * F[au] * F[av + 1] * psi[row + move_delta<I, B>(st, u, v, -1, pv)];
                if (av >= 1 && au < two_s)
                    s += 0.5 * F[av] * F[au + 1] * psi[row + move_delta<I, B>(st, u, v, +1, pv)];
                c = pi * s;
            }
            c = wave_sum(c);
            if (lane == 0) acc[wid * nb + b] += c;
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        double s = 0.0;
        for (int w = 0; w < nwaves; ++w) s += acc[w * nb + b];
        partial[(size_t)blockIdx.x * nb + b] = s;
    }
}

__global__ __launch_bounds__(kCorrBlock) void bond_corr_finish(const double *__restrict__ partial,
                                                               int nblocks, int nb,
                                                               double *__restrict__ out) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < nblocks; ++k) s += partial[(size_t)k * nb + b];
        out[b] = s;
    }
}

int bond_corr_blocks(const Basis *b) {
    int64_t g = (b->dim + kCorrBlock - 1) / kCorrBlock;
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    if (g >= kXcds) g -= g % kXcds;
    return (int)g;
}

int bond_corr_max_bonds() { return kCorrMaxBonds; }

template <typename I, int B>
static void launch_t(const Basis *b, const void *d_prefix, const double *d_ladder,
                     const int32_t *d_uv, int nb, const double *d_psi, double *d_partial,
                     int nblocks, double *d_out, hipStream_t st) {
    const size_t plen = b->prefix_len();
    size_t lds = ((plen * sizeof(I) + 15) / 16) * 16;
    lds += ((b->two_s + 2) * sizeof(double) + 15) / 16 * 16;
    lds += (size_t)(kCorrBlock / 64) * nb * sizeof(double);
    hipLaunchKernelGGL((bond_corr_kernel<I, B>), dim3(nblocks), dim3(kCorrBlock), lds, st,
                       (const I *)d_prefix, d_ladder, d_uv, nb, b->N, b->A, b->two_s,
                       (I)b->dim, d_psi, d_partial);
    hipLaunchKernelGGL(bond_corr_finish, dim3((nb + kCorrBlock - 1) / kCorrBlock),
                       dim3(kCorrBlock), 0, st, d_partial, nblocks, nb, d_out);
}

template <typename I>
static int launch_bits(const Basis *b, const void *tp, const double *tl, const int32_t *d_uv,
                       int nb, const double *d_psi, double *d_partial, int nblocks,
                       double *d_out, hipStream_t st) {
    switch (b->bits) {
        case 1: launch_t<I, 1>(b, tp, tl, d_uv, nb, d_psi, d_partial, nblocks, d_out, st); break;
        case 2: launch_t<I, 2>(b, tp, tl, d_uv, nb, d_psi, d_partial, nblocks, d_out, st); break;
        case 3: launch_t<I, 3>(b, tp, tl, d_uv, nb, d_psi, d_partial, nblocks, d_out, st); break;
        case 4: launch_t<I, 4>(b, tp, tl, d_uv, nb, d_psi, d_partial, nblocks, d_out, st); break;
        case 5: launch_t<I, 5>(b, tp, tl, d_uv, nb, d_psi, d_partial, nblocks, d_out, st); break;
        case 6: launch_t<I, 6>(b, tp, tl, d_uv, nb, d_psi, d_partial, nblocks, d_out, st); break;
        case 7: launch_t<I, 7>(b, tp, tl, d_uv, nb, d_psi, d_partial, nblocks, d_out, st); break;
        case 8: launch_t<I, 8>(b, tp, tl, d_uv, nb, d_psi, d_partial, nblocks, d_out, st); break;
        default: return fail(HM_ERANGE, "bits per digit %d unsupported", b->bits);
    }
    return HM_OK;
}

static int corr_lds_check(const Basis *b, int nb) {
    const size_t lds = ((b->prefix_len() * (b->idx32 ? 4 : 8) + 15) / 16) * 16 +
                       ((b->two_s + 2) * sizeof(double) + 15) / 16 * 16 +
                       (size_t)(kCorrBlock / 64) * nb * sizeof(double);
    if (lds > 64 * 1024) return fail(HM_ERANGE, "bond correlation tables exceed LDS");
    return HM_OK;
}

// Device tables from the handle (built on first device use).
int launch_bond_corr(const Basis *b, const int32_t *d_uv, int nb, const double *d_psi,
                     double *d_partial, int nblocks, double *d_out, hipStream_t st) {
    HM_TRY(corr_lds_check(b, nb));
    HM_TRY(b->idx32 ? launch_bits<uint32_t>(b, b->d_prefix, b->d_ladder, d_uv, nb, d_psi,
                                            d_partial, nblocks, d_out, st)
                    : launch_bits<uint64_t>(b, b->d_prefix, b->d_ladder, d_uv, nb, d_psi,
                                            d_partial, nblocks, d_out, st));
    HM_HIP(hipGetLastError());
    return HM_OK;
}

// ---------------------------------------------------------------------------
// The bond correlations without any device allocation, for callers that
// cannot allocate (code under graph capture, tight serving loops).  The
// prefix and ladder tables, the bond list, the per-workgroup partial sums
// and the results are staged in one file-scope device array.  In host code
// the array's name is only a stand-in for a device address: its address on
// each device is looked up once with hipGetSymbolAddress and that pointer is
// what the copies and kernels are given.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)4 << 20;
constexpr int kScratchMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kScratchMaxDevices] = {};

static int scratch_on_device(int dev, unsigned char **out) {
    if (dev < 0 || dev >= kScratchMaxDevices)
        return fail(HM_EDEVICE, "device %d outside 0..%d", dev, kScratchMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(HM_EDEVICE, "no device address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = (unsigned char *)g_scratch_ptr[dev];
    return HM_OK;
}

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace hm

using hm::fail;

extern "C" int hm_bond_corr_noalloc(hm_basis h, const int32_t *uv, int32_t nb,
                                    const double *d_psi, double *corr, void *stream) {
    hm::clear_error();
    if (!h || !uv || !d_psi || !corr) return fail(HM_EINVAL, "null argument");
    if (nb < 0) return fail(HM_EINVAL, "nb < 0");
    if (nb == 0) return HM_OK;
    hm::Basis *b = &h->impl;
    for (int i = 0; i < nb; ++i) {
        const int u = uv[2 * i], v = uv[2 * i + 1];
        if (u < 0 || v < 0 || u >= b->N || v >= b->N || u == v)
            return fail(HM_EINVAL, "bad bond %d: (%d, %d)", i, u, v);
    }
    if (nb > hm::kCorrMaxBonds)
        return fail(HM_ERANGE, "at most %d bonds per call without allocation", hm::kCorrMaxBonds);
    HM_TRY(hm::corr_lds_check(b, nb));
    int dev = 0;
    HM_HIP(hipGetDevice(&dev));
    if (b->device >= 0 && b->device != dev)
        return fail(HM_EDEVICE, "basis handle is bound to device %d, current is %d", b->device,
                    dev);
    hipDeviceProp_t prop;
    HM_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(HM_EDEVICE, "device %d is %s; this library is built for gfx950", dev,
                    prop.gcnArchName);
    // layout: prefix table, ladder factors, bond list, partial sums, results
    const int nblocks = hm::bond_corr_blocks(b);
    const size_t es = b->idx32 ? 4 : 8;
    std::vector<unsigned char> tables(b->prefix_len() * es);
    if (b->idx32) {
        uint32_t *p32 = (uint32_t *)tables.data();
        for (size_t i = 0; i < b->prefix_len(); ++i)
            p32[i] = b->prefix[i] > (int64_t)UINT32_MAX ? UINT32_MAX : (uint32_t)b->prefix[i];
    } else {
        std::memcpy(tables.data(), b->prefix.data(), tables.size());
    }
    std::vector<int32_t> sorted(2 * (size_t)nb);
    for (int i = 0; i < nb; ++i) {   // u < v, as the kernel expects
        const int u = uv[2 * i], v = uv[2 * i + 1];
        sorted[2 * i] = u < v ? u : v;
        sorted[2 * i + 1] = u < v ? v : u;
    }
    size_t off = 0;
    const size_t o_prefix = off;
    off = hm::al256(off + tables.size());
    const size_t o_ladder = off;
    off = hm::al256(off + b->ladder.size() * sizeof(double));
    const size_t o_uv = off;
    off = hm::al256(off + sorted.size() * sizeof(int32_t));
    const size_t o_part = off;
    off = hm::al256(off + (size_t)nblocks * nb * sizeof(double));
    const size_t o_out = off;
    off = hm::al256(off + (size_t)nb * sizeof(double));
    if (off > hm::kScratchBytes)
        return fail(HM_ERANGE, "%d bonds on %lld rows need %zu bytes of scratch, more than the "
                    "%zu the call without allocation has", nb, (long long)b->dim, off,
                    hm::kScratchBytes);
    unsigned char *ptr = nullptr;
    HM_TRY(hm::scratch_on_device(dev, &ptr));
    hipStream_t st = (hipStream_t)stream;
    HM_HIP(hipMemcpyAsync(ptr + o_prefix, tables.data(), tables.size(), hipMemcpyHostToDevice,
                          st));
    HM_HIP(hipMemcpyAsync(ptr + o_ladder, b->ladder.data(), b->ladder.size() * sizeof(double),
                          hipMemcpyHostToDevice, st));
    HM_HIP(hipMemcpyAsync(ptr + o_uv, sorted.data(), sorted.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, st));
    double *d_out = (double *)(ptr + o_out);
    int rc = b->idx32
        ? hm::launch_bits<uint32_t>(b, ptr + o_prefix, (const double *)(ptr + o_ladder),
                                    (const int32_t *)(ptr + o_uv), nb, d_psi,
                                    (double *)(ptr + o_part), nblocks, d_out, st)
        : hm::launch_bits<uint64_t>(b, ptr + o_prefix, (const double *)(ptr + o_ladder),
                                    (const int32_t *)(ptr + o_uv), nb, d_psi,
                                    (double *)(ptr + o_part), nblocks, d_out, st);
    if (rc == HM_OK) {
        hipError_t e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(corr, d_out, sizeof(double) * nb, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = fail(HM_EDEVICE, "bond correlation: %s", hipGetErrorString(e));
    }
    (void)hipStreamSynchronize(st);   // the host tables outlive the copies
    return rc;
}
