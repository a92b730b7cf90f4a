// C entry points for the device codec, the plain H x product and the bond
// correlations.  Argument checks happen here; kernels live in the .hip files.
#include <vector>

#include "hm_internal.h"

namespace hm {
int bond_corr_max_bonds();
}

using hm::fail;

extern "C" {

int hm_unrank_dev(hm_basis h, const int64_t *d_idx, int64_t n, uint64_t *d_state,
                  void *stream) {
    hm::clear_error();
    if (!h) return fail(HM_EINVAL, "null handle");
    if (n < 0) return fail(HM_EINVAL, "n < 0");
    if (n == 0) return HM_OK;
    if (!d_idx || !d_state) return fail(HM_EINVAL, "null device pointer");
    hm::Basis *b = &h->impl;
    {
        std::lock_guard<std::mutex> lock(b->mu);
        HM_TRY(hm::device_prepare(b));
    }
    return hm::launch_unrank(b, d_idx, n, d_state, (hipStream_t)stream);
}

int hm_rank_dev(hm_basis h, const uint64_t *d_state, int64_t n, int64_t *d_idx,
                void *stream) {
    hm::clear_error();
    if (!h) return fail(HM_EINVAL, "null handle");
    if (n < 0) return fail(HM_EINVAL, "n < 0");
    if (n == 0) return HM_OK;
    if (!d_idx || !d_state) return fail(HM_EINVAL, "null device pointer");
    hm::Basis *b = &h->impl;
    {
        std::lock_guard<std::mutex> lock(b->mu);
        HM_TRY(hm::device_prepare(b));
    }
    return hm::launch_rank(b, d_state, n, d_idx, (hipStream_t)stream);
}

int hm_apply(hm_basis h, const double *J, const void *d_x, void *d_y, int32_t dtype,
             void *stream) {
    hm::clear_error();
    if (!h || !d_x || !d_y) return fail(HM_EINVAL, "null argument");
    if (dtype != HM_F64 && dtype != HM_F32) return fail(HM_EINVAL, "unknown dtype %d", dtype);
    if (d_x == d_y) return fail(HM_EINVAL, "x and y must not alias");
    hm::Basis *b = &h->impl;
    hm::CouplingsRef cref;
    HM_TRY(hm::get_couplings(b, J, &cref));
    const hm::Couplings *c = cref.get();
    hm::HxPass p;
    p.x = d_x;
    p.y = d_y;
    return hm::launch_hx(b, c, dtype, hm::choose_kernel(b, c, 0), p, (hipStream_t)stream);
}

// Variant of hm_apply that forces one H x kernel (1: generic digits, 2: the
// spin-1/2 block kernel, 3: successor sweep, 4: column scatter); used to
// cross-check the kernels and to time the paper's design alternatives.
int hm_apply_kernel(hm_basis h, const double *J, const void *d_x, void *d_y, int32_t dtype,
                    int32_t kernel, void *stream) {
    hm::clear_error();
    if (!h || !d_x || !d_y) return fail(HM_EINVAL, "null argument");
    if (dtype != HM_F64 && dtype != HM_F32) return fail(HM_EINVAL, "unknown dtype %d", dtype);
    if (d_x == d_y) return fail(HM_EINVAL, "x and y must not alias");
    hm::Basis *b = &h->impl;
    if (kernel < 1 || kernel > 4) return fail(HM_EINVAL, "kernel must be 1, 2, 3 or 4");
    hm::CouplingsRef cref;
    HM_TRY(hm::get_couplings(b, J, &cref));
    const hm::Couplings *c = cref.get();
    if (kernel >= 3) return hm::launch_hx_ablation(b, c, dtype, kernel, d_x, d_y, (hipStream_t)stream);
    const int k = hm::choose_kernel(b, c, kernel);
    if (k < 0) return fail(HM_EINVAL, "kernel %d not applicable", kernel);
    hm::HxPass p;
    p.x = d_x;
    p.y = d_y;
    return hm::launch_hx(b, c, dtype, k, p, (hipStream_t)stream);
}

// Layout of the bond-correlation workspace: the sorted bond list, the
// per-workgroup partial sums of one chunk of bonds, the results.
static void bond_corr_layout(const hm::Basis *b, int nb, size_t *uv_off, size_t *part_off,
                             size_t *out_off, size_t *total) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const int chunk = hm::bond_corr_max_bonds();
    const int nchunk = nb < chunk ? nb : chunk;
    size_t off = 0;
    *uv_off = off;
    off = al(off + sizeof(int32_t) * 2 * (size_t)nb);
    *part_off = off;
    off = al(off + sizeof(double) * (size_t)hm::bond_corr_blocks(b) * (size_t)nchunk);
    *out_off = off;
    off = al(off + sizeof(double) * (size_t)nb);
    *total = off;
}

int hm_bond_corr_workspace(hm_basis h, int32_t nb, size_t *bytes) {
    hm::clear_error();
    if (!h || !bytes) return fail(HM_EINVAL, "null argument");
    if (nb < 0) return fail(HM_EINVAL, "nb < 0");
    size_t a, b2, c;
    bond_corr_layout(&h->impl, nb, &a, &b2, &c, bytes);
    return HM_OK;
}

int hm_bond_corr(hm_basis h, const int32_t *uv, int32_t nb, const double *d_psi,
                 void *d_work, size_t work_bytes, double *corr, void *stream) {
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
    size_t uv_off, part_off, out_off, total;
    bond_corr_layout(b, nb, &uv_off, &part_off, &out_off, &total);
    if (!d_work) return fail(HM_EINVAL, "null workspace");
    if (work_bytes < total)
        return fail(HM_EWORKSPACE, "workspace %zu bytes < required %zu", work_bytes, total);
    {
        std::lock_guard<std::mutex> lock(b->mu);
        HM_TRY(hm::device_prepare(b));
    }
    hipStream_t st = (hipStream_t)stream;
    const int chunk = hm::bond_corr_max_bonds();
    const int nblocks = hm::bond_corr_blocks(b);
    std::vector<int32_t> sorted(2 * (size_t)nb);
    for (int i = 0; i < nb; ++i) {   // u < v, as the kernels expect
        const int u = uv[2 * i], v = uv[2 * i + 1];
        sorted[2 * i] = u < v ? u : v;
        sorted[2 * i + 1] = u < v ? v : u;
    }
    unsigned char *w = (unsigned char *)d_work;
    int32_t *d_uv = (int32_t *)(w + uv_off);
    double *d_partial = (double *)(w + part_off), *d_out = (double *)(w + out_off);
    int rc = HM_OK;
    hipError_t e = hipMemcpyAsync(d_uv, sorted.data(), sizeof(int32_t) * 2 * (size_t)nb,
                                  hipMemcpyHostToDevice, st);
    if (e != hipSuccess) rc = fail(HM_EDEVICE, "bond correlation setup: %s", hipGetErrorString(e));
    for (int b0 = 0; rc == HM_OK && b0 < nb; b0 += chunk) {
        const int m = nb - b0 < chunk ? nb - b0 : chunk;
        rc = hm::launch_bond_corr(b, d_uv + 2 * b0, m, d_psi, d_partial, nblocks, d_out + b0, st);
    }
    if (rc == HM_OK) {
        e = hipMemcpyAsync(corr, d_out, sizeof(double) * nb, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = fail(HM_EDEVICE, "bond correlation: %s", hipGetErrorString(e));
    }
    (void)hipStreamSynchronize(st);   // the host bond list outlives the copy
    return rc;
}

}  // extern "C"
