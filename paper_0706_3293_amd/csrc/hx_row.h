// One row of the row-gather product (Sec. 4, Eq. (E-4-b)) for any spin s,
// shared by the generic kernel and its ablation variants so that they do the
// same arithmetic in the same order.
#pragma once

#include "device_common.h"
#include "hm_internal.h"

namespace hm {

constexpr size_t kMaxPrefixLds = 60 * 1024;

// (H x)_row for the decoded state st of `row`: the diagonal -sum J m_u m_v
// times x_row, plus x_j times the ladder matrix element for every bond whose
// two ladder terms do not annihilate the state (target j from the change of
// the encoding sum).  F holds the ladder factors sqrt(a(2s - a + 1)).
//
// Bonds go in groups of kRowGroup: the group's targets and gathers are all
// issued before the first product is added, so up to 2 kRowGroup gathers are
// in flight per lane; the sums still take the bonds in list order, so the
// result is the same as that of a plain loop over the bonds.
constexpr int kRowGroup = 4;

template <typename T, typename I, int B>
__device__ __forceinline__ T row_hx(uint64_t st, I row, T xi, const T *__restrict__ x,
                                    const BondDev *__restrict__ bonds, int nb, int two_s,
                                    const Prefix<I> &pv, const T *F) {
    T diag = 0, off = 0;
    for (int b0 = 0; b0 < nb; b0 += kRowGroup) {
        T cf[2 * kRowGroup], xv[2 * kRowGroup];
        bool on[2 * kRowGroup];
#pragma unroll
        for (int q = 0; q < kRowGroup; ++q) {
            on[2 * q] = on[2 * q + 1] = false;
            const int b = b0 + q;
            if (b < nb) {
                const int u = bonds[b].u, v = bonds[b].v;
                const T mJ4 = (T)bonds[b].mJ4, mJ2 = (T)bonds[b].mJ2;
                const int au = digit_at<B>(st, u), av = digit_at<B>(st, v);
                diag += mJ4 * (T)((two_s - 2 * au) * (two_s - 2 * av));
                if (au >= 1 && av < two_s) {   // s+(u) s-(v): a_u - 1, a_v + 1
                    const I j = row + move_delta<I, B>(st, u, v, -1, pv);
                    cf[2 * q] = mJ2 * F[au] * F[av + 1];
                    xv[2 * q] = x[j];
                    on[2 * q] = true;
                }
                if (av >= 1 && au < two_s) {   // s-(u) s+(v): a_u + 1, a_v - 1
                    const I j = row + move_delta<I, B>(st, u, v, +1, pv);
                    cf[2 * q + 1] = mJ2 * F[av] * F[au + 1];
                    xv[2 * q + 1] = x[j];
                    on[2 * q + 1] = true;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 2 * kRowGroup; ++q)
            if (on[q]) off += cf[q] * xv[q];
    }
    return diag * xi + off;
}

// row_hx with the row's encoding terms located first: for every site p the
// position base_p = ((p)(A+1) + A_p)(2s+1) + a_p of its term P[p+1][A_p][a_p]
// (A_p = digit sum of sites 0..p) goes to this lane's column of LDS,
// sb[p * stride].  A two-site move u < v changes the terms of sites u..v by
// fixed offsets from their bases (site u: du (2s+2), sites strictly between:
// du (2s+1), site v: -du), so a target index costs a few table reads instead
// of a digit walk.  The reads are the entries move_delta reads, the index sum
// is the same modulo 2^bits, and the products are added in the same order, so
// the result equals row_hx's bit for bit.
template <typename T, typename I, int B>
__device__ __forceinline__ T row_hx_tab(uint64_t st, I row, T xi, const T *__restrict__ x,
                                        const BondDev *__restrict__ bonds, int nb, int N,
                                        int two_s, const Prefix<I> &pv, const T *F,
                                        uint16_t *sb, int stride) {
    const int W = two_s + 1;
    const I *__restrict__ P = pv.p;
    {
        int A = 0;
        for (int p = 0; p < N; ++p) {
            const int ap = digit_at<B>(st, p);
            A += ap;
            sb[p * stride] = (uint16_t)((p * pv.A1 + A) * W + ap);
        }
    }
    T diag = 0, off = 0;
    for (int b0 = 0; b0 < nb; b0 += kRowGroup) {
        T cf[2 * kRowGroup], xv[2 * kRowGroup];
        bool on[2 * kRowGroup];
#pragma unroll
        for (int q = 0; q < kRowGroup; ++q) {
            on[2 * q] = on[2 * q + 1] = false;
            const int b = b0 + q;
            if (b < nb) {
                const int u = bonds[b].u, v = bonds[b].v;
                const T mJ4 = (T)bonds[b].mJ4, mJ2 = (T)bonds[b].mJ2;
                const int au = digit_at<B>(st, u), av = digit_at<B>(st, v);
                diag += mJ4 * (T)((two_s - 2 * au) * (two_s - 2 * av));
                const bool f1 = au >= 1 && av < two_s;   // s+(u) s-(v): a_u - 1, a_v + 1
                const bool f2 = av >= 1 && au < two_s;   // s-(u) s+(v): a_u + 1, a_v - 1
                if (f1 || f2) {
                    const int bu = sb[u * stride], bv = sb[v * stride];
                    const I ou = P[bu], ov = P[bv];
                    I mid1 = 0, mid2 = 0;                 // sites strictly between
                    for (int p = u + 1; p < v; ++p) {
                        const int bp = sb[p * stride];
                        const I op = P[bp];
                        if (f1) mid1 += P[bp - W] - op;
                        if (f2) mid2 += P[bp + W] - op;
                    }
                    if (f1) {
                        const I j = row + ((P[bu - W - 1] - ou) + mid1 + (P[bv + 1] - ov));
                        cf[2 * q] = mJ2 * F[au] * F[av + 1];
                        xv[2 * q] = x[j];
                        on[2 * q] = true;
                    }
                    if (f2) {
                        const I j = row + ((P[bu + W + 1] - ou) + mid2 + (P[bv - 1] - ov));
                        cf[2 * q + 1] = mJ2 * F[av] * F[au + 1];
                        xv[2 * q + 1] = x[j];
                        on[2 * q + 1] = true;
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 2 * kRowGroup; ++q)
            if (on[q]) off += cf[q] * xv[q];
    }
    return diag * xi + off;
}

// Launch helpers of the generic kernel family (hx_generic.hip).
size_t prefix_bytes(const Basis *b);
int check_lds(const Basis *b);
int generic_grid(int64_t rows);

}  // namespace hm
