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

// Launch helpers of the generic kernel family (hx_generic.hip).
size_t prefix_bytes(const Basis *b);
int check_lds(const Basis *b);
int generic_grid(int64_t rows);

}  // namespace hm
