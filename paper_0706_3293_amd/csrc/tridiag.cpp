// Ritz values and Gauss weights of a Lanczos tridiagonal on the host (FP64).
//
// All eigenvalues of T = diag(alpha) + offdiag(beta) and the squared first
// components of their unit eigenvectors.  For a Lanczos run from a unit start
// vector v0 these are the Ritz values theta_j and the weights |<v0|y_j>|^2
// of the Krylov quadrature sum_j w_j f(theta_j) ~ <v0|f(H)|v0> that
// finite-temperature Lanczos sums are built from.
//
// Method: implicit symmetric QR with Wilkinson shifts (bulge chasing with
// Givens rotations), deflating converged off-diagonals from the bottom; only
// the first row of the accumulated rotation matrix is carried, as Golub and
// Welsch do for Gauss quadrature (Math. Comp. 23, 1969).
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <numeric>
#include <vector>

#include "hm_internal.h"

namespace hm {

namespace {

// One implicit shifted QR step on the unreduced block [l, m] of (d, e):
// e[i] couples i and i + 1.  z is the first row of the rotation product.
void qr_step(std::vector<double> &d, std::vector<double> &e, std::vector<double> &z, int l,
             int m) {
    // Wilkinson shift: eigenvalue of the trailing 2x2 block nearer d[m]
    const double a = d[m - 1], b = d[m], f = e[m - 1];
    const double delta = 0.5 * (a - b);
    const double sgn = delta >= 0.0 ? 1.0 : -1.0;
    const double mu = b - f * f / (delta + sgn * std::hypot(delta, f));
    // first rotation from the shifted first column, then chase the bulge
    double x = d[l] - mu, y = e[l];
    for (int k = l; k < m; ++k) {
        const double r = std::hypot(x, y);
        const double c = r == 0.0 ? 1.0 : x / r;
        const double s = r == 0.0 ? 0.0 : -y / r;
        if (k > l) e[k - 1] = r;   // the bulge at (k-1, k+1) is annihilated
        const double dk = d[k], dk1 = d[k + 1], ek = e[k];
        // new basis q_k' = c q_k - s q_{k+1}, q_{k+1}' = s q_k + c q_{k+1}
        d[k] = c * c * dk - 2.0 * c * s * ek + s * s * dk1;
        d[k + 1] = s * s * dk + 2.0 * c * s * ek + c * c * dk1;
        e[k] = c * s * (dk - dk1) + (c * c - s * s) * ek;
        if (k + 1 < m) {
            x = e[k];
            y = -s * e[k + 1];     // the new bulge at (k, k+2)
            e[k + 1] *= c;
        }
        const double z0 = z[k], z1 = z[k + 1];
        z[k] = c * z0 - s * z1;
        z[k + 1] = s * z0 + c * z1;
    }
}

bool negligible(const std::vector<double> &d, const std::vector<double> &e, int i) {
    return std::fabs(e[i]) <= DBL_EPSILON * (std::fabs(d[i]) + std::fabs(d[i + 1]));
}

}  // namespace

int tridiag_ritz(int k, const double *alpha, const double *beta, double *values,
                 double *weights) {
    if (k < 1) return fail(HM_EINVAL, "k must be >= 1");
    if (!alpha || !values || !weights || (k > 1 && !beta)) return fail(HM_EINVAL, "null argument");
    std::vector<double> d(alpha, alpha + k), e(k, 0.0), z(k, 0.0);
    for (int i = 0; i + 1 < k; ++i) e[i] = beta[i];
    for (int i = 0; i < k; ++i)
        if (!std::isfinite(d[i]) || !std::isfinite(e[i]))
            return fail(HM_EINVAL, "alpha/beta must be finite");
    z[0] = 1.0;
    int m = k - 1, iter = 0;
    const int max_iter = 60 * k;
    while (m > 0) {
        if (negligible(d, e, m - 1)) {
            e[m - 1] = 0.0;
            --m;
            continue;
        }
        int l = m - 1;
        while (l > 0 && !negligible(d, e, l - 1)) --l;
        if (l > 0) e[l - 1] = 0.0;
        if (++iter > max_iter) return fail(HM_EINVAL, "tridiagonal QR did not converge");
        qr_step(d, e, z, l, m);
    }
    std::vector<int> order(k);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
    for (int j = 0; j < k; ++j) {
        values[j] = d[order[j]];
        weights[j] = z[order[j]] * z[order[j]];
    }
    return HM_OK;
}

// Eigenvalues of the symmetric block tridiagonal matrix of a block Lanczos
// run (the block form of the final tridiagonal step): assemble the dense
// m x m matrix (m = n p), reduce it to tridiagonal form by Householder
// similarity transformations (Golub and Van Loan, Matrix Computations,
// Sec. 8.3.1: for column k the reflector P = I - tau v v^T, v_0 = 1, maps
// T[k+1.., k] onto a multiple of e_1, and T <- P T P through
// w = tau T v - (tau^2 / 2)(v^T T v) v, T <- T - v w^T - w v^T), then take
// the eigenvalues of the tridiagonal by the implicit QR of tridiag_ritz.
int block_tridiag_eigenvalues(int n, int p, const double *A, const double *B,
                              double *values) {
    if (n < 1 || p < 1) return fail(HM_EINVAL, "need n >= 1 and p >= 1");
    if (!A || !values || (n > 1 && !B)) return fail(HM_EINVAL, "null argument");
    const size_t m = (size_t)n * p;
    if (m > 20000) return fail(HM_ERANGE, "block tridiagonal order %zu above 20000", m);
    std::vector<double> T(m * m, 0.0);
    auto at = [&](size_t i, size_t j) -> double & { return T[i * m + j]; };
    for (int k = 0; k < n; ++k)
        for (int r = 0; r < p; ++r)
            for (int c = 0; c < p; ++c) {
                const double a = A[((size_t)k * p + r) * p + c];
                const double at_rc = A[((size_t)k * p + c) * p + r];
                if (!std::isfinite(a)) return fail(HM_EINVAL, "non-finite block entry");
                // the diagonal blocks are symmetric up to rounding: use the mean
                at((size_t)k * p + r, (size_t)k * p + c) = 0.5 * (a + at_rc);
                if (k + 1 < n) {
                    const double b = B[((size_t)k * p + r) * p + c];   // block (k+1, k)
                    if (!std::isfinite(b)) return fail(HM_EINVAL, "non-finite block entry");
                    at((size_t)(k + 1) * p + r, (size_t)k * p + c) = b;
                    at((size_t)k * p + c, (size_t)(k + 1) * p + r) = b;
                }
            }
    std::vector<double> d(m), e(m, 0.0), v(m), w(m);
    for (size_t k = 0; k + 2 < m; ++k) {
        // reflector for x = T[k+1.., k]
        const size_t q = k + 1;
        double sigma = 0.0;
        for (size_t i = q + 1; i < m; ++i) sigma += at(i, k) * at(i, k);
        const double x0 = at(q, k);
        if (sigma == 0.0) {                // already reduced in this column
            e[k] = x0;
            continue;
        }
        const double mu = std::sqrt(x0 * x0 + sigma);
        const double v0 = x0 <= 0.0 ? x0 - mu : -sigma / (x0 + mu);
        const double tau = 2.0 * v0 * v0 / (sigma + v0 * v0);
        v[q] = 1.0;
        for (size_t i = q + 1; i < m; ++i) v[i] = at(i, k) / v0;
        e[k] = mu;                         // P x = mu e_1 (sign absorbed: only |e| matters)
        // w = tau T v on the trailing block, then w -= (tau/2)(w^T v) v
        double wv = 0.0;
        for (size_t i = q; i < m; ++i) {
            double s = 0.0;
            for (size_t j = q; j < m; ++j) s += at(i, j) * v[j];
            w[i] = tau * s;
            wv += w[i] * v[i];
        }
        for (size_t i = q; i < m; ++i) w[i] -= 0.5 * tau * wv * v[i];
        for (size_t i = q; i < m; ++i)
            for (size_t j = q; j < m; ++j) at(i, j) -= v[i] * w[j] + w[i] * v[j];
    }
    for (size_t i = 0; i < m; ++i) d[i] = at(i, i);
    if (m >= 2) e[m - 2] = at(m - 1, m - 2);
    std::vector<double> weights(m);
    return tridiag_ritz((int)m, d.data(), e.data(), values, weights.data());
}

// Finite-temperature Lanczos sums over the Ritz values and Gauss weights of
// many runs (see hm_ftl_sums in hm.h).
int ftl_sums(int32_t nruns, const int32_t *run_len, const double *levels,
             const double *weights, const double *run_scale, int32_t nT, const double *T,
             double *Z, double *E, double *C, double *E_min) {
    if (nruns < 1 || nT < 1 || !run_len || !levels || !weights || !run_scale || !T || !Z ||
        !E || !C || !E_min)
        return fail(HM_EINVAL, "ftl_sums: nruns and nT must be >= 1 and pointers non-null");
    int64_t n = 0;
    for (int32_t r = 0; r < nruns; ++r) {
        if (run_len[r] < 0 || !std::isfinite(run_scale[r]) || run_scale[r] < 0.0)
            return fail(HM_EINVAL, "ftl_sums: run %d has a negative length or a bad scale", r);
        n += run_len[r];
    }
    if (n < 1) return fail(HM_EINVAL, "ftl_sums: no (level, weight) pairs");
    double emin = levels[0];
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(levels[i]) || !std::isfinite(weights[i]))
            return fail(HM_EINVAL, "ftl_sums: non-finite level or weight at %lld", (long long)i);
        emin = std::min(emin, levels[i]);
    }
    for (int32_t t = 0; t < nT; ++t)
        if (!std::isfinite(T[t]) || T[t] <= 0.0)
            return fail(HM_EINVAL, "ftl_sums: temperature %d is not a positive number", t);
    // compensated sums (Neumaier's variant of Kahan summation): C below
    // cancels <H^2> against <H>^2, so the sums are kept to about one ulp
    // however many levels there are
    struct Sum {
        double s = 0.0, c = 0.0;
        void add(double v) {
            const double t = s + v;
            c += std::fabs(s) >= std::fabs(v) ? (s - t) + v : (v - t) + s;
            s = t;
        }
        double value() const { return s + c; }
    };
    for (int32_t t = 0; t < nT; ++t) {
        Sum z, e, e2;
        int64_t i = 0;
        for (int32_t r = 0; r < nruns; ++r)
            for (int32_t k = 0; k < run_len[r]; ++k, ++i) {
                const double b = run_scale[r] * weights[i] * std::exp(-(levels[i] - emin) / T[t]);
                z.add(b);
                e.add(b * levels[i]);
                e2.add(b * levels[i] * levels[i]);
            }
        const double zt = z.value();
        if (!(zt > 0.0)) return fail(HM_EINVAL, "ftl_sums: the weights sum to zero");
        Z[t] = zt;
        E[t] = e.value() / zt;
        C[t] = (e2.value() / zt - E[t] * E[t]) / (T[t] * T[t]);
    }
    *E_min = emin;
    return HM_OK;
}

}  // namespace hm

extern "C" int hm_block_tridiag_eigenvalues(int32_t n, int32_t p, const double *A,
                                            const double *B, double *values) {
    hm::clear_error();
    return hm::block_tridiag_eigenvalues(n, p, A, B, values);
}

extern "C" int hm_tridiag_ritz(int32_t k, const double *alpha, const double *beta,
                               double *values, double *weights) {
    hm::clear_error();
    return hm::tridiag_ritz(k, alpha, beta, values, weights);
}

extern "C" int hm_ftl_sums(int32_t nruns, const int32_t *run_len, const double *levels,
                           const double *weights, const double *run_scale, int32_t nT,
                           const double *T, double *Z, double *E, double *C, double *E_min) {
    hm::clear_error();
    return hm::ftl_sums(nruns, run_len, levels, weights, run_scale, nT, T, Z, E, C, E_min);
}
