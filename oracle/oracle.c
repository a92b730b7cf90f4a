/*
 * Plain FP64 CPU oracle for the Heisenberg Lanczos hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or table with the HIP library; every routine here is written from
 * the paper's text (Schnack, Hage, Schmidt, "Optimized implementation of the
 * Lanczos method for magnetic systems"), in the paper's notation, with no
 * blocking, fusion or reordering beyond what the paper states.
 *
 * Conventions (readings of the paper, listed in the design notes):
 *   - site index u = 1..N in the paper is u-1 = 0..N-1 here;
 *   - digits a_u = s - m_u in {0..2s}; the spin is passed as two_s = 2s;
 *   - A = sum_u a_u, i.e. M = N s - A (Sec. 3);
 *   - basis indices are 0-based: index = (paper's 1-based index) - 1;
 *   - the Hamiltonian sum of Eq. (E-2-1) runs over unordered pairs u<v.
 *
 * Every function reports failure by a negative return value; none aborts.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_EXPORT __attribute__((visibility("default")))

/* ---------------------------------------------------------------------------
 * Count table D(n, A), Sec. 3, Eq. (E-3-c).
 *
 * D(n, A) is the number of n-site digit strings over {0..2s} whose digits sum
 * to A.  The paper builds it by the recursion
 *     D(n, A) = sum_{k=0}^{2s} D(n-1, A-k),
 * seeded with D(1, A) = 1 for A = 0..2s, and D(n, A) = 0 whenever A lies
 * outside {0, .., 2 n s}.  The table is stored as D[n * (N*two_s + 1) + A]
 * for n = 0..N, A = 0..N*two_s.  Row n = 0 holds D(0, 0) = 1 (the empty
 * string), which the recursion for n = 1 reproduces the paper's seed from.
 * Returns 0, or -1 if an entry would overflow int64.
 * ------------------------------------------------------------------------- */
OR_EXPORT int or_count_table(int N, int two_s, int64_t *D)
{
    const int W = N * two_s + 1;
    memset(D, 0, sizeof(int64_t) * (size_t)(N + 1) * (size_t)W);
    D[0] = 1;
    for (int n = 1; n <= N; ++n) {
        for (int A = 0; A <= n * two_s; ++A) {
            int64_t sum = 0;
            for (int k = 0; k <= two_s; ++k) {
                int prev = A - k;
                if (prev < 0 || prev > (n - 1) * two_s)
                    continue; /* zero outside the valid range */
                int64_t term = D[(size_t)(n - 1) * W + prev];
                if (term > INT64_MAX - sum)
                    return -1;
                sum += term;
            }
            D[(size_t)n * W + A] = sum;
        }
    }
    return 0;
}

/* D(n, A) with the paper's zero padding outside the valid index range. */
static int64_t count_at(const int64_t *D, int N, int two_s, int n, int A)
{
    if (n < 0 || n > N || A < 0 || A > n * two_s)
        return 0;
    return D[(size_t)n * (N * two_s + 1) + A];
}

/* ---------------------------------------------------------------------------
 * Cumulative block bound for the codec of Secs. 3.1 and 3.2.
 *
 * Among the strings on sites 1..k with digit sum T, those whose digit on site
 * k is m number D(k-1, T-m) (the other k-1 sites carry the rest, Eq. (E-3-c)).
 * In the order of Eq. (E-3-a) site k is the most significant of the k, so the
 * strings with a smaller digit on site k all come first.  below(k, T, n) is
 * the number of strings on sites 1..k with sum T and digit on site k smaller
 * than n, i.e. the position where the block with digit n starts.
 * ------------------------------------------------------------------------- */
static int64_t below(const int64_t *D, int N, int two_s, int k, int T, int n)
{
    int64_t start = 0;
    for (int m = 0; m < n && m <= two_s; ++m)
        start += count_at(D, N, two_s, k - 1, T - m);
    return start;
}

/* ---------------------------------------------------------------------------
 * Encoding |a_1 .. a_N> -> i, Sec. 3.2.
 *
 * The index of a state is the number of basis states that sort before it.
 * A state b sorts before a exactly when, at the most significant site k where
 * the two differ, b_k < a_k; b then agrees with a on sites k+1..N, so its
 * sites 1..k carry the same digit sum T_k = a_1 + .. + a_k.  Those states
 * number below(k, T_k, a_k) for each k, and the index is their total over
 * k = 1..N (the k = 1 term is zero: one site holds its sum in one way).
 * Sites are visited from k = 1 upward with T_k as a running prefix sum.
 * Returns the 0-based index, or -1 if a digit is out of {0..2s} or the digits
 * do not sum to A.
 * ------------------------------------------------------------------------- */
OR_EXPORT int64_t or_rank(int N, int two_s, int A, const int64_t *D,
                          const int *a)
{
    int64_t index = 0;
    int T = 0; /* digit sum of sites 1..k */
    for (int k = 1; k <= N; ++k) {
        const int digit = a[k - 1];
        if (digit < 0 || digit > two_s)
            return -1;
        T += digit;
        index += below(D, N, two_s, k, T, digit);
    }
    return T == A ? index : -1;
}

/* ---------------------------------------------------------------------------
 * Decoding i -> |a_1 .. a_N>, Sec. 3.1.
 *
 * The inverse of the count above, taken from the most significant site down.
 * On site k (with T the digit sum left for sites 1..k and r the position left
 * to reach among those strings) the blocks of strings with digit 0, 1, .., 2s
 * on site k follow one another, block n starting at below(k, T, n).  The digit
 * is the block that holds position r: the largest feasible n (n <= T, n <= 2s)
 * whose block starts at or before r.  Position r - below(k, T, n) inside that
 * block is what remains for sites 1..k-1.  On site 1 the rule leaves n = T.
 * `a` receives a[u-1] = a_u.  Returns 0, or -1 if i is not in [0, D(N, A)).
 * ------------------------------------------------------------------------- */
OR_EXPORT int or_unrank(int N, int two_s, int A, const int64_t *D, int64_t i,
                        int *a)
{
    if (i < 0 || i >= count_at(D, N, two_s, N, A))
        return -1;
    int64_t r = i;
    int T = A;
    for (int k = N; k >= 1; --k) {
        int digit = 0;
        for (int n = 1; n <= two_s && n <= T; ++n)
            if (below(D, N, two_s, k, T, n) <= r)
                digit = n;
        r -= below(D, N, two_s, k, T, digit);
        a[k - 1] = digit;
        T -= digit;
    }
    return (r == 0 && T == 0) ? 0 : -1;
}

/* Decoding of the consecutive indices first .. first+n-1 into rows of N
 * digits (out[t * N + u] = a_{u+1} of index first + t); each index is decoded
 * on its own with or_unrank.  Used to check device decoding over whole
 * subspaces.  Returns 0, or -1 if an index is out of range. */
OR_EXPORT int or_unrank_range(int N, int two_s, int A, const int64_t *D,
                              int64_t first, int64_t n, uint8_t *out)
{
    int failed = 0;
#pragma omp parallel
    {
        int *a = (int *)malloc(sizeof(int) * (size_t)N);
#pragma omp for schedule(static)
        for (int64_t t = 0; t < n; ++t) {
            if (!a || or_unrank(N, two_s, A, D, first + t, a) != 0) {
#pragma omp atomic write
                failed = 1;
                continue;
            }
            for (int u = 0; u < N; ++u)
                out[(size_t)t * N + u] = (uint8_t)a[u];
        }
        free(a);
    }
    return failed ? -1 : 0;
}

/* ---------------------------------------------------------------------------
 * Successor of a basis state, Sec. 3.1 ("balls in boxes").
 *
 * (1) find the leftmost box k holding a ball whose right neighbour k+1 holds
 *     fewer than 2s balls; if there is none the state is the last one;
 * (2) move one ball from box k to box k+1;
 * (3) collect the balls of boxes 1..k and refill them from the left, at most
 *     2s per box.
 * Returns 1 and updates `a` in place, or 0 if `a` has no successor.
 * ------------------------------------------------------------------------- */
OR_EXPORT int or_successor(int N, int two_s, int *a)
{
    int k = -1;
    for (int u = 0; u + 1 < N; ++u) {
        if (a[u] > 0 && a[u + 1] < two_s) {
            k = u;
            break;
        }
    }
    if (k < 0)
        return 0;
    a[k] -= 1;
    a[k + 1] += 1;
    int balls = 0;
    for (int u = 0; u <= k; ++u) {
        balls += a[u];
        a[u] = 0;
    }
    for (int u = 0; u <= k && balls > 0; ++u) {
        int put = balls < two_s ? balls : two_s;
        a[u] = put;
        balls -= put;
    }
    return 1;
}

/* ---------------------------------------------------------------------------
 * Row of H applied to a vector: the gather form of Eq. (E-4-b), Sec. 4.
 *
 * H = - sum_{u<v} J_uv s(u).s(v), Eq. (E-2-1), with
 *     s(u).s(v) = s_z(u) s_z(v) + (s+(u) s-(v) + s-(u) s+(v)) / 2.
 * Acting on the final basis state |i> gives
 *   - the diagonal element  -sum_{u<v} J_uv m_u m_v  with m = s - a;
 *   - for each bond and each of the two ladder terms that does not annihilate
 *     |i>, one state |j> and the element <i|H|j>.  With digits a = s - m the
 *     standard ladder algebra gives
 *         s+(u) s-(v): a_u -> a_u - 1, a_v -> a_v + 1,
 *                      factor sqrt(a_u (2s - a_u + 1)) sqrt((2s - a_v)(a_v + 1));
 *         s-(u) s+(v): the same with u and v exchanged;
 *     each multiplied by -J_uv / 2.
 * The output entry is y_i = sum over those j of <i|H|j> x_j; j comes from the
 * encoding above.  Only y_i is written, so rows are independent (the paper's
 * point about avoiding write conflicts).
 *
 * `J` is the dense N x N coupling matrix (row-major); only u<v entries are
 * read.  `cur` is the digit string of row i and is left unchanged; `work`
 * must hold N ints.
 * ------------------------------------------------------------------------- */
/* x_j of the input vector: x[j], or, when x is NULL, the counter-based value
 * of index j (Knuth's multiplicative hash with the 64-bit golden-ratio
 * constant, top 24 bits as a fraction, minus 1/2; exact in FP32 and FP64).
 * The hashed form checks single rows of problems whose vectors do not fit in
 * host memory. */
static double x_at(const double *x, int64_t j)
{
    if (x)
        return x[j];
    const uint64_t h = (uint64_t)j * 0x9E3779B97F4A7C15ull;
    return (double)(h >> 40) / 16777216.0 - 0.5;
}

static double apply_row(int N, int two_s, int A, const int64_t *D,
                        const double *J, const double *x, int64_t i,
                        const int *cur, int *work)
{
    const double s = 0.5 * two_s;
    double diag = 0.0;
    double y = 0.0;
    for (int u = 0; u < N; ++u) {
        for (int v = u + 1; v < N; ++v) {
            double Juv = J[(size_t)u * N + v];
            if (Juv == 0.0)
                continue;
            double mu = s - cur[u], mv = s - cur[v];
            diag += -Juv * mu * mv;
            /* s+(u) s-(v) */
            if (cur[u] >= 1 && cur[v] <= two_s - 1) {
                double f = sqrt((double)cur[u] * (two_s - cur[u] + 1)) *
                           sqrt((double)(two_s - cur[v]) * (cur[v] + 1));
                memcpy(work, cur, sizeof(int) * (size_t)N);
                work[u] -= 1;
                work[v] += 1;
                int64_t j = or_rank(N, two_s, A, D, work);
                y += -0.5 * Juv * f * x_at(x, j);
            }
            /* s-(u) s+(v) */
            if (cur[v] >= 1 && cur[u] <= two_s - 1) {
                double f = sqrt((double)cur[v] * (two_s - cur[v] + 1)) *
                           sqrt((double)(two_s - cur[u]) * (cur[u] + 1));
                memcpy(work, cur, sizeof(int) * (size_t)N);
                work[v] -= 1;
                work[u] += 1;
                int64_t j = or_rank(N, two_s, A, D, work);
                y += -0.5 * Juv * f * x_at(x, j);
            }
        }
    }
    return diag * x_at(x, i) + y;
}

/* ---------------------------------------------------------------------------
 * y = H x on the whole subspace H(M), Eqs. (E-4-a)/(E-4-b), Sec. 4.
 *
 * The loop over final rows i is the outer loop, as the paper prescribes.
 * Rows are visited in order: the first row of a chunk is decoded with
 * or_unrank, the following ones are reached with or_successor.  With OpenMP
 * the chunks of rows run on separate threads (the paper's shared-memory
 * scheme); without it the loop is serial.  Returns 0, or -1 on bad input.
 * ------------------------------------------------------------------------- */
OR_EXPORT int or_apply(int N, int two_s, int A, const int64_t *D,
                       const double *J, const double *x, double *y)
{
    const int64_t dim = count_at(D, N, two_s, N, A);
    if (dim <= 0)
        return -1;
    const int64_t chunk = 4096;
    const int64_t nchunks = (dim + chunk - 1) / chunk;
    int failed = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < nchunks; ++c) {
        int *cur = (int *)malloc(sizeof(int) * (size_t)N);
        int *work = (int *)malloc(sizeof(int) * (size_t)N);
        int64_t first = c * chunk;
        int64_t last = first + chunk < dim ? first + chunk : dim;
        if (!cur || !work || or_unrank(N, two_s, A, D, first, cur) != 0) {
#pragma omp atomic write
            failed = 1;
        } else {
            for (int64_t i = first; i < last; ++i) {
                y[i] = apply_row(N, two_s, A, D, J, x, i, cur, work);
                if (i + 1 < last)
                    or_successor(N, two_s, cur);
            }
        }
        free(cur);
        free(work);
    }
    return failed ? -1 : 0;
}

/* The same rows as or_apply, but only for the listed row indices: used to
 * check single rows of very large problems.  Each row is decoded on its own. */
OR_EXPORT int or_apply_rows(int N, int two_s, int A, const int64_t *D,
                            const double *J, const double *x,
                            const int64_t *rows, int64_t nrows, double *y)
{
    int failed = 0;
#pragma omp parallel
    {
        int *cur = (int *)malloc(sizeof(int) * (size_t)N);
        int *work = (int *)malloc(sizeof(int) * (size_t)N);
#pragma omp for schedule(static)
        for (int64_t r = 0; r < nrows; ++r) {
            if (!cur || !work || or_unrank(N, two_s, A, D, rows[r], cur) != 0) {
#pragma omp atomic write
                failed = 1;
                continue;
            }
            y[r] = apply_row(N, two_s, A, D, J, x, rows[r], cur, work);
        }
        free(cur);
        free(work);
    }
    return failed ? -1 : 0;
}

/* or_apply_rows with the counter-based input x_j of x_at (no x array). */
OR_EXPORT int or_apply_rows_hashed(int N, int two_s, int A, const int64_t *D,
                                   const double *J, const int64_t *rows, int64_t nrows,
                                   double *y)
{
    return or_apply_rows(N, two_s, A, D, J, NULL, rows, nrows, y);
}

/* Number of threads the OpenMP runtime would use (1 without OpenMP). */
OR_EXPORT int or_max_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
