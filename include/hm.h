/*
 * hm.h -- C ABI of the MI355X (gfx950) Lanczos hot path for isotropic
 * Heisenberg spin systems in a subspace of fixed total magnetic quantum number.
 *
 * Model (Sec. 2, Eq. (E-2-1)):  H = - sum_{u<v} J_uv s(u).s(v), all spins s.
 * The basis of the subspace H(M) is the set of product states |a_1..a_N> with
 * digits a_u = s - m_u in {0..2s} and digit sum A = N s - M (Sec. 3), numbered
 * in ascending order of the base-(2s+1) number sum_u a_u (2s+1)^(u-1), site 1
 * least significant (Eq. (E-3-a)).  Indices are 0-based (the paper counts from
 * 1).  Sites are numbered 0..N-1 here (site u here is the paper's u+1).
 *
 * Conventions shared by every call:
 *   - Every call returns an int status: HM_OK (0) or a negative HM_E* code.
 *     On failure hm_last_error() returns a message for the calling thread.
 *     No C++ exception crosses this boundary.
 *   - Spin and magnetization are passed doubled: two_s = 2s >= 1 and
 *     two_M = 2M, so half-integers are exact.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory on the current device.  The caller owns every buffer.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Device work is
 *     enqueued on it.  Calls that return host results synchronize the stream
 *     before returning; hm_apply, hm_unrank_dev and hm_rank_dev return right
 *     after enqueueing.
 *   - Coupling matrices J are host arrays of N*N doubles, row-major, which
 *     must be symmetric with a zero diagonal and finite entries (HM_EINVAL
 *     otherwise).  Only pairs with J_uv != 0 become bonds.
 *   - A basis handle is immutable once created (it keeps an internal,
 *     mutex-protected cache of uploaded coupling lists) and may be shared by
 *     threads.
 */
#ifndef HM_H
#define HM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define HM_OK 0
#define HM_EINVAL (-1)     /* invalid argument                                 */
#define HM_ERANGE (-2)     /* size not supported (bits, dimension, tables)     */
#define HM_ENOMEM (-3)     /* host or device allocation failed                 */
#define HM_EDEVICE (-4)    /* HIP runtime error or no usable gfx950 device     */
#define HM_EWORKSPACE (-5) /* workspace smaller than hm_lanczos_workspace says */

/* Element type of device vectors. */
#define HM_F64 0
#define HM_F32 1

/* Lanczos precision policy (north of the vector storage type):
 *   HM_PREC_F64       vectors, matrix elements and dots in FP64;
 *   HM_PREC_F32_MIXED vectors stored and H x matrix elements applied in FP32;
 *                     alpha/beta dots, norms, reorthogonalization
 *                     coefficients and ground-state accumulation in FP64. */
#define HM_PREC_F64 0
#define HM_PREC_F32_MIXED 1

typedef struct hm_basis_s *hm_basis;

/* Message describing the last failure on the calling thread ("" if none). */
const char *hm_last_error(void);

/* Library version string. */
const char *hm_version(void);

/* ---------------------------------------------------------------------------
 * Count table, Sec. 3 Eq. (E-3-c): D(n, A) is the number of n-digit strings
 * over {0..2s} with digit sum A; zero for A outside 0..2ns.
 * Writes D(n, A) to *out.  HM_EINVAL: n < 0, two_s < 1, null out.
 * HM_ERANGE: the value does not fit int64.
 * ------------------------------------------------------------------------- */
int hm_count(int32_t n, int32_t two_s, int32_t A, int64_t *out);

/* ---------------------------------------------------------------------------
 * Basis of H(M) (Sec. 3).  Builds the count table and the prefix tables the
 * encoding and decoding use (host memory; device copies are made on first
 * device use).  A = (N*two_s - two_M) / 2.
 * HM_EINVAL: N < 1, two_s < 1, N*two_s - two_M odd, or A outside 0..N*two_s;
 * null out.  HM_ERANGE: N * bits(2s) > 64 (a state does not fit the packed
 * 64-bit format below) or dim >= 2^62.
 * ------------------------------------------------------------------------- */
int hm_basis_init(int32_t N, int32_t two_s, int32_t two_M, hm_basis *out);

/* Releases the handle, its tables and cached device data.  Work enqueued
 * with the handle must have completed.  NULL is accepted. */
int hm_basis_free(hm_basis h);

/* Number of coupling lists the handle currently keeps on the device.  Each
 * distinct J passed with the handle is uploaded once (with the spin-1/2 block
 * kernel's neighbour table); at most 4 are kept, least recently used first
 * out, and one still in use by a running call is freed when that call
 * returns.  HM_EINVAL: null argument. */
int hm_basis_cached_couplings(hm_basis h, int32_t *count);

/* Dimension D(N, A) of the subspace. */
int hm_basis_dim(hm_basis h, int64_t *dim);

/* N, two_s, A, and the bits per digit of the packed state format. */
int hm_basis_info(hm_basis h, int32_t *N, int32_t *two_s, int32_t *A,
                  int32_t *bits_per_digit);

/* Schedule of the spin-1/2 block kernel (see hm_apply_kernel): the number of
 * low sites K whose words are decoded and encoded through LDS tables (rows
 * sharing the other N-K sites form one contiguous block), the threads per
 * workgroup, and the rows each lane carries (rows with one low word and
 * different high words, sharing the low-word work).  0 keeps the default
 * (K = min(N, 12) for N <= 30, 13 for N <= 36, else 14; 256 threads; 4 rows per lane when
 * dim >= 2^22, else 1).  Must be called before the first device use of the
 * handle.  HM_EINVAL: K outside 1..min(14, N) or N - K > 24, block_threads
 * not 64/128/256, rows_per_lane not 1/2/4/8, or tables already built.  Used
 * by the autotuner. */
int hm_basis_set_schedule(hm_basis h, int32_t low_bits, int32_t block_threads,
                          int32_t rows_per_lane);

/* Grid of the spin-1/2 block kernel: about items_per_wave work items per
 * wave (a work item is R blocks in the staged split, or R blocks' 64-row chunk
 * in the chunked one), so the grid may exceed the workgroups that are resident
 * at once and the hardware dispatcher balances items of unequal size; at most
 * 2^20 workgroups.  0 keeps the default: one item per wave up to 2048
 * workgroups, which then take several items each.  The Lanczos workspace
 * grows by one FP64 partial sum per workgroup.  Must be called before the
 * first device use of the handle.  Used by the autotuner.
 * HM_EINVAL: items_per_wave outside 0..65536, or tables already built. */
int hm_basis_set_items_per_wave(hm_basis h, int32_t items_per_wave);

/* Work split of the spin-1/2 block kernel: 1 = items of 64 rows of a block
 * (the low-word gathers read global memory); 2 = staged blocks: one wave takes
 * all rows of its R blocks, copies them to LDS and serves the gathers of the
 * bonds inside the low word from there (needs C(K, K/2) <= 512, i.e. K <= 11,
 * 32-bit indices, rows_per_lane <= 4 (<= 2 when K = 11); otherwise the first
 * device use fails with HM_EINVAL); 0 = automatic.  Must be called before the
 * first device use of the handle.  The two give bitwise equal results.
 * HM_EINVAL: mode outside 0..2 or tables already built. */
int hm_basis_set_staging(hm_basis h, int32_t mode);

/* ---------------------------------------------------------------------------
 * Decoding i -> |a_1..a_N> (Sec. 3.1) and encoding |a> -> i (Sec. 3.2) on the
 * host.  digits is a host array of N bytes, digits[u] = a_{u+1}.
 * hm_unrank: HM_EINVAL if i is outside [0, dim) or digits is null.
 * hm_rank:   HM_EINVAL if a digit exceeds 2s or the digits do not sum to A.
 * ------------------------------------------------------------------------- */
int hm_unrank(hm_basis h, int64_t i, uint8_t *digits);
int hm_rank(hm_basis h, const uint8_t *digits, int64_t *i);

/* ---------------------------------------------------------------------------
 * The same on the device, for n states at once.  Packed state format: a
 * uint64 holding digit a_{u+1} in bits [u*b, (u+1)*b), b = bits_per_digit
 * (b = 1 for s = 1/2, 2 for s = 1 and 3/2, 3 for s = 2..7/2, ...); unused high
 * bits are zero.
 * hm_unrank_dev: d_idx (device, n int64) -> d_state (device, n uint64);
 *   an index outside [0, dim) yields the state ~0 (all bits set).
 * hm_rank_dev: d_state -> d_idx; a state that is not in the subspace (digit
 *   above 2s, wrong digit sum, stray high bits) yields -1.
 * n = 0 is a no-op.  Asynchronous on `stream`.
 * ------------------------------------------------------------------------- */
int hm_unrank_dev(hm_basis h, const int64_t *d_idx, int64_t n,
                  uint64_t *d_state, void *stream);
int hm_rank_dev(hm_basis h, const uint64_t *d_state, int64_t n,
                int64_t *d_idx, void *stream);

/* ---------------------------------------------------------------------------
 * y = H x on the whole subspace, the gather form of Sec. 4 Eq. (E-4-b): each
 * output row i is produced by applying H to the basis state |i>, so every
 * entry of y is written by exactly one GPU lane and no atomics are used.
 * d_x, d_y: device arrays of dim elements of type `dtype` (HM_F64 or HM_F32);
 * they must not overlap.  With HM_F32 the matrix elements are rounded to
 * FP32 once and applied in FP32.  Asynchronous on `stream`.
 * HM_EINVAL: bad J (see above), null pointers, unknown dtype, d_x == d_y.
 * ------------------------------------------------------------------------- */
int hm_apply(hm_basis h, const double *J, const void *d_x, void *d_y,
             int32_t dtype, void *stream);

/* hm_apply with an explicit choice of H x kernel: 1 = the generic digit
 * kernel (any s), 2 = the spin-1/2 block kernel (s = 1/2 only; HM_EINVAL
 * otherwise).  Two more exist only to measure the paper's design
 * alternatives (bits per digit <= 4):
 *   3 = successor sweep (Sec. 3.1): each lane decodes the first of 16
 *       consecutive rows and reaches the others with the successor
 *       operation; y is bitwise equal to kernel 1's;
 *   4 = column scatter (Sec. 4, the loop order the paper rejects for its
 *       write conflicts): source row j outer, y_i += H_ij x_j with
 *       floating-point atomic adds after y is cleared; the order of the
 *       additions into each y_i varies from run to run.
 * All give y = H x; this entry point exists to cross-check the kernels and
 * to time them separately. */
int hm_apply_kernel(hm_basis h, const double *J, const void *d_x, void *d_y,
                    int32_t dtype, int32_t kernel, void *stream);

/* ---------------------------------------------------------------------------
 * Lanczos iteration (Sec. 1 and Sec. 4 name the method; the paper does not
 * write it out).  Paige's ordering:
 *   v_1 = v0/|v0|;  w = H v_k - beta_{k-1} v_{k-1};  alpha_k = <w, v_k>;
 *   w -= alpha_k v_k;  [full_reorth: twice w -= V_k (V_k^T w)];
 *   beta_k = |w|;  stop if beta_k <= breakdown_tol * max_{j<=k}(|alpha_j|, beta_j);
 *   v_{k+1} = w / beta_k.
 * E0 is the lowest eigenvalue of the tridiagonal T with diagonal alpha_1..k
 * and off-diagonal beta_1..k-1, found on the host in FP64 (Sturm bisection).
 * ------------------------------------------------------------------------- */
typedef struct hm_lanczos_opts {
    int32_t precision;    /* HM_PREC_F64 or HM_PREC_F32_MIXED               */
    int32_t full_reorth;  /* 1: classical Gram-Schmidt twice vs all v_j     */
    double breakdown_tol; /* relative; <= 0 selects 1e-12 (FP64) or 1e-6     *
                           * (FP32-mixed: the FP32 rounding floor of beta) */
    int32_t use_graph;    /* 1: run all steps as one hipGraph.  The step
                             loop is captured and instantiated on the first
                             call with a given handle, coupling matrix,
                             workspace address, step count and options,
                             kept with the handle (its 4 most recent
                             graphs) and replayed by later such calls; the
                             start vector may change between calls (same
                             kernels, bitwise equal results to direct
                             launches)                                    */
    int32_t kernel;       /* 0: automatic choice (the one-workgroup run
                             without full_reorth when dim x bonds <=
                             16384, else the H x kernel that suits
                             the basis); 1: generic digit kernel; 2:
                             spin-1/2 block kernel (if the basis is spin
                             1/2); 3: one-workgroup run (every step in one
                             launch of a single 1024-thread workgroup with
                             the generic row product; dim <= 2^20, else
                             HM_ERANGE; use_graph is ignored)            */
} hm_lanczos_opts;

/* Bytes of device workspace hm_lanczos / hm_lanczos_ritz need. */
int hm_lanczos_workspace(hm_basis h, int32_t steps, const hm_lanczos_opts *o,
                         size_t *bytes);

/* Runs up to `steps` steps from the device FP64 start vector d_v0 (dim
 * entries, any nonzero norm; it is normalized internally and not modified).
 * Outputs (host): alpha[steps], beta[steps] (entries past *steps_done are
 * zero), *E0, *steps_done.  A breakdown is not an error: HM_OK with
 * *steps_done < steps.  d_work: device workspace of work_bytes bytes (>=
 * hm_lanczos_workspace).  Synchronizes `stream`.
 * HM_EINVAL: bad J, steps < 1, null pointers, zero start vector.
 * HM_EWORKSPACE: work_bytes too small. */
int hm_lanczos(hm_basis h, const double *J, const double *d_v0, int32_t steps,
               const hm_lanczos_opts *o, void *d_work, size_t work_bytes,
               double *alpha, double *beta, double *E0, int32_t *steps_done,
               void *stream);

/* Ground-state recompute: repeats exactly the recurrence hm_lanczos ran
 * (same J, d_v0, options and workspace size, steps_done steps) and
 * accumulates psi = sum_k c_k v_k in FP64 on the device, then normalizes it.
 * c: host array of steps_done doubles (an eigenvector of T).  d_psi: device
 * FP64 array of dim entries (output).  alpha_out/beta_out (host, may be
 * NULL) receive the recomputed coefficients, which equal the first pass's
 * bit for bit.  Synchronizes `stream`. */
int hm_lanczos_ritz(hm_basis h, const double *J, const double *d_v0,
                    int32_t steps_done, const double *c,
                    const hm_lanczos_opts *o, void *d_work, size_t work_bytes,
                    double *d_psi, double *alpha_out, double *beta_out,
                    void *stream);

/* Lowest eigenpair of the k x k tridiagonal matrix diag(alpha) +
 * offdiag(beta[0..k-2]) on the host in FP64 (bisection on the Sturm sequence,
 * then inverse iteration).  evec (may be NULL): k doubles, unit norm, first
 * nonzero component made positive. */
int hm_tridiag_lowest(int32_t k, const double *alpha, const double *beta,
                      double *eval, double *evec);

/* ---------------------------------------------------------------------------
 * Block Lanczos: several lowest eigenpairs of H on H(M) at once, degenerate
 * ones included (the block form of the method's Lanczos recurrence, with p x p
 * blocks in place of alpha_k and beta_k; FP64 throughout):
 *   V_0 R_0 = X0;  W = H V_k - V_{k-1} B_{k-1}^T;  A_k = V_k^T W;
 *   W -= V_k A_k;  twice W -= sum_{j<=k} V_j (V_j^T W);  V_{k+1} B_k = W
 * (QR by Cholesky QR applied twice, B_k upper triangular).  The eigenvalues of
 * the block tridiagonal matrix with diagonal blocks A_0..A_{n-1} and
 * sub-diagonal blocks B_0..B_{n-2} (n = *steps_done) approximate the lowest
 * eigenvalues.  p: 1, 2, 4, 8 or 16 (and <= dim); bits per digit <= 4.
 * d_X0: device FP64 start block, row-interleaved [dim][p] (entry (i, q) at
 * i * p + q), linearly independent columns (else HM_EINVAL).  d_work:
 * hm_block_lanczos_workspace bytes of device memory, which hold all
 * (steps + 1) blocks of the Krylov basis.  A, B: host arrays of steps * p * p
 * doubles, row-major p x p blocks; unused entries are zero.  The run stops
 * early when the block Krylov space is exhausted (the rest of W is at the
 * rounding level of the recurrence).  Synchronizes `stream`.
 * ------------------------------------------------------------------------- */
int hm_block_lanczos_workspace(hm_basis h, int32_t p, int32_t steps, size_t *bytes);
int hm_block_lanczos(hm_basis h, const double *J, const double *d_X0, int32_t p,
                     int32_t steps, void *d_work, size_t work_bytes, double *A,
                     double *B, int32_t *steps_done, void *stream);

/* All Ritz values of a Lanczos tridiagonal and their Gauss weights (the
 * tridiagonal eigensolve of the method's final step, here with every
 * eigenpair).  values[j] (ascending) are the eigenvalues of the k x k matrix
 * diag(alpha) + offdiag(beta[0..k-2]); weights[j] = z_1j^2, the squared first
 * component of the unit eigenvector of values[j] (= |<v0|y_j>|^2 for a
 * Lanczos run from the unit start vector v0; the weights sum to 1).  Host
 * FP64, implicit shifted QR carrying only the first row of the eigenvector
 * matrix.  All pointers are host arrays of k (beta: k - 1) doubles owned by
 * the caller.  HM_EINVAL on k < 1, null or non-finite input, or no
 * convergence. */
int hm_tridiag_ritz(int32_t k, const double *alpha, const double *beta,
                    double *values, double *weights);

/* Finite-temperature Lanczos sums (k_B = 1; the estimator of Jaklic and
 * Prelovsek, Phys. Rev. B 49, 5065 (1994), built on the Ritz values and Gauss
 * weights of hm_tridiag_ritz).  nruns Lanczos runs: run r contributes
 * run_len[r] (level, weight) pairs, concatenated over the runs in run order
 * in `levels` and `weights`, and every weight of run r is multiplied by
 * run_scale[r] (for a run of one sector: the sector's multiplicity times its
 * dimension over the number of start vectors).  With E_min the lowest level
 * and b = scale * weight * exp(-(level - E_min) / T[t]), for each t:
 *   Z[t] = sum b   (the partition function divided by exp(-E_min / T[t])),
 *   E[t] = sum b level / Z[t],
 *   C[t] = (sum b level^2 / Z[t] - E[t]^2) / T[t]^2.
 * *E_min receives E_min.  Host FP64 with compensated sums; all
 * pointers are host arrays owned by the caller.  HM_EINVAL: nruns < 1,
 * nT < 1, a null pointer, a negative run length or scale, no pairs in all,
 * a non-finite input, T[t] <= 0, or weights that sum to zero. */
int hm_ftl_sums(int32_t nruns, const int32_t *run_len, const double *levels,
                const double *weights, const double *run_scale, int32_t nT,
                const double *T, double *Z, double *E, double *C, double *E_min);

/* Eigenvalues (ascending) of the symmetric block tridiagonal matrix of a block
 * Lanczos run: n diagonal blocks A (host, n x p x p row-major) and n - 1
 * sub-diagonal blocks B (host, (n - 1) x p x p; block k is the (k+1, k)
 * block, whose transpose sits above the diagonal).  values: host array of
 * n * p doubles.  Host FP64: Householder reduction of the assembled matrix to
 * tridiagonal form, then implicit shifted QR (the block form of the method's
 * final tridiagonal step).  HM_EINVAL: n < 1, p < 1, null or non-finite
 * input; HM_ERANGE: n * p > 20000. */
int hm_block_tridiag_eigenvalues(int32_t n, int32_t p, const double *A,
                                 const double *B, double *values);

/* ---------------------------------------------------------------------------
 * Bond correlations <psi| s(u).s(v) |psi> for nb bonds (uv: host int32
 * [nb][2], 0 <= u != v < N), psi a device FP64 vector of dim entries.
 * By Hellmann-Feynman dE0/dJ_uv = -<s(u).s(v)> for the normalized ground
 * state.  corr: host array of nb doubles.  Rows are processed in the gather
 * form of Eq. (E-4-b); per-bond sums are reduced in a fixed order (bitwise
 * reproducible).  d_work: caller-owned device workspace of at least
 * hm_bond_corr_workspace(h, nb) bytes (the bond list, per-workgroup partial
 * sums and the results live there; nothing is allocated per call).
 * Synchronizes `stream`.
 * HM_EINVAL: null pointers, nb < 0, a bond with u == v or a site outside
 * 0..N-1.  HM_EWORKSPACE: work_bytes too small.  nb == 0 is a no-op.
 * ------------------------------------------------------------------------- */
int hm_bond_corr_workspace(hm_basis h, int32_t nb, size_t *bytes);
int hm_bond_corr(hm_basis h, const int32_t *uv, int32_t nb, const double *d_psi,
                 void *d_work, size_t work_bytes, double *corr, void *stream);

/* hm_bond_corr for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same fixed-order sums (bitwise equal results),
 * with the device copies of the handle's tables, the bond list, the partial
 * sums and the results kept in one 4 MiB device array that the library owns
 * for the life of the process (one per GPU).  Calls no allocating routine,
 * does not need the handle's device tables to exist, and takes no workspace.
 * At most 1024 bonds, and the staged data must fit the array: prefix table +
 * bond list + (number of workgroups, <= 1024, ~dim/256) x nb doubles of
 * partial sums + nb results; HM_ERANGE beyond that (nb <= 480 fits any
 * dim).  Every call on one GPU uses that GPU's array and leaves it holding the
 * last call's data: calls that overlap on one GPU (other threads or streams)
 * race and must be serialized by the caller.  Synchronizes `stream`.
 * HM_EINVAL: as hm_bond_corr.  HM_EDEVICE: HIP error or not a gfx950 device.
 */
int hm_bond_corr_noalloc(hm_basis h, const int32_t *uv, int32_t nb,
                         const double *d_psi, double *corr, void *stream);

/* ---------------------------------------------------------------------------
 * Batched Lanczos: ninst independent problems, each with nvec start vectors,
 * solved together in FP32-mixed precision by one persistent (cooperative)
 * kernel launch that runs all steps; the multi-vector product H X shares one
 * decoding and one encoding per row among the nvec vectors.
 *   bases[k]     basis handle of instance k (any mix of N, s, M; states are
 *                packed with the digit width of the largest spin in the
 *                batch, so N_k * bits(s_max) <= 64 for every k);
 *   J[k]         host N_k x N_k coupling matrix;
 *   d_v0[k]      device FP64 array [dim_k][nvec] (row-major: the nvec start
 *                vectors interleaved, entry (i, r) at i*nvec + r);
 *   nvec         1..16 vectors per instance;
 *   alpha, beta  host arrays [ninst][nvec][steps];
 *   E0           host array [ninst][nvec];
 *   steps_done   host array [ninst][nvec].
 * Each (instance, vector) pair runs its own recurrence; a breakdown stops
 * only that pair.  Schedule: the rows are cut into 256-row items and the
 * persistent workgroups take `chunk` consecutive items at a time (1..64, 0 =
 * 4), with `wg_per_cu` workgroups resident per compute unit (1..8, capped by
 * occupancy; 0 = 4).  Every sum has a fixed order for a given schedule, so a
 * run is reproducible; the autotuner picks the schedule per workload.
 * d_work: device workspace of at least hm_lanczos_batched_workspace bytes.
 * Synchronizes `stream`.  HM_EINVAL: bad arguments or schedule.  HM_ERANGE:
 * an instance with N_k * bits(s_max) > 64, a dimension of 2^32 or more, or a
 * prefix table larger than the batch's LDS budget.
 * ------------------------------------------------------------------------- */
int hm_lanczos_batched_workspace(int32_t ninst, const hm_basis *bases,
                                 int32_t nvec, int32_t steps, size_t *bytes);
int hm_lanczos_batched(int32_t ninst, const hm_basis *bases,
                       const double *const *J, const double *const *d_v0,
                       int32_t nvec, int32_t steps, double breakdown_tol,
                       int32_t chunk, int32_t wg_per_cu, void *d_work,
                       size_t work_bytes, double *alpha, double *beta,
                       double *E0, int32_t *steps_done, void *stream);

/* Per-kernel timing of the last hm_lanczos call on this thread, measured
 * with HIP events on the call's stream: total milliseconds and launch count
 * of the H x pass (the dominant kernel) and of the whole step loop.  Timing
 * is recorded only when enabled with hm_set_timing(1) (events add a little
 * overhead and prevent graph capture of the steps). */
int hm_set_timing(int32_t enable);
int hm_last_timing(double *hx_ms, int32_t *hx_launches, double *loop_ms);

#ifdef __cplusplus
}
#endif

#endif /* HM_H */
