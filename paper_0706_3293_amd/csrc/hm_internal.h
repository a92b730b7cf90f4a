// Internal declarations shared by the host-side translation units of libhm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hm.h"

namespace hm {

// ---------------------------------------------------------------------------
// Error reporting: every failing path records a message for the calling
// thread and returns its status code.
// ---------------------------------------------------------------------------
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define HM_HIP(call)                                                          \
    do {                                                                      \
        hipError_t hm_e_ = (call);                                            \
        if (hm_e_ != hipSuccess)                                              \
            return ::hm::fail(HM_EDEVICE, "%s failed: %s", #call,             \
                              hipGetErrorString(hm_e_));                      \
    } while (0)

#define HM_TRY(expr)                                                          \
    do {                                                                      \
        int hm_rc_ = (expr);                                                  \
        if (hm_rc_ != HM_OK)                                                  \
            return hm_rc_;                                                    \
    } while (0)

// ---------------------------------------------------------------------------
// Device form of one bond (u < v) of H = -sum J_uv s(u).s(v).
// ---------------------------------------------------------------------------
struct BondDev {
    int32_t u, v;
    double mJ4;   // -J/4: diagonal element is mJ4 * (2 m_u)(2 m_v)
    double mJ2;   // -J/2: off-diagonal element is mJ2 * ladder factors
};

// One uploaded coupling list (immutable once built).  Calls hold it through a
// shared reference, so an entry evicted from the per-basis cache lives until
// the last call that uses it returns; its device arrays are freed after a
// device-wide synchronization (work enqueued with them may still be running).
struct Couplings {
    uint64_t serial = 0;      // unique per uploaded list (never reused)
    int nb = 0;
    std::vector<BondDev> host;
    BondDev *dev = nullptr;   // nb entries (nullptr when nb == 0)
    double diag_shift = 0.0;  // sum_b mJ4 (used by the spin-1/2 kernel)
    // bonds regrouped for the spin-1/2 block kernel (built on first use)
    void *half = nullptr;
    void (*half_free)(void *) = nullptr;
    ~Couplings() {
        if (dev || half) (void)hipDeviceSynchronize();
        if (dev) (void)hipFree(dev);
        if (half && half_free) half_free(half);
    }
};
using CouplingsRef = std::shared_ptr<Couplings>;

// Distinct coupling lists a basis handle keeps on the device (least recently
// used first out).
constexpr size_t kCouplingCacheEntries = 4;

// ---------------------------------------------------------------------------
// Basis of H(M): count table, prefix tables, device copies.
//
// Prefix table (Sec. 3.2 encoding):
//   P[k][Ak][a] = sum_{n < a} D(k-1, Ak - n),  k = 1..N, Ak = 0..A,
//   a = 0..2s, stored at ((k-1)*(A+1) + Ak)*(2s+1) + a.
// The index of a state is sum_{k=1..N} P[k][A_k][a_k] with A_k the digit sum
// of sites 1..k; decoding walks k = N..1 and picks the digit whose block holds
// the remaining offset.
// ---------------------------------------------------------------------------
struct Basis {
    int N = 0, two_s = 0, A = 0, bits = 0;
    int64_t dim = 0;
    bool idx32 = false;                 // dim < 2^32: 32-bit index arithmetic
    std::vector<int64_t> D;             // (N+1) x (N*two_s+1)
    std::vector<int64_t> prefix;        // N x (A+1) x (two_s+1)
    std::vector<double> ladder;         // F[a] = sqrt(a (2s - a + 1)), a = 0..2s+1

    int64_t count(int n, int a) const {
        if (n < 0 || n > N || a < 0 || a > n * two_s)
            return 0;
        return D[(size_t)n * (N * two_s + 1) + a];
    }
    size_t prefix_len() const { return (size_t)N * (A + 1) * (two_s + 1); }

    // lazily created device data, guarded by mu
    std::mutex mu;
    int device = -1;
    void *d_prefix = nullptr;           // uint32 or uint64 copy of prefix
    double *d_ladder = nullptr;
    // uploaded coupling lists, most recently used first (at most
    // kCouplingCacheEntries)
    std::list<std::pair<std::vector<double>, CouplingsRef>> couplings;
    // spin-1/2 block kernel: schedule (0 = default) and tables (first use)
    int half_K = 0;          // low bits per block word
    int half_block = 0;      // threads per workgroup (64, 128 or 256)
    int half_R = 0;          // rows per lane (high words sharing one low word)
    int half_staging = 0;    // 0 automatic, 1 chunked items, 2 staged blocks
    int half_ipw = 0;        // work items per wave that size the grid (0: default grid)
    void *half_tables = nullptr;
    void (*half_tables_free)(void *) = nullptr;
    // instantiated graphs of Lanczos step loops, most recently used first,
    // with the key of everything a capture bakes in (see lanczos.hip)
    struct Graph {
        std::vector<uint64_t> key;
        hipGraphExec_t exec = nullptr;
    };
    std::list<Graph> graphs;

    ~Basis();
};

// Step-loop graphs a basis handle keeps instantiated.
constexpr size_t kGraphCacheEntries = 4;

int device_prepare(Basis *b);                      // device tables + device check
int get_couplings(Basis *b, const double *J, CouplingsRef *out);
int validate_J(const Basis *b, const double *J);

// Host codec (Sec. 3.1 / 3.2), used by hm_unrank / hm_rank.
void host_unrank(const Basis *b, int64_t i, uint8_t *digits);
int64_t host_rank(const Basis *b, const uint8_t *digits);

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip translation units).
// ---------------------------------------------------------------------------
struct LzDev;   // device-side Lanczos scalars (see lanczos.cpp)

int launch_unrank(const Basis *b, const int64_t *d_idx, int64_t n,
                  uint64_t *d_state, hipStream_t st);
int launch_rank(const Basis *b, const uint64_t *d_state, int64_t n,
                int64_t *d_idx, hipStream_t st);

// Arguments of the fused H x pass used by hm_apply and by Lanczos.
//   y_i = sigma * (H x)_i - c * p_i,  sigma/c read from device scalars when
//   scal != nullptr (Lanczos) or taken as 1/0 otherwise (plain apply);
//   optional: partial[blk] = sum over the workgroup's rows of y_i sigma x_i
//             (FP64), store[i] = sigma * x_i (normalized Lanczos vector).
struct HxPass {
    const void *x = nullptr;
    void *y = nullptr;
    const void *p = nullptr;            // previous vector (nullptr: none)
    const double *sigma = nullptr;      // device scalar (nullptr: 1)
    const double *cprev = nullptr;      // device scalar (nullptr: 0)
    double *partial = nullptr;          // per-workgroup FP64 partial sums
    void *store = nullptr;              // optional normalized copy
    const int *stopped = nullptr;       // device flag: skip when nonzero
};

int hx_partial_count(const Basis *b, int kernel);      // partial slots needed
int launch_hx(const Basis *b, const Couplings *c, int dtype, int kernel,
              const HxPass &pass, hipStream_t st);
int choose_kernel(const Basis *b, const Couplings *c, int requested);
// Ablation kernels of hm_apply_kernel: 3 = successor sweep, 4 = column scatter.
int launch_hx_ablation(const Basis *b, const Couplings *c, int dtype, int kernel,
                       const void *x, void *y, hipStream_t st);

// Bond correlations.
int launch_bond_corr(const Basis *b, const int32_t *d_uv, int nb,
                     const double *d_psi, double *d_partial, int nblocks,
                     double *d_out, hipStream_t st);
int bond_corr_blocks(const Basis *b);

}  // namespace hm

struct hm_basis_s {
    hm::Basis impl;
};
