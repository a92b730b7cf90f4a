// Basis of H(M): count table, prefix tables and host encoding/decoding
// (Sec. 3 of the paper), handle management, argument validation and the
// per-handle cache of uploaded coupling lists.
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>

#include "hm_internal.h"

namespace hm {

static thread_local std::string g_error;

int fail(int code, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

void clear_error() { g_error.clear(); }

Basis::~Basis() {
    // Handles are freed after their work completed (documented contract).
    for (Graph &g : graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
    if (d_prefix) (void)hipFree(d_prefix);
    if (d_ladder) (void)hipFree(d_ladder);
    couplings.clear();   // each Couplings frees its device arrays
    if (half_tables && half_tables_free) half_tables_free(half_tables);
}

static int bits_for(int two_s) {
    int b = 0;
    while ((1 << b) <= two_s) ++b;
    return b;
}

// D(n, a) for n = 0..N, a = 0..N*two_s by the recursion of Eq. (E-3-c),
// saturating at INT64_MAX (saturated entries are rejected by the callers
// that need them).
static void build_counts(int N, int two_s, std::vector<int64_t> &D) {
    const int W = N * two_s + 1;
    D.assign((size_t)(N + 1) * W, 0);
    D[0] = 1;
    const int64_t cap = std::numeric_limits<int64_t>::max();
    for (int n = 1; n <= N; ++n)
        for (int a = 0; a <= n * two_s; ++a) {
            unsigned __int128 sum = 0;
            for (int k = 0; k <= two_s; ++k) {
                int prev = a - k;
                if (prev < 0 || prev > (n - 1) * two_s) continue;
                sum += (unsigned __int128)D[(size_t)(n - 1) * W + prev];
            }
            D[(size_t)n * W + a] = sum > (unsigned __int128)cap ? cap : (int64_t)sum;
        }
}

void host_unrank(const Basis *b, int64_t i, uint8_t *digits) {
    const int W = b->two_s + 1;
    int64_t r = i;
    int Ak = b->A;
    for (int k = b->N; k >= 1; --k) {
        const int64_t *row = &b->prefix[((size_t)(k - 1) * (b->A + 1) + Ak) * W];
        int a = 0;
        for (int t = 1; t <= b->two_s; ++t)
            a += row[t] <= r ? 1 : 0;
        r -= row[a];
        Ak -= a;
        digits[k - 1] = (uint8_t)a;
    }
}

int64_t host_rank(const Basis *b, const uint8_t *digits) {
    const int W = b->two_s + 1;
    int Ak = b->A;
    int64_t idx = 0;
    for (int k = b->N; k >= 1; --k) {
        int a = digits[k - 1];
        idx += b->prefix[((size_t)(k - 1) * (b->A + 1) + Ak) * W + a];
        Ak -= a;
    }
    return idx;
}

int validate_J(const Basis *b, const double *J) {
    if (!J) return fail(HM_EINVAL, "J is null");
    const int N = b->N;
    for (int u = 0; u < N; ++u) {
        if (J[(size_t)u * N + u] != 0.0)
            return fail(HM_EINVAL, "J[%d][%d] must be zero (no self-coupling)", u, u);
        for (int v = 0; v < N; ++v) {
            double x = J[(size_t)u * N + v];
            if (!std::isfinite(x))
                return fail(HM_EINVAL, "J[%d][%d] is not finite", u, v);
            if (x != J[(size_t)v * N + u])
                return fail(HM_EINVAL, "J is not symmetric at (%d, %d)", u, v);
        }
    }
    return HM_OK;
}

int device_prepare(Basis *b) {
    int dev = 0;
    HM_HIP(hipGetDevice(&dev));
    if (b->device >= 0) {
        if (dev != b->device)
            return fail(HM_EDEVICE, "basis handle is bound to device %d, current is %d",
                        b->device, dev);
        return HM_OK;
    }
    hipDeviceProp_t prop;
    HM_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(HM_EDEVICE, "device %d is %s; this library is built for gfx950",
                    dev, prop.gcnArchName);
    const size_t n = b->prefix_len();
    if (b->idx32) {
        std::vector<uint32_t> p32(n);
        for (size_t i = 0; i < n; ++i)
            p32[i] = b->prefix[i] > (int64_t)UINT32_MAX ? UINT32_MAX : (uint32_t)b->prefix[i];
        HM_HIP(hipMalloc(&b->d_prefix, n * sizeof(uint32_t)));
        HM_HIP(hipMemcpy(b->d_prefix, p32.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice));
    } else {
        HM_HIP(hipMalloc(&b->d_prefix, n * sizeof(int64_t)));
        HM_HIP(hipMemcpy(b->d_prefix, b->prefix.data(), n * sizeof(int64_t),
                         hipMemcpyHostToDevice));
    }
    HM_HIP(hipMalloc(&b->d_ladder, b->ladder.size() * sizeof(double)));
    HM_HIP(hipMemcpy(b->d_ladder, b->ladder.data(), b->ladder.size() * sizeof(double),
                     hipMemcpyHostToDevice));
    b->device = dev;
    return HM_OK;
}

// Bonds of J (u < v, J_uv != 0) in row-major upper-triangle order, uploaded
// once per distinct J.  The handle keeps the kCouplingCacheEntries most
// recently used lists; older ones are dropped (and freed once no running call
// holds them), so loops over many distinct J keep device memory bounded.
int get_couplings(Basis *b, const double *J, CouplingsRef *out) {
    HM_TRY(validate_J(b, J));
    const int N = b->N;
    std::vector<double> key(J, J + (size_t)N * N);
    std::lock_guard<std::mutex> lock(b->mu);
    HM_TRY(device_prepare(b));
    for (auto it = b->couplings.begin(); it != b->couplings.end(); ++it) {
        if (it->first == key) {
            b->couplings.splice(b->couplings.begin(), b->couplings, it);
            *out = b->couplings.front().second;
            return HM_OK;
        }
    }
    static std::atomic<uint64_t> next_serial{1};
    auto c = std::make_shared<Couplings>();
    c->serial = next_serial.fetch_add(1);
    for (int u = 0; u < N; ++u)
        for (int v = u + 1; v < N; ++v) {
            double x = J[(size_t)u * N + v];
            if (x == 0.0) continue;
            BondDev bd;
            bd.u = u;
            bd.v = v;
            bd.mJ4 = -0.25 * x;
            bd.mJ2 = -0.5 * x;
            c->host.push_back(bd);
            c->diag_shift += bd.mJ4;
        }
    c->nb = (int)c->host.size();
    if (c->nb > 0) {
        HM_HIP(hipMalloc(&c->dev, c->host.size() * sizeof(BondDev)));
        HM_HIP(hipMemcpy(c->dev, c->host.data(), c->host.size() * sizeof(BondDev),
                         hipMemcpyHostToDevice));
    }
    while (b->couplings.size() >= kCouplingCacheEntries) b->couplings.pop_back();
    b->couplings.emplace_front(std::move(key), c);
    *out = std::move(c);
    return HM_OK;
}

}  // namespace hm

using hm::fail;

extern "C" {

const char *hm_last_error(void) { return hm::g_error.c_str(); }

const char *hm_version(void) { return "hm 0.1 (gfx950)"; }

int hm_count(int32_t n, int32_t two_s, int32_t A, int64_t *out) {
    hm::clear_error();
    if (!out) return fail(HM_EINVAL, "out is null");
    if (n < 0 || two_s < 1) return fail(HM_EINVAL, "need n >= 0 and two_s >= 1");
    if (A < 0 || A > n * two_s) {
        *out = 0;
        return HM_OK;
    }
    std::vector<int64_t> D;
    hm::build_counts(n, two_s, D);
    int64_t v = D[(size_t)n * (n * two_s + 1) + A];
    if (v == std::numeric_limits<int64_t>::max())
        return fail(HM_ERANGE, "D(%d, %d) does not fit int64", n, A);
    *out = v;
    return HM_OK;
}

int hm_basis_init(int32_t N, int32_t two_s, int32_t two_M, hm_basis *out) {
    hm::clear_error();
    if (!out) return fail(HM_EINVAL, "out is null");
    *out = nullptr;
    if (N < 1 || two_s < 1) return fail(HM_EINVAL, "need N >= 1 and two_s >= 1");
    if (N > 64 || two_s > 255) return fail(HM_ERANGE, "N <= 64 and two_s <= 255 supported");
    const int64_t twoA = (int64_t)N * two_s - two_M;
    if (twoA % 2 != 0) return fail(HM_EINVAL, "N*two_s - two_M must be even");
    const int64_t A = twoA / 2;
    if (A < 0 || A > (int64_t)N * two_s)
        return fail(HM_EINVAL, "|M| exceeds N s (A = %lld)", (long long)A);
    const int bits = hm::bits_for(two_s);
    if (N * bits > 64)
        return fail(HM_ERANGE, "N * bits_per_digit = %d exceeds 64", N * bits);

    auto h = new (std::nothrow) hm_basis_s;
    if (!h) return fail(HM_ENOMEM, "out of host memory");
    hm::Basis &b = h->impl;
    b.N = N;
    b.two_s = two_s;
    b.A = (int)A;
    b.bits = bits;
    hm::build_counts(N, two_s, b.D);
    // every entry a valid state can touch is D(n, a) with n <= N, a <= A
    for (int n = 0; n <= N; ++n)
        for (int a = 0; a <= b.A && a <= n * two_s; ++a)
            if (b.count(n, a) == std::numeric_limits<int64_t>::max()) {
                delete h;
                return fail(HM_ERANGE, "count table overflows int64");
            }
    b.dim = b.count(N, b.A);
    if (b.dim >= ((int64_t)1 << 62)) {
        delete h;
        return fail(HM_ERANGE, "dimension %lld too large", (long long)b.dim);
    }
    b.idx32 = b.dim < ((int64_t)1 << 32);
    const int W = two_s + 1;
    b.prefix.assign(b.prefix_len(), 0);
    for (int k = 1; k <= N; ++k)
        for (int Ak = 0; Ak <= b.A; ++Ak) {
            int64_t run = 0;
            for (int a = 0; a <= two_s; ++a) {
                b.prefix[((size_t)(k - 1) * (b.A + 1) + Ak) * W + a] = run;
                int64_t d = b.count(k - 1, Ak - a);
                run = (run > std::numeric_limits<int64_t>::max() - d)
                          ? std::numeric_limits<int64_t>::max() : run + d;
            }
        }
    b.ladder.assign(two_s + 2, 0.0);
    for (int a = 1; a <= two_s; ++a)
        b.ladder[a] = std::sqrt((double)a * (double)(two_s - a + 1));
    *out = h;
    return HM_OK;
}

int hm_basis_cached_couplings(hm_basis h, int32_t *count) {
    hm::clear_error();
    if (!h || !count) return fail(HM_EINVAL, "null argument");
    std::lock_guard<std::mutex> lock(h->impl.mu);
    *count = (int32_t)h->impl.couplings.size();
    return HM_OK;
}

int hm_basis_free(hm_basis h) {
    hm::clear_error();
    delete h;
    return HM_OK;
}

int hm_basis_dim(hm_basis h, int64_t *dim) {
    hm::clear_error();
    if (!h || !dim) return fail(HM_EINVAL, "null argument");
    *dim = h->impl.dim;
    return HM_OK;
}

int hm_basis_info(hm_basis h, int32_t *N, int32_t *two_s, int32_t *A,
                  int32_t *bits_per_digit) {
    hm::clear_error();
    if (!h) return fail(HM_EINVAL, "null handle");
    if (N) *N = h->impl.N;
    if (two_s) *two_s = h->impl.two_s;
    if (A) *A = h->impl.A;
    if (bits_per_digit) *bits_per_digit = h->impl.bits;
    return HM_OK;
}

int hm_basis_set_schedule(hm_basis h, int32_t low_bits, int32_t block_threads,
                          int32_t rows_per_lane) {
    hm::clear_error();
    if (!h) return fail(HM_EINVAL, "null handle");
    hm::Basis &b = h->impl;
    std::lock_guard<std::mutex> lock(b.mu);
    if (b.half_tables) return fail(HM_EINVAL, "schedule must be set before the first device use");
    if (low_bits != 0 && (low_bits < 1 || low_bits > 14 || low_bits > b.N || b.N - low_bits > 24))
        return fail(HM_EINVAL, "low_bits %d outside 1..min(14, N) with N - low_bits <= 24",
                    low_bits);
    if (block_threads != 0 && block_threads != 64 && block_threads != 128 && block_threads != 256)
        return fail(HM_EINVAL, "block_threads must be 64, 128 or 256");
    if (rows_per_lane != 0 && rows_per_lane != 1 && rows_per_lane != 2 && rows_per_lane != 4 &&
        rows_per_lane != 8)
        return fail(HM_EINVAL, "rows_per_lane must be 1, 2, 4 or 8");
    b.half_K = low_bits;
    b.half_block = block_threads;
    b.half_R = rows_per_lane;
    return HM_OK;
}

int hm_basis_set_items_per_wave(hm_basis h, int32_t items_per_wave) {
    hm::clear_error();
    if (!h) return fail(HM_EINVAL, "null handle");
    hm::Basis &b = h->impl;
    std::lock_guard<std::mutex> lock(b.mu);
    if (b.half_tables)
        return fail(HM_EINVAL, "items per wave must be set before the first device use");
    if (items_per_wave < 0 || items_per_wave > (1 << 16))
        return fail(HM_EINVAL, "items per wave %d outside 0..65536", items_per_wave);
    b.half_ipw = items_per_wave;
    return HM_OK;
}

int hm_basis_set_staging(hm_basis h, int32_t mode) {
    hm::clear_error();
    if (!h) return fail(HM_EINVAL, "null handle");
    hm::Basis &b = h->impl;
    std::lock_guard<std::mutex> lock(b.mu);
    if (b.half_tables) return fail(HM_EINVAL, "staging must be set before the first device use");
    if (mode < 0 || mode > 2) return fail(HM_EINVAL, "staging mode %d outside 0..2", mode);
    b.half_staging = mode;
    return HM_OK;
}

int hm_unrank(hm_basis h, int64_t i, uint8_t *digits) {
    hm::clear_error();
    if (!h || !digits) return fail(HM_EINVAL, "null argument");
    if (i < 0 || i >= h->impl.dim)
        return fail(HM_EINVAL, "index %lld outside [0, %lld)", (long long)i,
                    (long long)h->impl.dim);
    hm::host_unrank(&h->impl, i, digits);
    return HM_OK;
}

int hm_rank(hm_basis h, const uint8_t *digits, int64_t *i) {
    hm::clear_error();
    if (!h || !digits || !i) return fail(HM_EINVAL, "null argument");
    int sum = 0;
    for (int u = 0; u < h->impl.N; ++u) {
        if (digits[u] > h->impl.two_s)
            return fail(HM_EINVAL, "digit %d at site %d exceeds 2s = %d", digits[u], u,
                        h->impl.two_s);
        sum += digits[u];
    }
    if (sum != h->impl.A)
        return fail(HM_EINVAL, "digit sum %d differs from A = %d", sum, h->impl.A);
    *i = hm::host_rank(&h->impl, digits);
    return HM_OK;
}

}  // extern "C"
