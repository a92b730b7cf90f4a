// Device helpers shared by the HIP kernels: packed digit access, decoding
// (Sec. 3.1) and encoding (Sec. 3.2) through the prefix table, index deltas
// of a two-site move, deterministic wave64/workgroup reductions and the
// XCD-aware mapping of workgroups to contiguous row ranges.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hm {

constexpr int kBlock = 256;          // threads per workgroup of the row kernels
constexpr int kMaxGrid = 2048;       // workgroups of the row kernels (8 per CU)
constexpr int kXcds = 8;             // MI355X: 8 XCDs with one L2 each

// Workgroup b runs on XCD b % 8 (round-robin dispatch).  Give the workgroups
// of one XCD consecutive logical ids, so each XCD sweeps one contiguous slice
// of the rows and its L2 sees the neighbouring gathers.
__device__ __forceinline__ int xcd_logical_block(int b, int grid) {
    if (grid % kXcds != 0) return b;
    return (b % kXcds) * (grid / kXcds) + b / kXcds;
}

// Rows [first, last) of logical workgroup lb when `dim` rows are split into
// `grid` contiguous ranges.
template <typename I>
__device__ __forceinline__ void block_rows(int lb, int grid, I dim, I &first, I &last) {
    const uint64_t d = (uint64_t)dim;
    first = (I)(d * (uint64_t)lb / (uint64_t)grid);
    last = (I)(d * (uint64_t)(lb + 1) / (uint64_t)grid);
}

template <int B>
__device__ __forceinline__ int digit_at(uint64_t st, int u) {
    return (int)((st >> (u * B)) & ((1u << B) - 1u));
}

// Sum of the digits of sites 0..u (inclusive), by B popcounts.
template <int B>
__device__ __forceinline__ int digit_sum_upto(uint64_t st, int u) {
    const int nbits = (u + 1) * B;
    const uint64_t mask = nbits >= 64 ? ~0ull : ((1ull << nbits) - 1ull);
    if constexpr (B == 1) {
        return __popcll(st & mask);
    } else {
        // bit 0 of every B-bit field
        uint64_t low = 0;
#pragma unroll
        for (int f = 0; f < 64 / B; ++f) low |= 1ull << (f * B);
        int s = 0;
#pragma unroll
        for (int j = 0; j < B; ++j) s += __popcll((st >> j) & low & mask) << j;
        return s;
    }
}

// Prefix table view: P[k][Ak][a] at ((k-1)*(A+1) + Ak)*(two_s+1) + a.
template <typename I>
struct Prefix {
    const I *p;
    int A1;   // A + 1
    int W;    // two_s + 1
    __device__ __forceinline__ I at(int k, int Ak, int a) const {
        return p[((k - 1) * A1 + Ak) * W + a];
    }
};

// Decoding (Sec. 3.1): walk k = N..1; the digit at site k is the number of
// block offsets P[k][Ak][t], t = 1..2s, that do not exceed the remaining
// offset (empty blocks share their offset with the next one, so the count
// lands on the non-empty block that holds the offset).
template <typename I, int B>
__device__ __forceinline__ uint64_t unrank_state(I r, const Prefix<I> &P, int N, int A,
                                                  int two_s) {
    uint64_t st = 0;
    int Ak = A;
    for (int k = N; k >= 1; --k) {
        const I *row = P.p + ((k - 1) * P.A1 + Ak) * P.W;
        int a;
        if constexpr (B == 1) {
            a = row[1] <= r ? 1 : 0;
        } else {
            a = 0;
            for (int t = 1; t <= two_s; ++t) a += row[t] <= r ? 1 : 0;
        }
        r -= row[a];
        Ak -= a;
        st |= (uint64_t)a << ((k - 1) * B);
    }
    return st;
}

// Encoding (Sec. 3.2): index = sum_k P[k][A_k][a_k], A_k = digit sum of sites 1..k.
template <typename I, int B>
__device__ __forceinline__ I rank_state(uint64_t st, const Prefix<I> &P, int N, int A) {
    I idx = 0;
    int Ak = A;
    for (int k = N; k >= 1; --k) {
        const int a = digit_at<B>(st, k - 1);
        idx += P.at(k, Ak, a);
        Ak -= a;
    }
    return idx;
}

// Index change when site u (< v) gains du (= +1 or -1) and site v loses du.
// Only the terms of sites u..v of the encoding sum change: at sites strictly
// between, the partial digit sum A_p shifts by du; at v it is unchanged.
template <typename I, int B>
__device__ __forceinline__ I move_delta(uint64_t st, int u, int v, int du,
                                        const Prefix<I> &P) {
    int Ap = digit_sum_upto<B>(st, u);
    const int au = digit_at<B>(st, u);
    I delta = P.at(u + 1, Ap + du, au + du) - P.at(u + 1, Ap, au);
    for (int p = u + 1; p < v; ++p) {
        const int ap = digit_at<B>(st, p);
        Ap += ap;
        delta += P.at(p + 1, Ap + du, ap) - P.at(p + 1, Ap, ap);
    }
    const int av = digit_at<B>(st, v);
    Ap += av;
    delta += P.at(v + 1, Ap, av - du) - P.at(v + 1, Ap, av);
    return delta;
}

// Wave64 sum in a fixed butterfly order (bitwise reproducible).
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Workgroup sum (blockDim.x multiple of 64, <= 1024); result valid in thread 0.
__device__ __forceinline__ double block_sum(double x, double *lds /* >= 16 */) {
    x = wave_sum(x);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = x;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        for (int w = 0; w < nw; ++w) s += lds[w];
    }
    __syncthreads();
    return s;
}

}  // namespace hm
