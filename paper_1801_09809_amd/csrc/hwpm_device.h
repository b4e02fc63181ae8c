// Device helpers shared by the search and round kernels: the closing-edge
// probe by binary search, the Step-C winner record and its order, the
// cross-lane winner reduction and the LDS hash sets (hwpm_hash.h).
#pragma once

#include "hwpm_internal.h"

#define HWPM_HD __device__ __forceinline__
#include "hwpm_hash.h"

namespace hwpm {

// Round kernels launched after the round that ended the loop do nothing.
__device__ __forceinline__ bool round_over(const Work& W) { return W.counters[kDone] != 0; }

__device__ __forceinline__ unsigned long long gain_bits(double g) {
    // g > 0 (finite or +inf): the IEEE bit pattern orders like the value.
    return (unsigned long long)__double_as_longlong(g);
}

// Position of row r in column c, or -1 when the entry {r, c} is absent.
// Binary search down to a window of at most 9 positions, then an unrolled
// scan whose loads are independent (one memory round trip for short columns).
__device__ __forceinline__ int64_t find_row(const int64_t* __restrict__ col_ptr,
                                            const int32_t* __restrict__ row_idx, int32_t c,
                                            int32_t r) {
    int64_t lo = col_ptr[c];
    const int64_t end = col_ptr[c + 1];
    int64_t len = end - lo;
    while (len > 8) {
        const int64_t half = len >> 1;
        if (row_idx[lo + half] < r) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    // the first row >= r lies in [lo, lo + len]
    int64_t hit = -1;
#pragma unroll
    for (int q = 0; q <= 8; ++q) {
        const int64_t pos = lo + q;
        if (q <= len && pos < end && row_idx[pos] == r) hit = pos;
    }
    return hit;
}

// Four probes at once: out[q] = position of row r[q] in column c[q], or -1
// (also for c[q] < 0).  The same search as find_row, with the four searches
// advanced in lockstep so that their loads are independent: one memory round
// trip per step for all four instead of one per step for each.
__device__ __forceinline__ void find_row_x4(const int64_t* __restrict__ col_ptr,
                                            const int32_t* __restrict__ row_idx, const int32_t* c,
                                            const int32_t* r, int64_t* out) {
    int64_t lo[4], end[4], len[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        lo[q] = (c[q] >= 0) ? col_ptr[c[q]] : 0;
        end[q] = (c[q] >= 0) ? col_ptr[c[q] + 1] : 0;
        len[q] = end[q] - lo[q];
    }
    for (;;) {
        bool any = false;
        int32_t v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool go = len[q] > 8;
            any |= go;
            v[q] = go ? row_idx[lo[q] + (len[q] >> 1)] : 0;
        }
        if (!any) break;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (len[q] > 8) {
                const int64_t half = len[q] >> 1;
                if (v[q] < r[q]) {
                    lo[q] += half + 1;
                    len[q] -= half + 1;
                } else {
                    len[q] = half;
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int64_t hit = -1;
#pragma unroll
        for (int x = 0; x <= 8; ++x) {
            const int64_t pos = lo[q] + x;
            if (x <= len[q] && pos < end[q] && row_idx[pos] == r[q]) hit = pos;
        }
        out[q] = hit;
    }
}

// Winner order of Step C: larger gain first, then smaller row i.  Every
// candidate of one root lies in the root's own column j, whose rows increase
// with the CSC position, so the smaller row is the smaller position k: the
// search keys candidates by k and reads the row of the winner only.
struct Cand {
    double g;     // 0.0 = none (candidates have g > 0)
    int64_t k;    // position of {i, j}; INT64_MAX = none
    int32_t c;    // other column c = m_i
    int64_t p;    // position of {m_j, m_i}
};

constexpr int64_t kNoPos = INT64_MAX;

__device__ __forceinline__ bool better(double g1, int64_t k1, double g2, int64_t k2) {
    return g1 > g2 || (g1 == g2 && k1 < k2);
}

// Record the Step-C winner of root j (or its absence).
__device__ __forceinline__ void publish(const Csc& A, const Work& W, int32_t j, const Cand& b) {
    if (b.k == kNoPos) {
        W.best_i[j] = -1;
        return;
    }
    W.best_i[j] = A.row_idx[b.k];
    W.best_g[j] = b.g;
    W.best_c[j] = b.c;
    W.best_k[j] = b.k;
    W.best_p[j] = b.p;
}

// Fold a candidate into the running winner.
__device__ __forceinline__ void offer(Cand& b, double g, int64_t k, int32_t c, int64_t p) {
    if (g > 0.0 && better(g, k, b.g, b.k)) {
        b.g = g;
        b.k = k;
        b.c = c;
        b.p = p;
    }
}

// One entry {i, j} of root column j (mate row mj, matched weight wmj):
// Steps A and B for the cycle (i, j, m_j, m_i), folded into the running best.
__device__ __forceinline__ void try_entry(const Csc& A, const Work& W, int64_t k, int32_t mj,
                                          double wmj, Cand& b) {
    const int32_t i = A.row_idx[k];
    if (i <= mj) return;                    // rows i > m_j only
    const int32_t mi = W.mr[i];
    const int64_t p = find_row(A.col_ptr, A.row_idx, mi, mj);  // edge {m_j, m_i}
    if (p < 0) return;
    offer(b, (A.w[k] + A.w[p]) - (W.wm[mi] + wmj), k, mi, p);
}

template <int WIDTH>
__device__ __forceinline__ void reduce_best(Cand& b) {
#pragma unroll
    for (int off = WIDTH / 2; off >= 1; off >>= 1) {
        const double og = __shfl_xor(b.g, off, WIDTH);
        const int64_t ok = __shfl_xor(b.k, off, WIDTH);
        const int32_t oc = __shfl_xor(b.c, off, WIDTH);
        const int64_t op = __shfl_xor(b.p, off, WIDTH);
        if (better(og, ok, b.g, b.k)) {
            b.g = og;
            b.k = ok;
            b.c = oc;
            b.p = op;
        }
    }
}

// Compare-and-swap on an LDS slot, for the hash sets of hwpm_hash.h.
struct LdsCas32 {
    __device__ __forceinline__ int32_t operator()(int32_t* p, int32_t expected, int32_t desired) const {
        return atomicCAS(p, expected, desired);
    }
};

// LDS writes of the wave are done and visible to its lanes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

}  // namespace hwpm
