// HIP kernels for gfx950: CSC validation, matching set-up, the bulk-synchronous
// 4-cycle rounds (arXiv 1801.09809, Section 5.3) and the fixed-order total.
//
// Data layout in HBM: the caller's CSC (col_ptr int64, row_idx int32, w f64)
// is read in place; per-vertex state (mates, matched weights, the Step-C
// winner of every root column, the Step-D slots) lives in the caller's
// workspace as structure-of-arrays, so every per-column pass is a coalesced
// stream and every per-row access is a 4- or 8-byte gather.
#include <float.h>
#include <math.h>

#include "hwpm_internal.h"

namespace hwpm {

// ---------------------------------------------------------------------------
// helpers

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

// Winner order of Step C: larger gain first, then smaller row.
struct Cand {
    double g;     // 0.0 = none (candidates have g > 0)
    int32_t i;    // INT32_MAX = none
    int32_t c;
    int64_t k;
    int64_t p;
};

__device__ __forceinline__ bool better(double g1, int32_t i1, double g2, int32_t i2) {
    return g1 > g2 || (g1 == g2 && i1 < i2);
}

// Record the Step-C winner of root j (or its absence) and start Step D:
// raise the max-gain slot of the other column c.
__device__ __forceinline__ void publish(const Work& W, int32_t j, const Cand& b, int slot) {
    if (b.i == INT32_MAX) {
        W.best_i[j] = -1;
        return;
    }
    W.best_i[j] = b.i;
    W.best_g[j] = b.g;
    W.best_c[j] = b.c;
    W.best_k[j] = b.k;
    W.best_p[j] = b.p;
    const unsigned long long gb = gain_bits(b.g);
    if (__hip_atomic_load(&W.dgain[b.c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gb)
        atomicMax(&W.dgain[b.c], gb);
    const int32_t q = atomicAdd(&W.counters[kRoundBase + 2 * slot], 1);
    W.cand[q] = j;
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
    const double g = (A.w[k] + A.w[p]) - (W.wm[mi] + wmj);
    if (g > 0.0 && better(g, i, b.g, b.i)) {
        b.g = g;
        b.i = i;
        b.c = mi;
        b.k = k;
        b.p = p;
    }
}

template <int WIDTH>
__device__ __forceinline__ void reduce_best(Cand& b) {
#pragma unroll
    for (int off = WIDTH / 2; off >= 1; off >>= 1) {
        const double og = __shfl_xor(b.g, off, WIDTH);
        const int32_t oi = __shfl_xor(b.i, off, WIDTH);
        const int32_t oc = __shfl_xor(b.c, off, WIDTH);
        const int64_t ok = __shfl_xor(b.k, off, WIDTH);
        const int64_t op = __shfl_xor(b.p, off, WIDTH);
        if (better(og, oi, b.g, b.i)) {
            b.g = og;
            b.i = oi;
            b.c = oc;
            b.k = ok;
            b.p = op;
        }
    }
}

// ---------------------------------------------------------------------------
// CSC validation

__global__ void k_check_cols(int32_t n, int64_t nnz, const int64_t* __restrict__ col_ptr,
                             uint32_t* __restrict__ bitmap, int32_t* __restrict__ counters) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j <= n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = col_ptr[j];
        int flags = 0;
        if (v < 0 || v > nnz) {
            flags |= 1;
        } else {
            atomicOr(&bitmap[v >> 5], 1u << (v & 31));
        }
        if (j < n && col_ptr[j + 1] < v) flags |= 1;
        if (j == 0 && v != 0) flags |= 1;
        if (j == n && v != nnz) flags |= 1;
        if (flags) atomicOr(&counters[kErrCsc], flags);
    }
}

__global__ void k_check_entries(int32_t n, int64_t nnz, const int32_t* __restrict__ row_idx,
                                const double* __restrict__ w, const uint32_t* __restrict__ bitmap,
                                int32_t* __restrict__ counters) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = row_idx[k];
        int flags = 0;
        if (r < 0 || r >= n) flags |= 2;
        if (!isfinite(w[k])) flags |= 8;
        const bool col_start = (bitmap[k >> 5] >> (k & 31)) & 1u;
        if (k > 0 && !col_start && !(row_idx[k - 1] < r)) flags |= 4;
        if (flags) atomicOr(&counters[kErrCsc], flags);
    }
}

hipError_t launch_check_csc(const Csc& A, const Work& W, hipStream_t s, int cus) {
    const int blocks = cus * 8;
    hipLaunchKernelGGL(k_check_cols, dim3(blocks), dim3(256), 0, s, A.n, A.nnz, A.col_ptr,
                       W.bitmap, W.counters);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (A.nnz > 0) {
        hipLaunchKernelGGL(k_check_entries, dim3(blocks), dim3(256), 0, s, A.n, A.nnz, A.row_idx,
                           A.w, W.bitmap, W.counters);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Set-up: replicate the mates and matched weights (the initial broadcast of
// Algorithm 2), validate the matching, list the long columns.

__global__ void k_init_match(Csc A, Work W, const int32_t* __restrict__ mate_in,
                             int32_t long_threshold) {
    for (int64_t jj = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; jj < A.n;
         jj += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = (int32_t)jj;
        W.dgain[j] = 0ull;
        W.droot[j] = kNoRoot;
        const int64_t lo = A.col_ptr[j], hi = A.col_ptr[j + 1];
        if (hi - lo > long_threshold) {
            const int32_t q = atomicAdd(&W.counters[kNumLong], 1);
            W.long_list[q] = j;
        }
        const int32_t r = mate_in[j];
        if (r < 0 || r >= A.n) {
            atomicOr(&W.counters[kErrMatch], 1);
            continue;
        }
        if (atomicCAS(&W.mr[r], -1, j) != -1) atomicOr(&W.counters[kErrMatch], 2);
        W.mc[j] = r;
        const int64_t p = find_row(A.col_ptr, A.row_idx, j, r);
        if (p < 0) {
            atomicOr(&W.counters[kErrMatch], 4);
            W.wm[j] = 0.0;
        } else {
            W.wm[j] = A.w[p];
        }
    }
}

hipError_t launch_init_match(const Csc& A, const Work& W, const int32_t* mate_in,
                             int32_t long_threshold, hipStream_t s) {
    const int64_t blocks = ((int64_t)A.n + 255) / 256;
    hipLaunchKernelGGL(k_init_match, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256),
                       0, s, A, W, mate_in, long_threshold);
    return hipGetLastError();
}

// Chunk table of the long columns: chunk_off[q] = number of kLongChunk-entry
// chunks in long columns 0..q-1.  One block, sequential over 1024 segments.
__global__ __launch_bounds__(1024) void k_long_chunks(Work W, Csc A) {
    __shared__ int64_t seg[1024];
    const int32_t nl = W.counters[kNumLong];
    const int t = threadIdx.x;
    const int64_t per = ((int64_t)nl + 1023) / 1024;
    const int64_t b = t * per, e = (b + per < nl) ? b + per : nl;
    int64_t sum = 0;
    for (int64_t q = b; q < e; ++q) {
        const int32_t j = W.long_list[q];
        const int64_t len = A.col_ptr[j + 1] - A.col_ptr[j];
        sum += (len + kLongChunk - 1) / kLongChunk;
    }
    seg[t] = sum;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int u = 0; u < 1024; ++u) {
            const int64_t v = seg[u];
            seg[u] = run;
            run += v;
        }
        W.counters[kNumChunks] = (int32_t)run;
        W.chunk_off[nl] = run;
    }
    __syncthreads();
    int64_t run = seg[t];
    for (int64_t q = b; q < e; ++q) {
        W.chunk_off[q] = run;
        const int32_t j = W.long_list[q];
        const int64_t len = A.col_ptr[j + 1] - A.col_ptr[j];
        run += (len + kLongChunk - 1) / kLongChunk;
    }
}

hipError_t launch_long_chunks(const Work& W, const Csc& A, hipStream_t s) {
    hipLaunchKernelGGL(k_long_chunks, dim3(1), dim3(1024), 0, s, W, A);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Steps A-C.  Short columns: a tile of T lanes per root column, lanes stride
// over the column (coalesced row_idx reads), each probes its own closing
// edge, the tile reduces to the Step-C winner with cross-lane shuffles.

template <int T>
__global__ __launch_bounds__(256) void k_search_short(Csc A, Work W, int32_t long_threshold,
                                                      int slot) {
    const int lane = threadIdx.x & (T - 1);
    const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / T;
    if (tile >= A.n) return;  // tile-uniform
    const int32_t j = (int32_t)tile;
    const int64_t lo = A.col_ptr[j], hi = A.col_ptr[j + 1];
    if (hi - lo > long_threshold) return;  // split kernel handles it
    const int32_t mj = W.mc[j];
    const double wmj = W.wm[j];
    Cand b{0.0, INT32_MAX, -1, -1, -1};
    for (int64_t k = lo + lane; k < hi; k += T) try_entry(A, W, k, mj, wmj, b);
    reduce_best<T>(b);
    if (lane == 0) publish(W, j, b, slot);
}

// Long columns: each block takes kLongChunk entries of one column and writes
// a partial winner; k_merge_long reduces the partials of each column.
__global__ __launch_bounds__(256) void k_search_long(Csc A, Work W) {
    __shared__ double sg[4];
    __shared__ int32_t si[4], sc[4];
    __shared__ int64_t sk[4], sp[4];
    const int32_t nl = W.counters[kNumLong];
    const int32_t total = W.counters[kNumChunks];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int32_t cid = blockIdx.x; cid < total; cid += gridDim.x) {
        // q = last long column whose first chunk is <= cid
        int32_t a = 0, z = nl;  // chunk_off[a] <= cid < chunk_off[z]
        while (z - a > 1) {
            const int32_t m = (a + z) >> 1;
            if (W.chunk_off[m] <= cid) a = m; else z = m;
        }
        const int32_t j = W.long_list[a];
        const int64_t c0 = A.col_ptr[j];
        const int64_t lo = c0 + (int64_t)(cid - W.chunk_off[a]) * kLongChunk;
        const int64_t hi0 = A.col_ptr[j + 1];
        const int64_t hi = (lo + kLongChunk < hi0) ? lo + kLongChunk : hi0;
        const int32_t mj = W.mc[j];
        const double wmj = W.wm[j];
        Cand b{0.0, INT32_MAX, -1, -1, -1};
        for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) try_entry(A, W, k, mj, wmj, b);
        reduce_best<64>(b);
        if (lane == 0) {
            sg[wave] = b.g; si[wave] = b.i; sc[wave] = b.c; sk[wave] = b.k; sp[wave] = b.p;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int u = 1; u < 4; ++u) {
                if (better(sg[u], si[u], b.g, b.i)) {
                    b.g = sg[u]; b.i = si[u]; b.c = sc[u]; b.k = sk[u]; b.p = sp[u];
                }
            }
            W.part_g[cid] = b.g; W.part_i[cid] = b.i; W.part_c[cid] = b.c;
            W.part_k[cid] = b.k; W.part_p[cid] = b.p;
        }
        __syncthreads();
    }
}

__global__ void k_merge_long(Work W, int slot) {
    const int32_t nl = W.counters[kNumLong];
    for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nl; q += gridDim.x * blockDim.x) {
        Cand b{0.0, INT32_MAX, -1, -1, -1};
        for (int64_t cid = W.chunk_off[q]; cid < W.chunk_off[q + 1]; ++cid) {
            if (better(W.part_g[cid], W.part_i[cid], b.g, b.i)) {
                b.g = W.part_g[cid]; b.i = W.part_i[cid]; b.c = W.part_c[cid];
                b.k = W.part_k[cid]; b.p = W.part_p[cid];
            }
        }
        publish(W, W.long_list[q], b, slot);
    }
}

hipError_t launch_search(const Csc& A, const Work& W, int tile_width, int32_t long_threshold,
                         int slot, bool has_long, hipStream_t s, int cus) {
    const int64_t threads = (int64_t)A.n * tile_width;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    switch (tile_width) {
        case 4: hipLaunchKernelGGL(k_search_short<4>, dim3(blocks), dim3(256), 0, s, A, W, long_threshold, slot); break;
        case 8: hipLaunchKernelGGL(k_search_short<8>, dim3(blocks), dim3(256), 0, s, A, W, long_threshold, slot); break;
        case 16: hipLaunchKernelGGL(k_search_short<16>, dim3(blocks), dim3(256), 0, s, A, W, long_threshold, slot); break;
        case 32: hipLaunchKernelGGL(k_search_short<32>, dim3(blocks), dim3(256), 0, s, A, W, long_threshold, slot); break;
        case 64: hipLaunchKernelGGL(k_search_short<64>, dim3(blocks), dim3(256), 0, s, A, W, long_threshold, slot); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !has_long) return e;
    hipLaunchKernelGGL(k_search_long, dim3(cus * 8), dim3(256), 0, s, A, W);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_merge_long, dim3(64), dim3(256), 0, s, W, slot);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step D.  Pass 1 (the atomicMax of the gain bits) ran in publish(); pass 2
// picks the smallest root among the roots that reached the maximum.  A column
// that kept a cycle of its own accepts nothing.

__global__ void k_resolve(Work W, int slot) {
    const int32_t nc = W.counters[kRoundBase + 2 * slot];
    for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nc; t += gridDim.x * blockDim.x) {
        const int32_t j = W.cand[t];
        const int32_t c = W.best_c[j];
        if (W.best_i[c] >= 0) continue;
        if (W.dgain[c] == gain_bits(W.best_g[j])) atomicMin(&W.droot[c], j);
    }
}

hipError_t launch_resolve(const Work& W, int slot, hipStream_t s, int cus) {
    hipLaunchKernelGGL(k_resolve, dim3(cus * 2), dim3(256), 0, s, W, slot);
    return hipGetLastError();
}

// Flip every accepted cycle: m_j = i, m_i = j, m_c = l, m_l = c with l the old
// m_j (Algorithm 6).  Accepted cycles are vertex-disjoint, so the writes never
// collide.  The Step-D slots touched this round are cleared for the next one:
// a root clears its own column (nobody reads it: its column accepts nothing),
// the winner at column c clears c (the losers at c only compare the slot with
// their own index, which neither the old nor the cleared value equals).
__global__ void k_apply(Csc A, Work W, int slot) {
    const int32_t nc = W.counters[kRoundBase + 2 * slot];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int next = (slot + 1) % kSlots;
        W.counters[kRoundBase + 2 * next] = 0;
        W.counters[kRoundBase + 2 * next + 1] = 0;
    }
    int applied = 0;
    for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nc; t += gridDim.x * blockDim.x) {
        const int32_t j = W.cand[t];
        const int32_t c = W.best_c[j];
        W.dgain[j] = 0ull;
        W.droot[j] = kNoRoot;
        if (W.best_i[c] >= 0) continue;
        if (__hip_atomic_load(&W.droot[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != j) continue;
        const int32_t i = W.best_i[j];
        const int32_t l = W.mc[j];
        W.mc[j] = i;
        W.mr[i] = j;
        W.mc[c] = l;
        W.mr[l] = c;
        W.wm[j] = A.w[W.best_k[j]];
        W.wm[c] = A.w[W.best_p[j]];
        W.dgain[c] = 0ull;
        __hip_atomic_store(&W.droot[c], kNoRoot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ++applied;
    }
    if (applied) atomicAdd(&W.counters[kRoundBase + 2 * slot + 1], applied);
}

hipError_t launch_apply(const Csc& A, const Work& W, int slot, hipStream_t s, int cus) {
    hipLaunchKernelGGL(k_apply, dim3(cus * 2), dim3(256), 0, s, A, W, slot);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Total weight: a perfect binary tree over the values padded with +0.0 to a
// power of two, pairs (2t, 2t+1) at every level.  A block sums an aligned run
// of kTreeBlock = 2048 leaves (exactly one subtree); the block sums form the
// next level, and the last level (<= 2048 values) runs in one block over
// exactly next_pow2(m) leaves.

__global__ __launch_bounds__(256) void k_tree_block(const double* __restrict__ x, int64_t m,
                                                    double* __restrict__ out) {
    __shared__ double part[4];
    const int64_t base = (int64_t)blockIdx.x * kTreeBlock + threadIdx.x * 8;
    double v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (base + e < m) ? x[base + e] : 0.0;
    double s = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_down(s, off, 64);
        if ((lane & (2 * off - 1)) == 0) s = s + o;
    }
    if (lane == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (part[0] + part[1]) + (part[2] + part[3]);
}

__global__ __launch_bounds__(1024) void k_tree_final(const double* __restrict__ x, int64_t m,
                                                     double* __restrict__ out) {
    __shared__ double a[kTreeBlock], b[kTreeBlock];
    int64_t size = 1;
    while (size < m) size <<= 1;
    for (int64_t t = threadIdx.x; t < size; t += blockDim.x) a[t] = (t < m) ? x[t] : 0.0;
    __syncthreads();
    double* src = a;
    double* dst = b;
    for (int64_t len = size; len > 1; len >>= 1) {
        for (int64_t t = threadIdx.x; t < len / 2; t += blockDim.x) dst[t] = src[2 * t] + src[2 * t + 1];
        __syncthreads();
        double* tmp = src; src = dst; dst = tmp;
    }
    if (threadIdx.x == 0) out[0] = (m > 0) ? src[0] : 0.0;
}

hipError_t launch_tree_sum(const double* x, int64_t m, const Work& W, double* out, hipStream_t s) {
    const double* cur = x;
    double* bufs[2] = {W.tree_a, W.tree_b};
    int which = 0;
    while (m > kTreeBlock) {
        const int64_t blocks = (m + kTreeBlock - 1) / kTreeBlock;
        hipLaunchKernelGGL(k_tree_block, dim3((unsigned)blocks), dim3(256), 0, s, cur, m, bufs[which]);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        cur = bufs[which];
        which ^= 1;
        m = blocks;
    }
    hipLaunchKernelGGL(k_tree_final, dim3(1), dim3(1024), 0, s, cur, m, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Workspace layout (256-byte aligned sub-arrays).

static inline size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

size_t workspace_layout(int32_t n, int64_t nnz, char* base, Work* out) {
    const size_t N = (size_t)(n > 0 ? n : 0);
    const size_t Z = (size_t)(nnz > 0 ? nnz : 0);
    const size_t max_chunks = Z / kLongChunk + N + 1;
    const size_t tree1 = N / kTreeBlock + 2;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    Work W;
    W.mr = (int32_t*)take(N * 4);
    W.mc = (int32_t*)take(N * 4);
    W.wm = (double*)take(N * 8);
    W.best_g = (double*)take(N * 8);
    W.best_i = (int32_t*)take(N * 4);
    W.best_c = (int32_t*)take(N * 4);
    W.best_k = (int64_t*)take(N * 8);
    W.best_p = (int64_t*)take(N * 8);
    W.dgain = (unsigned long long*)take(N * 8);
    W.droot = (int32_t*)take(N * 4);
    W.cand = (int32_t*)take(N * 4);
    W.long_list = (int32_t*)take(N * 4);
    W.chunk_off = (int64_t*)take((N + 1) * 8);
    W.part_g = (double*)take(max_chunks * 8);
    W.part_i = (int32_t*)take(max_chunks * 4);
    W.part_c = (int32_t*)take(max_chunks * 4);
    W.part_k = (int64_t*)take(max_chunks * 8);
    W.part_p = (int64_t*)take(max_chunks * 8);
    W.tree_a = (double*)take(tree1 * 8);
    W.tree_b = (double*)take(tree1 * 8);
    W.bitmap = (uint32_t*)take((Z + 1) / 32 * 4 + 8);
    W.counters = (int32_t*)take(kCounterWords * 4);
    W.result = (double*)take(4 * 8);
    W.max_chunks = (int64_t)max_chunks;
    if (out) *out = W;
    return off;
}

}  // namespace hwpm
