// HIP kernels for the initial perfect matching of the HWPM pipeline
// (arXiv 1801.09809, Sections 5.1-5.2): a greedy maximal matching with the
// heavy-edge tie-break, then maximum-cardinality matching by multi-source BFS
// phases whose parent choice is the "max" semiring (heaviest edge).
//
// Both are bulk-synchronous.  Every choice is an argmax under a total order
// (weight descending, then index ascending), taken with two passes of integer
// atomics: pass 1 raises a monotone 64-bit key of the weight, pass 2 takes the
// smallest index among the entries that reached the maximum.  The result is
// therefore independent of scheduling, and equals the sequential definition.
#include <math.h>

#include "hwpm_internal.h"

namespace hwpm {

// Monotone unsigned key of a finite double (a < b  <=>  key(a) < key(b));
// -0.0 maps to the key of +0.0 so that the two compare equal, as doubles do.
__device__ __forceinline__ unsigned long long wkey(double w) {
    if (w == 0.0) w = 0.0;
    const unsigned long long u = (unsigned long long)__double_as_longlong(w);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// Greedy winner order per column: heavier first, then smaller row.
__device__ __forceinline__ bool g_better(bool heavy, double w1, int32_t r1, double w2, int32_t r2) {
    if (r2 == INT32_MAX) return r1 != INT32_MAX;
    if (r1 == INT32_MAX) return false;
    if (heavy && w1 != w2) return w1 > w2;
    return r1 < r2;
}

// Empty matching and clear row slots.
__global__ void k_mcm_init(Csc A, Mcm M) {
    for (int64_t jj = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; jj < A.n;
         jj += (int64_t)gridDim.x * blockDim.x) {
        M.mc[jj] = -1;
        M.mr[jj] = -1;
        M.rkey[jj] = 0ull;
        M.racc[jj] = kNoRoot;
    }
}

// Long-column list (columns the greedy step reads with a whole block).
__global__ void k_classify_long(Csc A, Work W, int32_t long_threshold) {
    for (int64_t jj = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; jj < A.n;
         jj += (int64_t)gridDim.x * blockDim.x) {
        const bool is_long = A.col_ptr[jj + 1] - A.col_ptr[jj] > long_threshold;
        const int32_t q = wave_append(&W.counters[kNumLong], is_long);
        if (is_long) W.long_list[q] = (int32_t)jj;
    }
}

hipError_t launch_mcm_init(const Csc& A, const Mcm& M, const Work& W, int32_t long_threshold,
                           hipStream_t s, int cus) {
    hipLaunchKernelGGL(k_mcm_init, dim3(cus * 8), dim3(256), 0, s, A, M);
    hipLaunchKernelGGL(k_classify_long, dim3(cus * 8), dim3(256), 0, s, A, W, long_threshold);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Greedy maximal matching: proposal rounds.

// Every unmatched column proposes to its best unmatched row; pass 1 of the
// rows' choice (largest weight key) is taken at once.
// Greedy rounds are queued several at a time: a round that finds no
// proposal raises kMcmDone and every greedy kernel queued after it returns.
__global__ void k_greedy_begin(Mcm M) {
    if (M.counters[kMcmDone]) return;
    if (threadIdx.x == 0) {
        M.counters[kMcmProposals] = 0;
        M.counters[kMcmListLen] = 0;
    }
}

__global__ void k_greedy_end(Mcm M) {
    if (M.counters[kMcmDone]) return;
    M.counters[kMcmRounds] += 1;
    if (M.counters[kMcmListLen] == 0) M.counters[kMcmDone] = 1;  // no proposal
}

template <int T>
__global__ __launch_bounds__(256) void k_greedy_propose(Csc A, Mcm M, int heavy, int32_t long_threshold) {
    if (M.counters[kMcmDone]) return;
    const int lane = threadIdx.x & (T - 1);
    const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / T;
    if (tile >= A.n) return;
    const int32_t j = (int32_t)tile;
    if (M.mc[j] >= 0) return;
    const int64_t lo = A.col_ptr[j], hi = A.col_ptr[j + 1];
    if (hi - lo > long_threshold) return;
    double bw = 0.0;
    int32_t br = INT32_MAX;
    for (int64_t k = lo + lane; k < hi; k += T) {
        const int32_t r = A.row_idx[k];
        if (M.mr[r] >= 0) continue;
        const double w = A.w[k];
        if (g_better(heavy, w, r, bw, br)) { bw = w; br = r; }
    }
#pragma unroll
    for (int off = T / 2; off >= 1; off >>= 1) {
        const double ow = __shfl_xor(bw, off, T);
        const int32_t orr = __shfl_xor(br, off, T);
        if (g_better(heavy, ow, orr, bw, br)) { bw = ow; br = orr; }
    }
    const bool propose = lane == 0 && br != INT32_MAX;
    const int32_t q = wave_append(&M.counters[kMcmListLen], propose);
    if (lane == 0) {
        M.prop_row[j] = br == INT32_MAX ? -1 : br;
        if (propose) {
            M.prop_w[j] = bw;
            if (heavy) atomicMax(&M.rkey[br], wkey(bw));
            M.list[q] = j;
        }
    }
}

// Long unmatched columns: one block per column.
__global__ __launch_bounds__(256) void k_greedy_propose_long(Csc A, Mcm M, const Work W, int heavy) {
    __shared__ double sw[4];
    __shared__ int32_t sr[4];
    if (M.counters[kMcmDone]) return;
    const int32_t nl = W.counters[kNumLong];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int32_t q = blockIdx.x; q < nl; q += gridDim.x) {
        const int32_t j = W.long_list[q];
        if (M.mc[j] >= 0) continue;  // block-uniform
        const int64_t lo = A.col_ptr[j], hi = A.col_ptr[j + 1];
        double bw = 0.0;
        int32_t br = INT32_MAX;
        for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) {
            const int32_t r = A.row_idx[k];
            if (M.mr[r] >= 0) continue;
            const double w = A.w[k];
            if (g_better(heavy, w, r, bw, br)) { bw = w; br = r; }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double ow = __shfl_xor(bw, off, 64);
            const int32_t orr = __shfl_xor(br, off, 64);
            if (g_better(heavy, ow, orr, bw, br)) { bw = ow; br = orr; }
        }
        if (lane == 0) { sw[wave] = bw; sr[wave] = br; }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int u = 1; u < 4; ++u)
                if (g_better(heavy, sw[u], sr[u], bw, br)) { bw = sw[u]; br = sr[u]; }
            M.prop_row[j] = br == INT32_MAX ? -1 : br;
            if (br != INT32_MAX) {
                M.prop_w[j] = bw;
                if (heavy) atomicMax(&M.rkey[br], wkey(bw));
                const int32_t s = atomicAdd(&M.counters[kMcmListLen], 1);
                M.list[s] = j;
            }
        }
        __syncthreads();
    }
}

// Pass 2 of the rows' choice: smallest column among the max-key proposers.
__global__ void k_greedy_accept(Mcm M, int heavy) {
    if (M.counters[kMcmDone]) return;
    const int32_t np = M.counters[kMcmListLen];
    for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < np; t += gridDim.x * blockDim.x) {
        const int32_t j = M.list[t];
        const int32_t r = M.prop_row[j];
        if (!heavy || M.rkey[r] == wkey(M.prop_w[j])) atomicMin(&M.racc[r], j);
    }
}

// Match the accepted pairs; the winner clears its row's slots (losers only
// compare the slot with their own index).
__global__ void k_greedy_match(Mcm M) {
    if (M.counters[kMcmDone]) return;
    const int32_t np = M.counters[kMcmListLen];
    for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < np; t += gridDim.x * blockDim.x) {
        const int32_t j = M.list[t];
        const int32_t r = M.prop_row[j];
        if (__hip_atomic_load(&M.racc[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != j) continue;
        M.mc[j] = r;
        M.mr[r] = j;
        M.rkey[r] = 0ull;
        __hip_atomic_store(&M.racc[r], kNoRoot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------------------
// Multi-source BFS phases.

// Phase start: every unmatched column is a root and forms the first frontier.
__global__ void k_bfs_roots(Csc A, Mcm M) {
    for (int64_t jj = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; jj < A.n;
         jj += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = (int32_t)jj;
        M.tree_row[j] = -1;   // rows and columns are both indexed 0..n-1
        M.parent[j] = kNoRoot;
        M.end_row[j] = kNoRoot;
        M.pkey[j] = 0ull;
        M.touched[j] = 0;
        const bool root = M.mc[j] < 0;
        const int32_t q = wave_append(&M.counters[kMcmFrontier], root);
        if (root) {
            M.tree_col[j] = j;
            M.front_a[q] = j;
        }
    }
}

// Levels are queued several at a time; the frontier of level L lives in
// front_a / front_b by the parity of L, its length in the counter word of the
// same parity (kMcmFrontier / kMcmNext).  A level whose frontier is empty does
// nothing but mark the next frontier empty, so levels queued after the last
// one are no-ops.  Level start: clear the level list and the next frontier's
// length, count the level.
__global__ void k_bfs_level_begin(Mcm M, int level) {
    const int cur = (level & 1) ? kMcmNext : kMcmFrontier;
    const int nxt = (level & 1) ? kMcmFrontier : kMcmNext;
    if (M.counters[cur] == 0) {  // past the last level: keep the emptiness going
        M.counters[nxt] = 0;
        return;
    }
    M.counters[kMcmLevelLen] = 0;
    M.counters[nxt] = 0;
    M.counters[kMcmLevels] += 1;
}

// Level step, pass 1: every row adjacent to a frontier column and not visited
// in an earlier level is touched (listed once) and its best parent key raised.
template <int T>
__global__ __launch_bounds__(256) void k_bfs_expand(Csc A, Mcm M, const int32_t* __restrict__ fr,
                                                    const int32_t* __restrict__ nfp, int heavy) {
    const int32_t nf = *nfp;
    const int lane = threadIdx.x & (T - 1);
    const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / T;
    const int64_t ntiles = ((int64_t)gridDim.x * blockDim.x) / T;
    for (int64_t f = tile; f < nf; f += ntiles) {
        const int32_t c = fr[f];
        const int64_t lo = A.col_ptr[c], hi = A.col_ptr[c + 1];
        for (int64_t k = lo + lane; k < hi; k += T) {
            const int32_t r = A.row_idx[k];
            if (M.tree_row[r] >= 0) continue;
            if (heavy) {
                const unsigned long long key = wkey(A.w[k]);
                if (__hip_atomic_load(&M.pkey[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < key)
                    atomicMax(&M.pkey[r], key);
            }
            const bool first = __hip_atomic_load(&M.touched[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
                               atomicExch(&M.touched[r], 1) == 0;
            const int32_t q = wave_append(&M.counters[kMcmLevelLen], first);
            if (first) M.level[q] = r;
        }
    }
}

// Level step, pass 2: parent = smallest frontier column among the heaviest.
template <int T>
__global__ __launch_bounds__(256) void k_bfs_parent(Csc A, Mcm M, const int32_t* __restrict__ fr,
                                                    const int32_t* __restrict__ nfp, int heavy) {
    const int32_t nf = *nfp;
    const int lane = threadIdx.x & (T - 1);
    const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / T;
    const int64_t ntiles = ((int64_t)gridDim.x * blockDim.x) / T;
    for (int64_t f = tile; f < nf; f += ntiles) {
        const int32_t c = fr[f];
        const int64_t lo = A.col_ptr[c], hi = A.col_ptr[c + 1];
        for (int64_t k = lo + lane; k < hi; k += T) {
            const int32_t r = A.row_idx[k];
            if (M.tree_row[r] >= 0) continue;
            if (!heavy || M.pkey[r] == wkey(A.w[k])) atomicMin(&M.parent[r], c);
        }
    }
}

// Level step, pass 3: the level's rows join their parents' trees; unmatched
// rows are endpoints (each tree keeps its smallest).
__global__ void k_bfs_join(Mcm M, const int32_t* __restrict__ nf) {
    if (*nf == 0) return;  // a level queued after the last one
    const int32_t nl = M.counters[kMcmLevelLen];
    for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nl; t += gridDim.x * blockDim.x) {
        const int32_t r = M.level[t];
        const int32_t tr = M.tree_col[M.parent[r]];
        M.tree_row[r] = tr;
        if (M.mr[r] < 0) atomicMin(&M.end_row[tr], r);
    }
}

// Level step, pass 4: the mates of the level's matched rows in trees that are
// still growing form the next frontier.
__global__ void k_bfs_next(Mcm M, int32_t* __restrict__ next, int32_t* __restrict__ next_len,
                           const int32_t* __restrict__ nf) {
    if (*nf == 0) return;
    const int32_t nl = M.counters[kMcmLevelLen];
    for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nl; t += gridDim.x * blockDim.x) {
        const int32_t r = M.level[t];
        const int32_t m = M.mr[r];
        const int32_t tr = M.tree_row[r];
        const bool grow = m >= 0 && M.end_row[tr] == kNoRoot;
        const int32_t q = wave_append(next_len, grow);
        if (!grow) continue;
        M.tree_col[m] = tr;
        next[q] = m;
    }
}

// Augment every recorded path (trees are vertex-disjoint).
__global__ void k_bfs_augment(Csc A, Mcm M) {
    for (int64_t tt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; tt < A.n;
         tt += (int64_t)gridDim.x * blockDim.x) {
        int32_t r = M.end_row[tt];
        wave_append(&M.counters[kMcmAugmented], r != kNoRoot);  // counts the paths
        if (r == kNoRoot) continue;
        while (r >= 0) {
            const int32_t c = M.parent[r];
            const int32_t r_next = M.mc[c];
            M.mc[c] = r;
            M.mr[r] = c;
            r = r_next;
        }
    }
}

// ---------------------------------------------------------------------------
// launchers

hipError_t launch_greedy_round(const Csc& A, const Mcm& M, const Work& W, int heavy,
                               int32_t long_threshold, bool has_long, hipStream_t s, int cus) {
    const unsigned blocks = (unsigned)(((int64_t)A.n * 16 + 255) / 256);
    hipLaunchKernelGGL(k_greedy_begin, dim3(1), dim3(64), 0, s, M);
    hipLaunchKernelGGL(k_greedy_propose<16>, dim3(blocks), dim3(256), 0, s, A, M, heavy, long_threshold);
    if (has_long) hipLaunchKernelGGL(k_greedy_propose_long, dim3(cus * 2), dim3(256), 0, s, A, M, W, heavy);
    hipLaunchKernelGGL(k_greedy_accept, dim3(cus * 2), dim3(256), 0, s, M, heavy);
    hipLaunchKernelGGL(k_greedy_match, dim3(cus * 2), dim3(256), 0, s, M);
    hipLaunchKernelGGL(k_greedy_end, dim3(1), dim3(1), 0, s, M);
    return hipGetLastError();
}

hipError_t launch_bfs_roots(const Csc& A, const Mcm& M, hipStream_t s, int cus) {
    hipLaunchKernelGGL(k_bfs_roots, dim3(cus * 8), dim3(256), 0, s, A, M);
    return hipGetLastError();
}

hipError_t launch_bfs_level(const Csc& A, const Mcm& M, int level, int heavy, hipStream_t s, int cus) {
    const int32_t* fr = (level & 1) ? M.front_b : M.front_a;
    int32_t* next = (level & 1) ? M.front_a : M.front_b;
    const int32_t* nf = M.counters + ((level & 1) ? kMcmNext : kMcmFrontier);
    int32_t* next_len = M.counters + ((level & 1) ? kMcmFrontier : kMcmNext);
    const int64_t want = ((int64_t)A.n * 64 + 255) / 256;
    const unsigned blocks = (unsigned)(want < cus * 16 ? (want > 0 ? want : 1) : cus * 16);
    hipLaunchKernelGGL(k_bfs_level_begin, dim3(1), dim3(1), 0, s, M, level);
    hipLaunchKernelGGL(k_bfs_expand<64>, dim3(blocks), dim3(256), 0, s, A, M, fr, nf, heavy);
    hipLaunchKernelGGL(k_bfs_parent<64>, dim3(blocks), dim3(256), 0, s, A, M, fr, nf, heavy);
    hipLaunchKernelGGL(k_bfs_join, dim3(cus * 2), dim3(256), 0, s, M, nf);
    hipLaunchKernelGGL(k_bfs_next, dim3(cus * 2), dim3(256), 0, s, M, next, next_len, nf);
    return hipGetLastError();
}

hipError_t launch_bfs_augment(const Csc& A, const Mcm& M, hipStream_t s, int cus) {
    hipLaunchKernelGGL(k_bfs_augment, dim3(cus * 8), dim3(256), 0, s, A, M);
    return hipGetLastError();
}

}  // namespace hwpm
