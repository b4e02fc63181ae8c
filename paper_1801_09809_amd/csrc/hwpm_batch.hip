// Batched solves: many matrices packed into one block-diagonal matrix.
//
// No entry of a block-diagonal matrix joins two blocks, so every alternating
// 4-cycle, every Step-C choice and every Step-D conflict stays inside one
// block: a round on the packed matrix is the same round on every block at
// once, and a block whose rounds have ended simply has no candidates any
// more.  The packed solve therefore gives every matrix exactly the result it
// gets alone.  These kernels pack the inputs, unpack the matchings, sum the
// matched weights of every block in its own fixed tree, and count the rounds
// in which each block flipped cycles.
#include "hwpm_internal.h"

namespace hwpm {

// Chunk of a packed array: entries [start, start + kPackChunk) of matrix b.
constexpr int kPackChunk = 4096;

// A block's own col_ptr must start at 0 and end at its nnz, and its rows and
// mates must lie inside the block (else the packed matrix would join blocks);
// violations set err[0].  Everything else is checked on the packed matrix.
__global__ __launch_bounds__(256) void k_pack_cols(const BatchItem* __restrict__ items,
                                                   const int32_t* __restrict__ chunk_item,
                                                   const int64_t* __restrict__ chunk_first,
                                                   int64_t* __restrict__ col_ptr,
                                                   int32_t* __restrict__ mate,
                                                   int32_t* __restrict__ mat_of_col, int32_t nchunks,
                                                   int64_t n_tot, int64_t nnz_tot,
                                                   int32_t* __restrict__ err) {
    for (int32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int32_t b = chunk_item[c];
        const BatchItem it = items[b];
        const int64_t j0 = chunk_first[c];
        const int64_t j1 = (j0 + kPackChunk < it.n) ? j0 + kPackChunk : it.n;
        if (j0 == 0 && threadIdx.x == 0 && (it.col_ptr[0] != 0 || it.col_ptr[it.n] != it.nnz))
            atomicOr(err, 1);
        for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
            const int64_t v = it.col_ptr[j];
            if (v < 0 || v > it.nnz) atomicOr(err, 1);
            col_ptr[it.col_off + j] = (v >= 0 && v <= it.nnz) ? it.nnz_off + v : it.nnz_off;
            if (mate) {
                const int32_t m = it.mate_in[j];
                if (m < 0 || m >= it.n) atomicOr(err, 4);
                mate[it.col_off + j] = (m >= 0 && m < it.n) ? (int32_t)(it.col_off + m) : (int32_t)it.col_off;
            }
            mat_of_col[it.col_off + j] = b;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) col_ptr[n_tot] = nnz_tot;
}

__global__ __launch_bounds__(256) void k_pack_entries(const BatchItem* __restrict__ items,
                                                      const int32_t* __restrict__ chunk_item,
                                                      const int64_t* __restrict__ chunk_first,
                                                      int32_t* __restrict__ row_idx,
                                                      double* __restrict__ w, int32_t nchunks,
                                                      int32_t* __restrict__ err) {
    for (int32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int32_t b = chunk_item[c];
        const BatchItem it = items[b];
        const int64_t k0 = chunk_first[c];
        const int64_t k1 = (k0 + kPackChunk < it.nnz) ? k0 + kPackChunk : it.nnz;
        for (int64_t k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
            const int32_t r = it.row_idx[k];
            // a row outside its block would join blocks: rejected
            if (r < 0 || r >= it.n) atomicOr(err, 2);
            row_idx[it.nnz_off + k] = (r >= 0 && r < it.n) ? (int32_t)(it.col_off + r) : 0;
            w[it.nnz_off + k] = it.w[k];
        }
    }
}

// skip (nullable): blocks with skip[b] != 0 keep their perm_out untouched.
__global__ __launch_bounds__(256) void k_unpack_perm(const BatchItem* __restrict__ items,
                                                     const int32_t* __restrict__ chunk_item,
                                                     const int64_t* __restrict__ chunk_first,
                                                     const int32_t* __restrict__ mc, int32_t nchunks,
                                                     const int32_t* __restrict__ skip) {
    for (int32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int32_t b = chunk_item[c];
        if (skip && skip[b] != 0) continue;  // block-uniform
        const BatchItem it = items[b];
        const int64_t j0 = chunk_first[c];
        const int64_t j1 = (j0 + kPackChunk < it.n) ? j0 + kPackChunk : it.n;
        for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x)
            it.perm_out[j] = (int32_t)(mc[it.col_off + j] - it.col_off);
    }
}

// Per-block totals: the same perfect binary tree as a single solve, over the
// block's own columns padded with +0.0 to next_pow2(n_b).  Level 1 sums
// aligned runs of kTreeBlock leaves of every block (one work item per run);
// level 2 gives each block one thread block over its run sums (at most
// kTreeBlock of them, i.e. blocks of up to 4M columns).
__global__ __launch_bounds__(256) void k_seg_tree_runs(const BatchItem* __restrict__ items,
                                                       const int32_t* __restrict__ run_item,
                                                       const int64_t* __restrict__ run_first,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ partial, int32_t nruns) {
    __shared__ double part[4];
    for (int32_t r = blockIdx.x; r < nruns; r += gridDim.x) {
        const BatchItem it = items[run_item[r]];
        const int64_t base = run_first[r] + threadIdx.x * 8;  // offset inside the block
        double v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (base + e < it.n) ? x[it.col_off + base + e] : 0.0;
        double s = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double o = __shfl_down(s, off, 64);
            if ((lane & (2 * off - 1)) == 0) s = s + o;
        }
        if (lane == 0) part[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) partial[r] = (part[0] + part[1]) + (part[2] + part[3]);
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void k_seg_tree_final(const BatchItem* __restrict__ items,
                                                         const int64_t* __restrict__ item_run0,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ partial,
                                                         double* __restrict__ out, int32_t count) {
    __shared__ double a[kTreeBlock], bb[kTreeBlock];
    for (int32_t b = blockIdx.x; b < count; b += gridDim.x) {
        const BatchItem it = items[b];
        // leaves: the block's own values when it fits one run, else its run sums
        const bool small = it.n <= kTreeBlock;
        const int64_t m = small ? it.n : (it.n + kTreeBlock - 1) / kTreeBlock;
        int64_t size = 1;
        while (size < m) size <<= 1;
        for (int64_t t = threadIdx.x; t < size; t += blockDim.x)
            a[t] = (t < m) ? (small ? x[it.col_off + t] : partial[item_run0[b] + t]) : 0.0;
        __syncthreads();
        double* src = a;
        double* dst = bb;
        for (int64_t len = size; len > 1; len >>= 1) {
            for (int64_t t = threadIdx.x; t < len / 2; t += blockDim.x) dst[t] = src[2 * t] + src[2 * t + 1];
            __syncthreads();
            double* tmp = src; src = dst; dst = tmp;
        }
        if (threadIdx.x == 0) out[b] = (m > 0) ? src[0] : 0.0;
        __syncthreads();
    }
}

// Rounds in which each block flipped at least one cycle.
__global__ void k_item_rounds(int32_t* __restrict__ flag, int32_t* __restrict__ rounds, int32_t count,
                              const int32_t* __restrict__ done) {
    if (*done) return;  // a round queued after the loop ended
    for (int32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < count; b += gridDim.x * blockDim.x) {
        if (flag[b]) {
            ++rounds[b];
            flag[b] = 0;
        }
    }
}

// Unmatched columns per block after the initial matching.
__global__ void k_item_unmatched(const int32_t* __restrict__ mc, const int32_t* __restrict__ mat_of_col,
                                 int64_t n_tot, int32_t* __restrict__ unmatched) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n_tot;
         j += (int64_t)gridDim.x * blockDim.x)
        if (mc[j] < 0) atomicAdd(&unmatched[mat_of_col[j]], 1);
}

hipError_t launch_pack(const BatchPlan& P, bool with_mates, hipStream_t s, int cus) {
    const unsigned g = (unsigned)(cus * 8);
    hipLaunchKernelGGL(k_pack_cols, dim3(g), dim3(256), 0, s, P.items, P.col_chunk_item, P.col_chunk_first,
                       P.col_ptr, with_mates ? P.mate : nullptr, P.mat_of_col, P.ncol_chunks, P.n_tot,
                       P.nnz_tot, P.item_err);
    if (P.nent_chunks > 0)
        hipLaunchKernelGGL(k_pack_entries, dim3(g), dim3(256), 0, s, P.items, P.ent_chunk_item,
                           P.ent_chunk_first, P.row_idx, P.w, P.nent_chunks, P.item_err);
    return hipGetLastError();
}

hipError_t launch_unpack(const BatchPlan& P, const int32_t* mc, hipStream_t s, int cus, const int32_t* skip) {
    hipLaunchKernelGGL(k_unpack_perm, dim3(cus * 8), dim3(256), 0, s, P.items, P.col_chunk_item,
                       P.col_chunk_first, mc, P.ncol_chunks, skip);
    return hipGetLastError();
}

hipError_t launch_seg_tree(const BatchPlan& P, const double* x, double* out, hipStream_t s, int cus) {
    if (P.nruns > 0)
        hipLaunchKernelGGL(k_seg_tree_runs, dim3(cus * 8), dim3(256), 0, s, P.items, P.run_item,
                           P.run_first, x, P.partial, P.nruns);
    hipLaunchKernelGGL(k_seg_tree_final, dim3(cus * 4), dim3(1024), 0, s, P.items, P.item_run0, x,
                       P.partial, out, P.count);
    return hipGetLastError();
}

hipError_t launch_item_rounds(const BatchPlan& P, const int32_t* done, hipStream_t s) {
    hipLaunchKernelGGL(k_item_rounds, dim3(64), dim3(256), 0, s, P.item_flag, P.item_rounds, P.count, done);
    return hipGetLastError();
}

hipError_t launch_item_unmatched(const BatchPlan& P, const int32_t* mc, hipStream_t s, int cus) {
    hipLaunchKernelGGL(k_item_unmatched, dim3(cus * 8), dim3(256), 0, s, mc, P.mat_of_col, P.n_tot,
                       P.item_unmatched);
    return hipGetLastError();
}

}  // namespace hwpm
