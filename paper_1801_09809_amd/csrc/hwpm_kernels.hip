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

#include "hwpm_device.h"

namespace hwpm {

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

// find_row, given the column's bounds, with the final window's nine reads
// issued together.  VEC (at least nine entries in the matrix): the window is
// read as two 16-byte loads and one 4-byte load from its start, moved back
// to keep inside the array (one thread per column, neighbouring lanes about
// a column apart, so each load instruction is one request per lane).
// Otherwise each index is clamped to the column's last entry (to entry 0 for
// an empty column, so the matrix must hold at least one entry).  Only the
// slots inside the column can hit.  The search kernels keep find_row.
template <bool VEC>
__device__ __forceinline__ int64_t find_row_window(const int32_t* __restrict__ row_idx, int64_t lo,
                                                   int64_t end, int32_t r, int64_t nnz) {
    // the column is row_idx[lo, end)
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
    int32_t v[9];
    int64_t hit = -1;
    if constexpr (VEC) {
        const int64_t base = lo + 9 <= nnz ? lo : nnz - 9;  // <= lo
        __builtin_memcpy(v, row_idx + base, 16);
        __builtin_memcpy(v + 4, row_idx + base + 4, 16);
        v[8] = row_idx[base + 8];
#pragma unroll
        for (int q = 0; q <= 8; ++q) {
            const int64_t pos = base + q;
            if (pos >= lo && pos <= lo + len && pos < end && v[q] == r) hit = pos;
        }
    } else {
#pragma unroll
        for (int q = 0; q <= 8; ++q) {
            const int64_t pos = lo + q;
            v[q] = row_idx[pos < end ? pos : (end > 0 ? end - 1 : 0)];
        }
#pragma unroll
        for (int q = 0; q <= 8; ++q)
            if (q <= len && lo + q < end && v[q] == r) hit = lo + q;
    }
    return hit;
}

// With pos32 (nnz < 2^31) it also fills the 32-bit column pointers and the
// matched positions the transposed searches read.
template <bool VEC>
__global__ void k_init_match(Csc A, Work W, const int32_t* __restrict__ mate_in,
                             int32_t long_threshold, int pos32) {
    for (int64_t jj = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; jj < A.n;
         jj += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = (int32_t)jj;
        W.dgain[j] = 0ull;
        W.droot[j] = kNoRoot;
        // the mate is read with the column bounds (the empty asm statement
        // keeps the compiler from sinking its load past the branches below)
        const int64_t lo = A.col_ptr[j], hi = A.col_ptr[j + 1];
        const int32_t r = mate_in[j];
        asm volatile("" ::"v"(lo), "v"(hi), "v"(r));
        const bool is_long = hi - lo > long_threshold;
        const int32_t q = wave_append(&W.counters[kNumLong], is_long);
        if (is_long) W.long_list[q] = j;
        if (pos32) {
            W.cp32[j] = (int32_t)lo;
            if (j == A.n - 1) W.cp32[A.n] = (int32_t)hi;
        }
        if (r < 0 || r >= A.n) {
            atomicOr(&W.counters[kErrMatch], 1);
            W.mc[j] = -1;
            continue;
        }
        W.mr[r] = j;  // a row claimed twice keeps one writer: k_check_match sees the other
        W.mc[j] = r;
        const int64_t p = find_row_window<VEC>(A.row_idx, lo, hi, r, A.nnz);
        if (p < 0) {
            atomicOr(&W.counters[kErrMatch], 4);
            W.wm[j] = 0.0;
        } else {
            W.wm[j] = A.w[p];
        }
        if (pos32) W.pm[j] = (int32_t)p;
    }
}

// n columns mapped into n rows form a permutation iff every column reads
// itself back through the row it claimed.
__global__ void k_check_match(Csc A, Work W) {
    for (int64_t jj = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; jj < A.n;
         jj += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = W.mc[jj];
        if (r >= 0 && W.mr[r] != (int32_t)jj) atomicOr(&W.counters[kErrMatch], 2);
    }
}

hipError_t launch_init_match(const Csc& A, const Work& W, const int32_t* mate_in,
                             int32_t long_threshold, hipStream_t s) {
    const int64_t blocks = ((int64_t)A.n + 255) / 256;
    const unsigned g = (unsigned)(blocks < 65536 ? blocks : 65536);
    const int pos32 = A.nnz < ((int64_t)1 << 31) ? 1 : 0;
    if (A.nnz >= 9)
        hipLaunchKernelGGL(k_init_match<true>, dim3(g), dim3(256), 0, s, A, W, mate_in, long_threshold, pos32);
    else
        hipLaunchKernelGGL(k_init_match<false>, dim3(g), dim3(256), 0, s, A, W, mate_in, long_threshold, pos32);
    hipLaunchKernelGGL(k_check_match, dim3(g), dim3(256), 0, s, A, W);
    return hipGetLastError();
}

// Chunk table of the long columns: chunk_off[q] = number of kLongChunk-entry
// chunks in long columns 0..q-1.  One block: each thread sums a contiguous
// run of long columns, a block scan of the run sums, then each thread writes
// its run's offsets.
__global__ __launch_bounds__(1024) void k_long_chunks(Work W, Csc A) {
    __shared__ int64_t wsum[16];
    const int32_t nl = W.counters[kNumLong];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t per = ((int64_t)nl + 1023) / 1024;
    const int64_t b = t * per, e = (b + per < nl) ? b + per : nl;
    int64_t sum = 0;
    for (int64_t q = b; q < e; ++q) {
        const int32_t j = W.long_list[q];
        const int64_t len = A.col_ptr[j + 1] - A.col_ptr[j];
        sum += (len + kLongChunk - 1) / kLongChunk;
    }
    int64_t incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int64_t run = incl - sum;
    for (int u = 0; u < wave; ++u) run += wsum[u];
    if (t == 1023) {
        W.counters[kNumChunks] = (int32_t)(run + sum);
        W.chunk_off[nl] = run + sum;
    }
    for (int64_t q = b; q < e; ++q) {
        W.chunk_off[q] = run;
        const int32_t j = W.long_list[q];
        const int64_t len = A.col_ptr[j + 1] - A.col_ptr[j];
        const int64_t nc = (len + kLongChunk - 1) / kLongChunk;
        for (int64_t c = 0; c < nc; ++c) W.chunk_col[run + c] = (int32_t)q;
        run += nc;
    }
}

hipError_t launch_long_chunks(const Work& W, const Csc& A, hipStream_t s) {
    hipLaunchKernelGGL(k_long_chunks, dim3(1), dim3(1024), 0, s, W, A);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step D.  Pass 1 (the atomicMax of the gain bits) ran in publish(); pass 2
// picks the smallest root among the roots that reached the maximum.  A column
// that kept a cycle of its own accepts nothing.

// The candidate list of the round (every root that holds a Step-C winner,
// searched this round or kept from an earlier one) and pass 1 of Step D:
// raise the max-gain slot of each candidate's other column.
__global__ void k_collect(Csc A, Work W, int slot) {
    if (round_over(W)) return;
    for (int64_t jj = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; jj < A.n;
         jj += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = (int32_t)jj;
        const bool has = W.best_i[j] >= 0;
        if (has) {
            const int32_t c = W.best_c[j];
            const unsigned long long gb = gain_bits(W.best_g[j]);
            if (__hip_atomic_load(&W.dgain[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gb)
                atomicMax(&W.dgain[c], gb);
        }
        const int32_t q = wave_append(&W.counters[slot_word(slot, kCand)], has);
        if (has) W.cand[q] = j;
    }
}

hipError_t launch_collect(const Csc& A, const Work& W, int slot, hipStream_t s, int cus) {
    hipLaunchKernelGGL(k_collect, dim3(cus * 4), dim3(256), 0, s, A, W, slot);
    return hipGetLastError();
}

__global__ void k_resolve(Work W, int slot) {
    if (round_over(W)) return;
    const int32_t nc = W.counters[slot_word(slot, kCand)];
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
__global__ void k_apply(Csc A, Work W, int slot, int transposed) {
    if (round_over(W)) return;
    const int32_t nc = W.counters[slot_word(slot, kCand)];
    if (blockIdx.x == 0 && threadIdx.x < kSlotWords)
        W.counters[slot_word((slot + 1) % kSlots, threadIdx.x)] = 0;
    if (blockIdx.x == 0 && threadIdx.x < kSpread)
        W.counters[spread_word((slot + 1) % kSlots, threadIdx.x)] = 0;
    for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nc; t += gridDim.x * blockDim.x) {
        const int32_t j = W.cand[t];
        const int32_t c = W.best_c[j];
        W.dgain[j] = 0ull;
        W.droot[j] = kNoRoot;
        const bool won = W.best_i[c] < 0 &&
                         __hip_atomic_load(&W.droot[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == j;
        // the two rows whose mate changed, for the per-entry mate columns
        const int32_t q = wave_append(&W.counters[slot_word(slot, kApplied)], won);
        if (!won) continue;
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
        if (transposed) {
            // the row lists follow their rows: j now holds row i (was c's),
            // and the matched positions follow the flip
            const int2 sj = W.rsl[j], sc = W.rsl[c];
            W.rsl[j] = sc;
            W.rsl[c] = sj;
            // rows too long for one block's refresh, for the grid (rare)
            if (sc.y > kHeavyRow) W.heavy[atomicAdd(&W.counters[slot_word(slot, kHeavy)], 1)] = j;
            if (sj.y > kHeavyRow) W.heavy[atomicAdd(&W.counters[slot_word(slot, kHeavy)], 1)] = c;
            if (W.rtab) {
                const int32_t tj = W.rtab[j], tc = W.rtab[c];
                W.rtab[j] = tc;
                W.rtab[c] = tj;
            }
            W.pm[j] = (int32_t)W.best_k[j];
            W.pm[c] = (int32_t)W.best_p[j];
        }
        if (W.mat_of_col) {
            const int32_t blk = W.mat_of_col[j];
            W.item_flag[blk] = 1;
            atomicAdd(&W.item_cycles[blk], 1ull);
        }
        W.flips[4 * (int64_t)q + 0] = i;
        W.flips[4 * (int64_t)q + 1] = j;
        W.flips[4 * (int64_t)q + 2] = l;
        W.flips[4 * (int64_t)q + 3] = c;
    }
}

hipError_t launch_apply(const Csc& A, const Work& W, int slot, bool transposed, hipStream_t s,
                        int cus) {
    hipLaunchKernelGGL(k_apply, dim3(cus * 2), dim3(256), 0, s, A, W, slot, transposed ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pattern transpose, built once per solve: the row list of every row (the
// columns holding an entry in that row, in no particular order) with the CSC
// position of each entry.  Counting sort: per-row counts with atomics, an
// exclusive scan, then a scatter through per-row atomic cursors.

__global__ void k_row_count(Csc A, const int32_t* __restrict__ mr, int32_t* __restrict__ cnt) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < A.nnz;
         k += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[mr[A.row_idx[k]]], 1);
}

// Exclusive scan of m int32 values into int64 out[0..m] (out[m] = total):
// per-block scans of 2048 values, one block scanning the block sums, and an
// add of the block offsets.
__global__ __launch_bounds__(256) void k_scan_local(const int32_t* __restrict__ in, int64_t m,
                                                    int64_t* __restrict__ out,
                                                    int64_t* __restrict__ sums) {
    __shared__ int64_t wsum[4];
    const int64_t base = (int64_t)blockIdx.x * 2048 + threadIdx.x * 8;
    int64_t v[8];
    int64_t s = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t x = (base + e < m) ? in[base + e] : 0;
        v[e] = s;
        s += x;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t incl = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int64_t woff = 0;
    for (int u = 0; u < wave; ++u) woff += wsum[u];
    const int64_t excl = incl - s + woff;
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if (base + e < m) out[base + e] = v[e] + excl;
    if (threadIdx.x == 255) sums[blockIdx.x] = woff + incl;
}

__global__ __launch_bounds__(1024) void k_scan_sums(int64_t* __restrict__ sums, int64_t nb,
                                                    int64_t* __restrict__ total) {
    __shared__ int64_t wsum[16];
    __shared__ int64_t carry;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
        const int64_t idx = c0 + t;
        const int64_t x = (idx < nb) ? sums[idx] : 0;
        int64_t incl = x;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t o = __shfl_up(incl, off, 64);
            if (lane >= off) incl += o;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        int64_t woff = carry;
        for (int u = 0; u < wave; ++u) woff += wsum[u];
        const int64_t excl = incl - x + woff;
        if (idx < nb) sums[idx] = excl;
        __syncthreads();
        if (t == 1023) carry = excl + x;
        __syncthreads();
    }
    if (t == 0) *total = carry;
}

__global__ void k_scan_add(int64_t* __restrict__ out, int64_t m, const int64_t* __restrict__ sums) {
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < m;
         x += (int64_t)gridDim.x * blockDim.x)
        out[x] += sums[x / 2048];
}

__device__ __forceinline__ void fill_entry(const Csc& A, const Work& W, int32_t j, int64_t k) {
    const int32_t r = W.mr[A.row_idx[k]];   // slot: the column matched to the row
    const int32_t slot = atomicAdd(&W.rowcnt[r], 1);
    const int64_t e = W.rowptr[r] + slot;
    W.colidx[e] = j;
    W.cscpos[e] = (int32_t)k;
}

template <int T>
__global__ __launch_bounds__(256) void k_row_fill_short(Csc A, Work W, int32_t long_threshold) {
    const int lane = threadIdx.x & (T - 1);
    const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / T;
    if (tile >= A.n) return;
    const int32_t j = (int32_t)tile;
    const int64_t lo = A.col_ptr[j], hi = A.col_ptr[j + 1];
    if (hi - lo > long_threshold) return;
    for (int64_t k = lo + lane; k < hi; k += T) fill_entry(A, W, j, k);
}

__global__ __launch_bounds__(256) void k_row_fill_long(Csc A, Work W) {
    const int32_t total = W.counters[kNumChunks];
    for (int32_t cid = blockIdx.x; cid < total; cid += gridDim.x) {
        const int32_t a = W.chunk_col[cid];
        const int32_t j = W.long_list[a];
        const int64_t lo = A.col_ptr[j] + (int64_t)(cid - W.chunk_off[a]) * kLongChunk;
        const int64_t hi0 = A.col_ptr[j + 1];
        const int64_t hi = (lo + kLongChunk < hi0) ? lo + kLongChunk : hi0;
        for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) fill_entry(A, W, j, k);
    }
}

// Slot pointers of the row lists: rsl[j] = (start, length) of the list of
// the row matched to j.
// Hash tables of the long row lists (filled by k_rowset_plan and
// k_rowset_fill, see there):
// the table words a list of len entries takes from the pool of nnz + 64
// words, or -1 (short list, or no room left).
__device__ __forceinline__ int32_t rowset_take(const Work& W, int32_t len, int64_t nnz) {
    if (len <= kRowSetMin) return -1;
    unsigned long long size = 64;
    while (size < 2ull * (unsigned long long)len) size <<= 1;
    const unsigned long long at = atomicAdd(reinterpret_cast<unsigned long long*>(W.counters + kTabUsed), 2 * size);
    return at + 2 * size <= (unsigned long long)nnz + 64 ? (int32_t)at : -1;
}

// Record slot j's table (or none) and list it for filling.  All active lanes
// of the wave call it together.
__device__ __forceinline__ void rowset_note(const Work& W, int32_t j, int32_t off, bool valid) {
    if (valid) W.rtab[j] = off;
    const int32_t q = wave_append(&W.counters[kTabRows], valid && off >= 0);
    if (valid && off >= 0) W.medium[q] = j;  // the buffer is free until the rounds
}

__global__ void k_slot_ptrs(Csc A, Work W) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < A.n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int32_t len = (int32_t)(W.rowptr[j + 1] - W.rowptr[j]);
        W.rsl[j] = make_int2((int32_t)W.rowptr[j], len);
        if (W.rtab) rowset_note(W, (int32_t)j, rowset_take(W, len, A.nnz), true);  // grid-uniform
    }
}

__global__ void k_mrk_fill(Csc A, Work W) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < A.nnz;
         k += (int64_t)gridDim.x * blockDim.x)
        W.mrk[k] = W.mr[A.row_idx[k]];
}

// Bucketed transpose (no global atomics), keyed by slot = the column matched
// to an entry's row.  Slots are grouped into buckets of 2^rb consecutive
// slots.  Pass 1 works on tiles of kTpTile consecutive entries: it counts each
// tile's entries per bucket (LDS histogram); a scan of the bucket-major count
// table gives every (bucket, tile) run its place; a second sweep sorts each
// tile by bucket in LDS and writes the (slot, column, position) triples out in
// contiguous runs, filling the per-entry mate columns on the way.  Pass 2
// gives each bucket one block, which counts its slots in LDS, writes the slot
// pointers and places every entry (the bucket's output range is small enough
// to stay in L2).
constexpr int kTpTile = 4096;     // entries per pass-1 tile (256 threads x 16)
constexpr int kTpMaxBuckets = 1024;
constexpr int kTpMaxRows = 8192;  // slots per bucket (LDS counters of pass 2)
constexpr int kTpScatterThreads = 512;  // pass-1b block size (against 256: pass 1b about 5% faster)

struct TpPlan {
    int rb;          // log2 slots per bucket
    int64_t nb;      // buckets
    int64_t nseg;    // pass-1 tiles
    bool ok;         // false: sizes beyond the LDS limits
};

TpPlan tp_plan(int64_t n, int64_t nnz) {
    // about 256 buckets (measured: against 512, each tile's runs per bucket
    // are twice as long and the count table half the size; the transpose of
    // the random 2^20 workload drops from 0.45 to 0.37 ms); more (up to
    // kTpMaxBuckets) once a bucket would exceed kTpMaxRows slots
    TpPlan P;
    int lg = 0;
    while (((int64_t)1 << lg) < n) ++lg;
    P.rb = lg - 8;
    if (P.rb < 6) P.rb = 6;
    while (P.rb > 6 && ((int64_t)1 << P.rb) > kTpMaxRows) --P.rb;
    P.nb = (n + ((int64_t)1 << P.rb) - 1) >> P.rb;
    P.nseg = (nnz + kTpTile - 1) / kTpTile;
    if (P.nseg < 1) P.nseg = 1;
    P.ok = P.nb <= kTpMaxBuckets && ((int64_t)1 << P.rb) <= kTpMaxRows && nnz < ((int64_t)1 << 31);
    return P;
}

// Blocks go to the chip's 8 dies (XCDs, each with its own L2) in turn:
// block b runs on die b mod 8.  This maps block b of a grid of nblk blocks
// to a tile such that each die takes one contiguous range of tiles, in
// order (a bijection on [0, nblk)).
constexpr int kXcds = 8;
__device__ __forceinline__ int32_t xcd_tile(int32_t b, int32_t nblk) {
    const int32_t x = b % kXcds, i = b / kXcds, q = nblk / kXcds, r = nblk % kXcds;
    return x * q + (x < r ? x : r) + i;
}

// The column of the first entry of every pass-1 tile: column c owns the
// tiles whose first entry lies in [col_ptr[c], col_ptr[c+1]).
__global__ __launch_bounds__(256) void k_tp_tile_cols(Csc A, Work W, int32_t nseg) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < A.n;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t lo = A.col_ptr[c], hi = A.col_ptr[c + 1];
        for (int64_t t = (lo + kTpTile - 1) / kTpTile; t < nseg && t * kTpTile < hi; ++t)
            W.tile_col[t] = (int32_t)c;
    }
}

// Exclusive scan in place of cnt[0..2*64) by the first wave of the block (two
// values per lane); returns nothing, the caller synchronises.
__device__ __forceinline__ void wave_scan128(int32_t* cnt) {
    const int t = threadIdx.x;
    if (t < 64) {
        const int32_t a0 = cnt[2 * t], a1 = cnt[2 * t + 1];
        const int32_t v = a0 + a1;
        int32_t incl = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t x = __shfl_up(incl, o, 64);
            if (t >= o) incl += x;
        }
        cnt[2 * t] = incl - v;
        cnt[2 * t + 1] = incl - v + a0;
    }
}

// Pass 1a: the slot of every entry (mrk[k] = m_i of its row, the mate
// column the search streams) and the per-(tile, bucket) counts, one row of
// nb counts per tile.
__global__ __launch_bounds__(256) void k_tp_hist(Csc A, Work W, int rb, int32_t nb, int32_t nseg,
                                                 int32_t* __restrict__ cnt) {
    constexpr int U = kTpTile / 256;
    __shared__ int32_t hist[kTpMaxBuckets];
    if (W.counters[kErrMatch]) return;  // block-uniform: no slots without a matching
    for (int b = threadIdx.x; b < nb; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    const int32_t seg = blockIdx.x;
    const int64_t k0 = (int64_t)seg * kTpTile;
    if (A.nnz > 0) {  // block-uniform
        // Loads first, with indices clamped to the last entry, so that the U
        // row-index loads and then the U gathers are each in flight
        // together; the stores and counts of the entries past the end are
        // skipped afterwards.  The two streams are marked nontemporal so
        // that they do not push the gathered mate array (n words, read at
        // random) out of L2.
        const int64_t last = A.nnz - 1;
        int32_t sl[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = k0 + threadIdx.x + 256 * u;
            sl[u] = __builtin_nontemporal_load(A.row_idx + (k < A.nnz ? k : last));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) sl[u] = W.mr[sl[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = k0 + threadIdx.x + 256 * u;
            if (k < A.nnz) {
                __builtin_nontemporal_store(sl[u], W.mrk + k);
                atomicAdd(&hist[sl[u] >> rb], 1);
            }
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += blockDim.x) cnt[(int64_t)seg * nb + b] = hist[b];
}

// Inclusive running maximum over the 64 lanes of a wave (values >= -1)
// with DPP moves: shifts by 1, 2, 4, 8 lanes inside each row of 16, then the
// last lane of row 0 into row 1 (and of row 2 into row 3), then the last lane
// of row 1 into rows 2 and 3.  Lanes without a source keep -1.
__device__ __forceinline__ int32_t wave_incl_max(int32_t v) {
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x111, 0xF, 0xF, false));  // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x112, 0xF, 0xF, false));  // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x114, 0xF, 0xF, false));  // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x118, 0xF, 0xF, false));  // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x142, 0xA, 0xF, false));  // row_bcast:15
    v = max(v, __builtin_amdgcn_update_dpp(-1, v, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return v;
}

// The entries of (tile, bucket) go after those of every earlier bucket and,
// in the same bucket, of every earlier tile: a scan down each column of the
// tile-major count table.  Part 1: block q takes tiles [q S, q S + S) and,
// per bucket, replaces each count by the sum of the counts above it inside
// the part, and writes the part's sums.
__global__ __launch_bounds__(256) void k_tp_colsum(int32_t* __restrict__ cnt, int32_t nb, int32_t nseg,
                                                   int32_t S, int64_t* __restrict__ part) {
    const int32_t s0 = blockIdx.x * S, s1 = (s0 + S < nseg) ? s0 + S : nseg;
    for (int32_t b = threadIdx.x; b < nb; b += blockDim.x) {
        int32_t run = 0, s = s0;
        for (; s + 8 <= s1; s += 8) {  // eight loads in flight, then the running sum
            int32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = cnt[(int64_t)(s + u) * nb + b];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                cnt[(int64_t)(s + u) * nb + b] = run;
                run += v[u];
            }
        }
        for (; s < s1; ++s) {
            const int32_t v = cnt[(int64_t)s * nb + b];
            cnt[(int64_t)s * nb + b] = run;
            run += v;
        }
        part[(int64_t)blockIdx.x * nb + b] = run;
    }
}

// Part 2: a wave per bucket scans the parts' sums down the parts (each
// part's value becomes where its entries of that bucket begin, counted from
// the bucket's start), and the last wave to finish scans the bucket totals
// across the buckets (bstart, with bstart[nb] = nnz).  Spread over the grid,
// the table's reads and writes are not bound by one CU's bandwidth.
__global__ __launch_bounds__(64) void k_tp_colscan(int64_t* __restrict__ part, int32_t nb, int32_t nparts,
                                                   int64_t* __restrict__ btot, int64_t* __restrict__ bstart,
                                                   int64_t nnz, int32_t* __restrict__ done) {
    const int32_t b = blockIdx.x;
    const int lane = threadIdx.x;
    int64_t carry = 0;
    for (int32_t q0 = 0; q0 < nparts; q0 += 64) {
        const int32_t q = q0 + lane;
        const int64_t v = q < nparts ? part[(int64_t)q * nb + b] : 0;
        int64_t incl = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t x = __shfl_up(incl, o, 64);
            if (lane >= o) incl += x;
        }
        if (q < nparts) part[(int64_t)q * nb + b] = carry + incl - v;
        carry += __shfl(incl, 63, 64);
    }
    int32_t ticket = 0;
    if (lane == 0) {
        __hip_atomic_store(&btot[b], carry, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ticket = __hip_atomic_fetch_add(done, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    }
    ticket = __shfl(ticket, 0, 64);
    if (ticket != nb - 1) return;  // wave-uniform: not the last bucket's wave
    int64_t run = 0;
    for (int32_t b0 = 0; b0 < nb; b0 += 64) {
        const int32_t bb = b0 + lane;
        const int64_t v = bb < nb ? __hip_atomic_load(&btot[bb], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
        int64_t incl = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t x = __shfl_up(incl, o, 64);
            if (lane >= o) incl += x;
        }
        if (bb < nb) bstart[bb] = run + incl - v;
        run += __shfl(incl, 63, 64);
    }
    if (lane == 0) {
        bstart[nb] = nnz;
        *done = 0;
    }
}

// Packed entries: when a slot's offset inside its bucket (rb bits) and a
// column fit one 32-bit word together (n <= 2^(32 - rb)), passes 1b-3 move
// that word instead of two, the column in the low 32 - rb bits.
__device__ __forceinline__ int32_t tp_pack(int32_t slot, int32_t col, int rb) {
    return (int32_t)(((uint32_t)slot & ((1u << rb) - 1u)) << (32 - rb) | (uint32_t)col);
}
__device__ __forceinline__ int32_t tp_local(int32_t word, int rb) { return (int32_t)((uint32_t)word >> (32 - rb)); }
__device__ __forceinline__ int32_t tp_col_of(int32_t word, int rb) {
    return (int32_t)((uint32_t)word & ((1u << (32 - rb)) - 1u));
}

// Pass 1b: sort the tile by bucket in LDS, write the triples in runs.  NT
// threads per block; MB bounds the bucket count (the LDS tables are sized by
// it, so the small form leaves room for more blocks per CU).
template <bool POS, int NT, int MB, bool PACK>
__global__ __launch_bounds__(NT) void k_tp_scatter(Csc A, Work W, int rb, int32_t nb, int32_t S,
                                                   const int64_t* __restrict__ part,
                                                   const int32_t* __restrict__ local,
                                                   const int64_t* __restrict__ bstart) {
    constexpr int U = kTpTile / NT, NW = NT / 64;
    __shared__ int32_t s_slot[kTpTile], s_col[kTpTile], s_pos[POS ? kTpTile : 1];
    __shared__ int32_t hist[MB], start[MB], base[MB];
    __shared__ int32_t wsum[NW], wmax[NW * U];
    if (W.counters[kErrMatch]) return;  // block-uniform: no slots without a matching
    // consecutive tiles on one die: a bucket's runs from neighbouring tiles
    // are neighbours in memory, so their partial lines meet in one L2
    const int32_t seg = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t k0 = (int64_t)seg * kTpTile;
    const int32_t len = (int32_t)((k0 + kTpTile < A.nnz) ? kTpTile : A.nnz - k0);
    // The column of every entry of the tile: the tile's first column, a mark
    // at the first entry of each later column that starts inside the tile,
    // and a running maximum along the tile (columns do not decrease along the
    // entries; an empty column starts where the next one does and loses).
    int32_t* mark = s_col;  // free until the placement below
    for (int b = threadIdx.x; b < nb; b += NT) {  // rows of the scanned tables: coalesced
        hist[b] = 0;
        base[b] = (int32_t)(bstart[b] + part[(int64_t)(seg / S) * nb + b] + local[(int64_t)seg * nb + b]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) mark[threadIdx.x + NT * u] = -1;
    __syncthreads();
    int32_t cf = W.tile_col[seg];
    cf = cf < 0 ? 0 : (cf >= A.n ? A.n - 1 : cf);
    if (threadIdx.x == 0) mark[0] = cf;
    for (int64_t c = (int64_t)cf + 1 + threadIdx.x; c <= A.n; c += NT) {
        const int64_t p = A.col_ptr[c];
        if (p >= k0 + len) break;  // and so for every later column
        if (p > k0) atomicMax(&mark[p - k0], (int32_t)c);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t sl[U], co[U], rk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t k = k0 + threadIdx.x + NT * u;
        sl[u] = (k < A.nnz) ? W.mrk[k] : -1;
        co[u] = wave_incl_max(mark[threadIdx.x + NT * u]);  // the wave's part of row u
        if (lane == 63) wmax[NW * u + wave] = co[u];
    }
    __syncthreads();
    {
        // entry x = NT u + threadIdx.x follows rows 0..u-1 and, in row u, the
        // waves before this one
        int32_t pre = -1;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int32_t rp = pre;
            for (int w = 0; w < wave; ++w) rp = rp > wmax[NW * u + w] ? rp : wmax[NW * u + w];
            co[u] = co[u] > rp ? co[u] : rp;
            co[u] = co[u] > cf ? co[u] : cf;  // no-op: every entry's column is >= cf
#pragma unroll
            for (int w = 0; w < NW; ++w) pre = pre > wmax[NW * u + w] ? pre : wmax[NW * u + w];
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (sl[u] >= 0) rk[u] = atomicAdd(&hist[sl[u] >> rb], 1);
    __syncthreads();
    // exclusive scan of hist[0..nb): each thread owns up to MB / NT buckets
    const int per = (nb + NT - 1) / NT;
    const int bb = threadIdx.x * per, be = (bb + per < nb) ? bb + per : nb;
    int32_t run = 0;
    for (int b = bb; b < be; ++b) run += hist[b];
    int32_t incl = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int32_t acc = incl - run;
    for (int u = 0; u < wave; ++u) acc += wsum[u];
    for (int b = bb; b < be; ++b) {
        start[b] = acc;
        acc += hist[b];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (sl[u] >= 0) {
            const int32_t x = start[sl[u] >> rb] + rk[u];
            s_slot[x] = sl[u];
            s_col[x] = co[u];
            if (POS) s_pos[x] = (int32_t)(k0 + threadIdx.x + NT * u);
        }
    }
    __syncthreads();
    for (int32_t e = threadIdx.x; e < len; e += NT) {
        const int32_t slot = s_slot[e];
        const int32_t b = slot >> rb;
        const int32_t g = base[b] + (e - start[b]);
        if (PACK) {
            W.tp_row[g] = tp_pack(slot, s_col[e], rb);
        } else {
            W.tp_row[g] = slot;
            W.tp_col[g] = s_col[e];
        }
        if (POS) W.tp_pos[g] = s_pos[e];
    }
}

// Pass 2: one block per bucket splits it into kTpSub sub-buckets of
// 2^(rb - 6) consecutive slots, again sorting tiles in LDS so the triples
// leave in runs, and records where each sub-bucket starts.
constexpr int kTpSub = 64;

template <bool POS, bool PACK>
__global__ __launch_bounds__(1024) void k_tp_split(Csc A, Work W, int rb, int32_t nb,
                                                   const int64_t* __restrict__ bstart, int64_t big_min) {
    __shared__ int32_t s_slot[kTpTile], s_col[PACK ? 1 : kTpTile], s_pos[POS ? kTpTile : 1];
    __shared__ int32_t hist[kTpSub], start[kTpSub], cursor[kTpSub];
    if (W.counters[kErrMatch]) return;  // block-uniform: no slots without a matching
    const int32_t b = blockIdx.x;
    const int64_t r0 = (int64_t)b << rb;
    const int sb = rb - 6;
    const int64_t e0 = bstart[b], e1 = bstart[b + 1];
    const int t = threadIdx.x;
    if (b == nb - 1 && t == 0) W.tp_sub[(int64_t)nb * kTpSub] = A.nnz;
    if (e1 - e0 > big_min) return;  // an oversized bucket: the grid-wide split takes it
    if (t < kTpSub) hist[t] = 0;
    __syncthreads();
    // loads first (four per thread, indices clamped into the bucket), then
    // the counts: the loads of a pass are in flight together
    for (int64_t eb = e0; eb < e1; eb += 4 * (int64_t)blockDim.x) {  // uniform trip count
        int32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t e = eb + t + (int64_t)blockDim.x * u;
            v[u] = W.tp_row[e < e1 ? e : e1 - 1];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (eb + t + (int64_t)blockDim.x * u < e1)
                atomicAdd(&hist[(PACK ? tp_local(v[u], rb) : v[u] - (int32_t)r0) >> sb], 1);
    }
    __syncthreads();
    if (t < 64) {  // one wave scans the 64 sub-bucket counts
        const int32_t v = hist[t];
        int32_t incl = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t x = __shfl_up(incl, o, 64);
            if (t >= o) incl += x;
        }
        cursor[t] = incl - v;  // relative to e0
        W.tp_sub[(int64_t)b * kTpSub + t] = e0 + incl - v;
    }
    __syncthreads();
    for (int64_t t0 = e0; t0 < e1; t0 += kTpTile) {
        const int32_t len = (int32_t)((t0 + kTpTile < e1) ? kTpTile : e1 - t0);
        if (t < kTpSub) hist[t] = 0;
        __syncthreads();
        int32_t sl[4], co[4], ps[4], rk[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {  // loads first, indices clamped into the tile
            const int32_t x = t + 1024 * u;
            const int64_t xc = t0 + (x < len ? x : len - 1);
            sl[u] = W.tp_row[xc];
            co[u] = PACK ? 0 : W.tp_col[xc];
            ps[u] = POS ? W.tp_pos[xc] : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)  // rank -1: past the tile
            rk[u] = (t + 1024 * u < len)
                        ? atomicAdd(&hist[(PACK ? tp_local(sl[u], rb) : sl[u] - (int32_t)r0) >> sb], 1)
                        : -1;
        __syncthreads();
        if (t < 64) {
            const int32_t v = hist[t];
            int32_t incl = v;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int32_t x = __shfl_up(incl, o, 64);
                if (t >= o) incl += x;
            }
            start[t] = incl - v;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (rk[u] >= 0) {
                const int32_t x = start[(PACK ? tp_local(sl[u], rb) : sl[u] - (int32_t)r0) >> sb] + rk[u];
                s_slot[x] = sl[u];
                if (!PACK) s_col[x] = co[u];
                if (POS) s_pos[x] = ps[u];
            }
        }
        __syncthreads();
        for (int32_t x = t; x < len; x += blockDim.x) {
            const int32_t g = (PACK ? tp_local(s_slot[x], rb) : s_slot[x] - (int32_t)r0) >> sb;
            const int64_t q = e0 + cursor[g] + (x - start[g]);
            W.tp_row2[q] = s_slot[x];
            if (!PACK) W.tp_col2[q] = s_col[x];
            if (POS) W.tp_pos2[q] = s_pos[x];
        }
        __syncthreads();
        if (t < kTpSub) cursor[t] += hist[t];
        __syncthreads();
    }
}

// Pass 2 for oversized buckets (more than big_min entries; on skewed
// matrices one bucket can hold a large share of all entries, which one block
// would work through alone): the same split, spread over the whole grid.
// The oversized buckets' entries are cut into kTpTile-entry tiles, numbered
// bucket by bucket; each tile's sub-bucket counts go to a table (a row of
// kTpSub counts per tile), a block per bucket scans the table's columns into
// each tile's place in each sub-bucket, and the tiles are then sorted by
// sub-bucket in LDS and written in runs, as in pass 1.

// The oversized buckets in order, and the number of the first tile of each
// (vt[k], with vt[nbig] the total), built in LDS by every block of NT
// threads (wsum: 2 NT / 64 words); returns nbig.
template <int NT>
__device__ int32_t big_buckets(const int64_t* __restrict__ bstart, int32_t nb, int64_t big_min, int32_t* bk,
                               int32_t* vt, int32_t* wsum) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    constexpr int PER = kTpMaxBuckets / NT;
    int32_t nbig = 0, ntile = 0;
    int32_t flag[PER], tiles[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int32_t b = t * PER + u;
        const int64_t len = b < nb ? bstart[b + 1] - bstart[b] : 0;
        flag[u] = len > big_min ? 1 : 0;
        tiles[u] = flag[u] ? (int32_t)((len + kTpTile - 1) / kTpTile) : 0;
        nbig += flag[u];
        ntile += tiles[u];
    }
    // exclusive scans of (nbig, ntile) over the block, packed as one 64-bit value
    int64_t v = ((int64_t)nbig << 32) | (uint32_t)ntile, incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t x = __shfl_up(incl, o, 64);
        if (lane >= o) incl += x;
    }
    if (lane == 63) {
        wsum[2 * wave] = (int32_t)(incl >> 32);
        wsum[2 * wave + 1] = (int32_t)incl;
    }
    __syncthreads();
    int64_t pre = incl - v;
    for (int w = 0; w < wave; ++w) pre += ((int64_t)wsum[2 * w] << 32) + wsum[2 * w + 1];
    int32_t kb = (int32_t)(pre >> 32), kt = (int32_t)pre;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        if (flag[u]) {
            bk[kb] = t * PER + u;
            vt[kb] = kt;
            ++kb;
            kt += tiles[u];
        }
    }
    int32_t total_b = 0, total_t = 0;
    for (int w = 0; w < NT / 64; ++w) {
        total_b += wsum[2 * w];
        total_t += wsum[2 * w + 1];
    }
    if (t == 0) vt[total_b] = total_t;
    __syncthreads();
    return total_b;
}

// The oversized bucket and the entry range of tile x of the numbering.
__device__ __forceinline__ void big_tile(const int32_t* bk, const int32_t* vt, int32_t nbig, int32_t x,
                                         const int64_t* __restrict__ bstart, int32_t* b, int64_t* e0,
                                         int64_t* e1) {
    int32_t lo = 0, hi = nbig - 1;  // the last k with vt[k] <= x
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (vt[mid] <= x) lo = mid; else hi = mid - 1;
    }
    *b = bk[lo];
    const int64_t s0 = bstart[*b] + (int64_t)(x - vt[lo]) * kTpTile, end = bstart[*b + 1];
    *e0 = s0;
    *e1 = s0 + kTpTile < end ? s0 + kTpTile : end;
}

template <bool PACK>
__global__ __launch_bounds__(256) void k_tp_big_count(Work W, int rb, int32_t nb, const int64_t* __restrict__ bstart,
                                                      int64_t big_min, int32_t* __restrict__ cnt) {
    __shared__ int32_t bk[kTpMaxBuckets], vt[kTpMaxBuckets + 1], wsum[8], hist[kTpSub];
    const int32_t nbig = big_buckets<256>(bstart, nb, big_min, bk, vt, wsum);
    const int sb = rb - 6, t = threadIdx.x;
    for (int32_t x = blockIdx.x; x < vt[nbig]; x += gridDim.x) {
        int32_t b;
        int64_t e0, e1;
        big_tile(bk, vt, nbig, x, bstart, &b, &e0, &e1);
        if (t < kTpSub) hist[t] = 0;
        __syncthreads();
        const int32_t r0 = b << rb;
        for (int64_t e = e0 + t; e < e1; e += 256) {
            const int32_t wd = W.tp_row[e];
            atomicAdd(&hist[(PACK ? tp_local(wd, rb) : wd - r0) >> sb], 1);
        }
        __syncthreads();
        if (t < kTpSub) cnt[(int64_t)x * kTpSub + t] = hist[t];
        __syncthreads();
    }
}

// One block per oversized bucket: 16 parts of its tiles per sub-bucket.
// Each count becomes the place of that tile's run in its bucket.
__global__ __launch_bounds__(1024) void k_tp_big_scan(Work W, int32_t nb, const int64_t* __restrict__ bstart,
                                                      int64_t big_min, int32_t* __restrict__ cnt) {
    __shared__ int32_t bk[kTpMaxBuckets], vt[kTpMaxBuckets + 1], wsum[32];
    __shared__ int32_t part[16][kTpSub];
    const int32_t nbig = big_buckets<1024>(bstart, nb, big_min, bk, vt, wsum);
    const int t = threadIdx.x, sub = t & 63, pt = t >> 6;
    for (int32_t k = blockIdx.x; k < nbig; k += gridDim.x) {
        const int32_t b = bk[k], x0 = vt[k], nt = vt[k + 1] - vt[k];
        const int32_t per = (nt + 15) / 16;
        const int32_t xa = x0 + (pt * per < nt ? pt * per : nt), xb = x0 + ((pt + 1) * per < nt ? (pt + 1) * per : nt);
        int32_t run = 0;
        for (int32_t x = xa; x < xb; ++x) run += cnt[(int64_t)x * kTpSub + sub];
        part[pt][sub] = run;
        __syncthreads();
        if (t < 64) {  // prefix over the parts, then over the sub-buckets
            int32_t acc = 0;
            for (int p = 0; p < 16; ++p) {
                const int32_t c = part[p][t];
                part[p][t] = acc;
                acc += c;
            }
            int32_t incl = acc;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int32_t y = __shfl_up(incl, o, 64);
                if (t >= o) incl += y;
            }
            const int32_t st = incl - acc;
            W.tp_sub[(int64_t)b * kTpSub + t] = bstart[b] + st;
            for (int p = 0; p < 16; ++p) part[p][t] += st;
        }
        __syncthreads();
        run = part[pt][sub];
        for (int32_t x = xa; x < xb; ++x) {
            const int32_t c = cnt[(int64_t)x * kTpSub + sub];
            cnt[(int64_t)x * kTpSub + sub] = run;
            run += c;
        }
        __syncthreads();
    }
}

template <bool POS, bool PACK>
__global__ __launch_bounds__(1024) void k_tp_big_scatter(Csc A, Work W, int rb, int32_t nb,
                                                         const int64_t* __restrict__ bstart, int64_t big_min,
                                                         const int32_t* __restrict__ cnt) {
    __shared__ int32_t bk[kTpMaxBuckets], vt[kTpMaxBuckets + 1], wsum[32];
    __shared__ int32_t s_slot[kTpTile], s_col[PACK ? 1 : kTpTile], s_pos[POS ? kTpTile : 1];
    __shared__ int32_t hist[kTpSub], start[kTpSub];
    const int32_t nbig = big_buckets<1024>(bstart, nb, big_min, bk, vt, wsum);
    const int sb = rb - 6, t = threadIdx.x;
    for (int32_t x = blockIdx.x; x < vt[nbig]; x += gridDim.x) {
        int32_t b;
        int64_t e0, e1;
        big_tile(bk, vt, nbig, x, bstart, &b, &e0, &e1);
        const int32_t len = (int32_t)(e1 - e0), r0 = b << rb;
        if (t < kTpSub) hist[t] = 0;
        __syncthreads();
        int32_t sl[4], co[4], ps[4], rk[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {  // loads first, indices clamped into the tile
            const int32_t y = t + 1024 * u;
            const int64_t yc = e0 + (y < len ? y : len - 1);
            sl[u] = W.tp_row[yc];
            co[u] = PACK ? 0 : W.tp_col[yc];
            ps[u] = POS ? W.tp_pos[yc] : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            rk[u] = (t + 1024 * u < len) ? atomicAdd(&hist[(PACK ? tp_local(sl[u], rb) : sl[u] - r0) >> sb], 1) : -1;
        __syncthreads();
        if (t < 64) {
            const int32_t v = hist[t];
            int32_t incl = v;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int32_t y = __shfl_up(incl, o, 64);
                if (t >= o) incl += y;
            }
            start[t] = incl - v;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (rk[u] >= 0) {
                const int32_t y = start[(PACK ? tp_local(sl[u], rb) : sl[u] - r0) >> sb] + rk[u];
                s_slot[y] = sl[u];
                if (!PACK) s_col[y] = co[u];
                if (POS) s_pos[y] = ps[u];
            }
        }
        __syncthreads();
        for (int32_t y = t; y < len; y += 1024) {
            const int32_t g = (PACK ? tp_local(s_slot[y], rb) : s_slot[y] - r0) >> sb;
            const int64_t q = bstart[b] + cnt[(int64_t)x * kTpSub + g] + (y - start[g]);
            W.tp_row2[q] = s_slot[y];
            if (!PACK) W.tp_col2[q] = s_col[y];
            if (POS) W.tp_pos2[q] = s_pos[y];
        }
        __syncthreads();
    }
}

// Pass 3: one block per sub-bucket (at most 128 slots, a few hundred entries
// on average): count its slots, write their pointers, then sort the entries
// by slot in LDS and write them out contiguously.  A sub-bucket larger than
// one LDS tile (a heavy row) is placed tile by tile, each tile sorted in LDS
// and written as one run per slot.
constexpr int kPlaceTile = 2048;  // entries per LDS tile (256 threads x 8)

template <bool POS, bool PACK>
__global__ __launch_bounds__(256) void k_tp_place(Csc A, Work W, int rb, int32_t nb, int64_t big_sub) {
    constexpr int NS = kTpMaxRows / kTpSub;  // slots per sub-bucket, at most 128
    constexpr int U = kPlaceTile / 256;
    __shared__ int32_t rc[NS], tc[NS], ts[NS];
    __shared__ int32_t s_key[kPlaceTile], s_col[kPlaceTile], s_pos[POS ? kPlaceTile : 1];
    if (W.counters[kErrMatch]) return;  // block-uniform: no slots without a matching
    const int32_t g = blockIdx.x;
    const int32_t b = g / kTpSub, sub = g % kTpSub;
    const int sb = rb - 6;
    const int64_t s0 = ((int64_t)b << rb) + ((int64_t)sub << sb);
    const int64_t s1 = (s0 + ((int64_t)1 << sb) < A.n) ? s0 + ((int64_t)1 << sb) : A.n;
    const int32_t nr = (s1 > s0) ? (int32_t)(s1 - s0) : 0;
    const int64_t e0 = W.tp_sub[g], e1 = W.tp_sub[g + 1];
    const int64_t len = e1 - e0;
    const bool one_tile = len <= kPlaceTile;
    const int t = threadIdx.x;
    if (g == nb * kTpSub - 1 && t == 0) W.rowptr[A.n] = A.nnz;
    if (len > big_sub) {  // block-uniform: the grid-wide placement takes it while its list has room
        __shared__ int32_t s_q;
        if (t == 0) {
            const int32_t q = atomicAdd(&W.counters[kBigSubs], 1);
            if (q < kMaxBigSubs) W.tp_biglist[q] = g;
            s_q = q;
        }
        __syncthreads();
        if (s_q < kMaxBigSubs) return;
    }
    if (t < NS) rc[t] = 0;
    __syncthreads();
    int32_t key[U], col[U], pos[U], rk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) rk[u] = -1;
    for (int64_t c0 = 0; c0 < len; c0 += kPlaceTile) {  // counts (uniform trip count)
        // loads first (indices clamped into the sub-bucket), then the counts
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t x = c0 + t + 256 * u;
            const int64_t xc = e0 + (x < len ? x : len - 1);
            const int32_t wd = W.tp_row2[xc];
            key[u] = PACK ? (tp_local(wd, rb) & ((1 << sb) - 1)) : (int32_t)(wd - s0);
            if (one_tile) {
                col[u] = PACK ? tp_col_of(wd, rb) : W.tp_col2[xc];
                pos[u] = POS ? W.tp_pos2[xc] : 0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) rk[u] = (c0 + t + 256 * u < len) ? atomicAdd(&rc[key[u]], 1) : -1;
    }
    __syncthreads();
    if (t < 64) {  // slot pointers; rc becomes the exclusive starts
        const int32_t a0 = rc[2 * t], a1 = rc[2 * t + 1];
        const int32_t v = a0 + a1;
        int32_t incl = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t x = __shfl_up(incl, o, 64);
            if (t >= o) incl += x;
        }
        const int32_t ex = incl - v;
        rc[2 * t] = ex;
        rc[2 * t + 1] = ex + a0;
        if (2 * t < nr) {
            W.rowptr[s0 + 2 * t] = e0 + ex;
            W.rsl[s0 + 2 * t] = make_int2((int32_t)(e0 + ex), a0);
        }
        if (2 * t + 1 < nr) {
            W.rowptr[s0 + 2 * t + 1] = e0 + ex + a0;
            W.rsl[s0 + 2 * t + 1] = make_int2((int32_t)(e0 + ex + a0), a1);
        }
        if (W.rtab) {  // the whole first wave: the long lists' hash tables
            rowset_note(W, (int32_t)(s0 + 2 * t), 2 * t < nr ? rowset_take(W, a0, A.nnz) : -1, 2 * t < nr);
            rowset_note(W, (int32_t)(s0 + 2 * t + 1), 2 * t + 1 < nr ? rowset_take(W, a1, A.nnz) : -1,
                        2 * t + 1 < nr);
        }
    }
    __syncthreads();
    if (one_tile) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (rk[u] >= 0) {
                const int32_t d = rc[key[u]] + rk[u];
                s_col[d] = col[u];
                if (POS) s_pos[d] = pos[u];
            }
        }
        __syncthreads();
        for (int32_t x = t; x < (int32_t)len; x += 256) {
            W.colidx[e0 + x] = s_col[x];
            if (POS) W.cscpos[e0 + x] = s_pos[x];
        }
        return;
    }
    for (int64_t c0 = 0; c0 < len; c0 += kPlaceTile) {
        const int32_t tl = (int32_t)((len - c0 < kPlaceTile) ? len - c0 : kPlaceTile);
        if (t < NS) tc[t] = 0;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < U; ++u) {  // loads first, indices clamped into the tile
            const int32_t x = t + 256 * u;
            const int64_t xc = e0 + c0 + (x < tl ? x : tl - 1);
            const int32_t wd = W.tp_row2[xc];
            key[u] = PACK ? (tp_local(wd, rb) & ((1 << sb) - 1)) : (int32_t)(wd - s0);
            col[u] = PACK ? tp_col_of(wd, rb) : W.tp_col2[xc];
            pos[u] = POS ? W.tp_pos2[xc] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) rk[u] = (t + 256 * u < tl) ? atomicAdd(&tc[key[u]], 1) : -1;
        __syncthreads();
        if (t < NS) ts[t] = tc[t];
        __syncthreads();
        wave_scan128(ts);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (rk[u] >= 0) {
                const int32_t d = ts[key[u]] + rk[u];
                s_key[d] = key[u];
                s_col[d] = col[u];
                if (POS) s_pos[d] = pos[u];
            }
        }
        __syncthreads();
        for (int32_t x = t; x < tl; x += 256) {
            const int32_t k = s_key[x];
            const int64_t dst = e0 + rc[k] + (x - ts[k]);
            W.colidx[dst] = s_col[x];
            if (POS) W.cscpos[dst] = s_pos[x];
        }
        __syncthreads();
        if (t < NS) rc[t] += tc[t];
        __syncthreads();
    }
}

// Pass 3 for oversized sub-buckets (more than big_sub entries, listed by
// k_tp_place: the hub rows of skewed matrices, which one block would place
// alone, tile after tile): the same placement spread over the grid, in the
// pass-1 scheme.  The listed sub-buckets' entries are cut into kTpTile-entry
// tiles, numbered sub-bucket by sub-bucket; each tile's slot counts go to a
// table (kSubSlots per tile), a block per sub-bucket scans the table's
// columns into each tile's place in each slot's list (and writes the slot
// pointers), and the tiles are then sorted by slot in LDS and written in
// runs.
constexpr int kSubSlots = kTpMaxRows / kTpSub;  // slots per sub-bucket, at most 128

// The listed sub-buckets and the number of the first tile of each (vt[k],
// vt[nl] the total), built in LDS by every block of NT threads (wsum: 2 NT /
// 64 words); returns nl.
template <int NT>
__device__ int32_t big_subs(const Work& W, int32_t* gk, int32_t* vt, int32_t* wsum) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    constexpr int PER = kMaxBigSubs / NT;
    const int32_t listed = W.counters[kBigSubs];
    const int32_t nl = listed < kMaxBigSubs ? listed : kMaxBigSubs;
    int32_t tiles[PER], ntile = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int32_t k = t * PER + u;
        int32_t c = 0;
        if (k < nl) {
            const int32_t g = W.tp_biglist[k];
            gk[k] = g;
            c = (int32_t)((W.tp_sub[g + 1] - W.tp_sub[g] + kTpTile - 1) / kTpTile);
        }
        tiles[u] = c;
        ntile += c;
    }
    int32_t incl = ntile;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t x = __shfl_up(incl, o, 64);
        if (lane >= o) incl += x;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int32_t pre = incl - ntile;
    for (int w = 0; w < wave; ++w) pre += wsum[w];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int32_t k = t * PER + u;
        if (k < nl) vt[k] = pre;
        pre += tiles[u];
    }
    int32_t total = 0;
    for (int w = 0; w < NT / 64; ++w) total += wsum[w];
    if (t == 0) vt[nl] = total;
    __syncthreads();
    return nl;
}

// The listed sub-bucket of tile x, its number in the list and the tile's
// entry range.
__device__ __forceinline__ void sub_tile(const Work& W, const int32_t* gk, const int32_t* vt, int32_t nl, int32_t x,
                                         int32_t* k, int32_t* g, int64_t* e0, int64_t* e1) {
    int32_t lo = 0, hi = nl - 1;  // the last k with vt[k] <= x
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (vt[mid] <= x) lo = mid; else hi = mid - 1;
    }
    *k = lo;
    *g = gk[lo];
    const int64_t s = W.tp_sub[*g] + (int64_t)(x - vt[lo]) * kTpTile, end = W.tp_sub[*g + 1];
    *e0 = s;
    *e1 = s + kTpTile < end ? s + kTpTile : end;
}

// The slot of a placed word within its sub-bucket.
template <bool PACK>
__device__ __forceinline__ int32_t sub_key(int32_t wd, int rb, int64_t s0) {
    const int sb = rb - 6;
    return PACK ? (tp_local(wd, rb) & ((1 << sb) - 1)) : (int32_t)(wd - s0);
}

__device__ __forceinline__ int64_t sub_first_slot(int32_t g, int rb) {
    return ((int64_t)(g / kTpSub) << rb) + ((int64_t)(g % kTpSub) << (rb - 6));
}

template <bool PACK>
__global__ __launch_bounds__(256) void k_tp_sbig_count(Work W, int rb, int32_t* __restrict__ cnt) {
    __shared__ int32_t gk[kMaxBigSubs], vt[kMaxBigSubs + 1], wsum[4], hist[kSubSlots];
    const int32_t nl = big_subs<256>(W, gk, vt, wsum);
    const int t = threadIdx.x;
    for (int32_t x = blockIdx.x; x < vt[nl]; x += gridDim.x) {
        int32_t k, g;
        int64_t e0, e1;
        sub_tile(W, gk, vt, nl, x, &k, &g, &e0, &e1);
        const int64_t s0 = sub_first_slot(g, rb);
        if (t < kSubSlots) hist[t] = 0;
        __syncthreads();
        for (int64_t e = e0 + t; e < e1; e += 256) atomicAdd(&hist[sub_key<PACK>(W.tp_row2[e], rb, s0)], 1);
        __syncthreads();
        if (t < kSubSlots) cnt[(int64_t)x * kSubSlots + t] = hist[t];
        __syncthreads();
    }
}

// One block per listed sub-bucket: 8 parts of its tiles per slot.  Each
// count becomes the place of that tile's run in the sub-bucket; the slot
// pointers (and the long lists' tables) are recorded as k_tp_place does.
__global__ __launch_bounds__(1024) void k_tp_sbig_scan(Csc A, Work W, int rb, int32_t* __restrict__ cnt) {
    __shared__ int32_t gk[kMaxBigSubs], vt[kMaxBigSubs + 1], wsum[16];
    __shared__ int32_t part[8][kSubSlots], tot[kSubSlots];
    const int32_t nl = big_subs<1024>(W, gk, vt, wsum);
    const int t = threadIdx.x, slot = t % kSubSlots, pt = t / kSubSlots;
    for (int32_t k = blockIdx.x; k < nl; k += gridDim.x) {  // block-uniform
        const int32_t g = gk[k], x0 = vt[k], nt = vt[k + 1] - vt[k];
        const int64_t e0 = W.tp_sub[g], s0 = sub_first_slot(g, rb);
        const int64_t s1 = s0 + ((int64_t)1 << (rb - 6)) < A.n ? s0 + ((int64_t)1 << (rb - 6)) : A.n;
        const int32_t nr = s1 > s0 ? (int32_t)(s1 - s0) : 0;
        const int32_t per = (nt + 7) / 8;
        const int32_t xa = x0 + (pt * per < nt ? pt * per : nt), xb = x0 + ((pt + 1) * per < nt ? (pt + 1) * per : nt);
        int32_t run = 0;
        for (int32_t x = xa; x < xb; ++x) run += cnt[(int64_t)x * kSubSlots + slot];
        part[pt][slot] = run;
        __syncthreads();
        int32_t total = 0;  // the slot's entries (threads t < kSubSlots)
        if (t < kSubSlots) {  // prefix over the parts
            for (int p = 0; p < 8; ++p) {
                const int32_t c = part[p][t];
                part[p][t] = total;
                total += c;
            }
            tot[t] = total;
        }
        __syncthreads();
        wave_scan128(tot);  // the slots' starts in the sub-bucket
        __syncthreads();
        if (t < kSubSlots) {  // two whole waves
            const int32_t st = tot[t];
            if (t < nr) {
                W.rowptr[s0 + t] = e0 + st;
                W.rsl[s0 + t] = make_int2((int32_t)(e0 + st), total);
            }
            if (W.rtab) rowset_note(W, (int32_t)(s0 + t), t < nr ? rowset_take(W, total, A.nnz) : -1, t < nr);
            for (int p = 0; p < 8; ++p) part[p][t] += st;
        }
        __syncthreads();
        run = part[pt][slot];
        for (int32_t x = xa; x < xb; ++x) {
            const int32_t c = cnt[(int64_t)x * kSubSlots + slot];
            cnt[(int64_t)x * kSubSlots + slot] = run;
            run += c;
        }
        __syncthreads();
    }
}

template <bool POS, bool PACK>
__global__ __launch_bounds__(1024) void k_tp_sbig_scatter(Csc A, Work W, int rb, const int32_t* __restrict__ cnt) {
    __shared__ int32_t gk[kMaxBigSubs], vt[kMaxBigSubs + 1], wsum[16];
    __shared__ int32_t s_key[kTpTile], s_col[kTpTile], s_pos[POS ? kTpTile : 1];
    __shared__ int32_t hist[kSubSlots], start[kSubSlots];
    const int32_t nl = big_subs<1024>(W, gk, vt, wsum);
    const int t = threadIdx.x;
    for (int32_t x = blockIdx.x; x < vt[nl]; x += gridDim.x) {  // block-uniform
        int32_t k, g;
        int64_t e0, e1;
        sub_tile(W, gk, vt, nl, x, &k, &g, &e0, &e1);
        const int64_t s0 = sub_first_slot(g, rb), base = W.tp_sub[g];
        const int32_t len = (int32_t)(e1 - e0);
        if (t < kSubSlots) hist[t] = 0;
        __syncthreads();
        int32_t key[4], col[4], pos[4], rk[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {  // loads first, indices clamped into the tile
            const int32_t y = t + 1024 * u;
            const int64_t yc = e0 + (y < len ? y : len - 1);
            const int32_t wd = W.tp_row2[yc];
            key[u] = sub_key<PACK>(wd, rb, s0);
            col[u] = PACK ? tp_col_of(wd, rb) : W.tp_col2[yc];
            pos[u] = POS ? W.tp_pos2[yc] : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) rk[u] = (t + 1024 * u < len) ? atomicAdd(&hist[key[u]], 1) : -1;
        __syncthreads();
        if (t < kSubSlots) start[t] = hist[t];
        __syncthreads();
        wave_scan128(start);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (rk[u] >= 0) {
                const int32_t y = start[key[u]] + rk[u];
                s_key[y] = key[u];
                s_col[y] = col[u];
                if (POS) s_pos[y] = pos[u];
            }
        }
        __syncthreads();
        for (int32_t y = t; y < len; y += 1024) {
            const int32_t kk = s_key[y];
            const int64_t dst = base + cnt[(int64_t)x * kSubSlots + kk] + (y - start[kk]);
            W.colidx[dst] = s_col[y];
            if (POS) W.cscpos[dst] = s_pos[y];
        }
        __syncthreads();
    }
}

// Pass 1b (scatter) in one of its forms; S tiles per part of the column scan.
template <bool POS, bool PACK>
void launch_tp_scatter(const Csc& A, const Work& W, const TpPlan& P, int32_t S, hipStream_t s) {
    const int32_t nb = (int32_t)P.nb, nseg = (int32_t)P.nseg;
    constexpr int NT = kTpScatterThreads;
    if (nb <= 256)
        hipLaunchKernelGGL((k_tp_scatter<POS, NT, 256, PACK>), dim3(nseg), dim3(NT), 0, s, A, W, P.rb, nb, S, W.tp_off,
                           W.tp_cnt, W.tp_bstart);
    else
        hipLaunchKernelGGL((k_tp_scatter<POS, NT, kTpMaxBuckets, PACK>), dim3(nseg), dim3(NT), 0, s, A, W, P.rb, nb, S,
                           W.tp_off, W.tp_cnt, W.tp_bstart);
}

// Passes 2 and 3 (split, place); with big, buckets of more than kBigBucket
// entries are split, and sub-buckets of more than kBigSub placed, by the
// whole grid.
constexpr int64_t kBigBucket = (int64_t)1 << 17;
constexpr int64_t kBigSub = (int64_t)1 << 16;

template <bool POS, bool PACK>
void launch_tp_rest(const Csc& A, const Work& W, const TpPlan& P, bool big, hipStream_t s, int cus) {
    const int32_t nb = (int32_t)P.nb;
    const int64_t big_min = big ? kBigBucket : INT64_MAX;
    hipLaunchKernelGGL((k_tp_split<POS, PACK>), dim3(nb), dim3(1024), 0, s, A, W, P.rb, nb, W.tp_bstart, big_min);
    if (big) {
        hipLaunchKernelGGL(k_tp_big_count<PACK>, dim3(cus * 4), dim3(256), 0, s, W, P.rb, nb, W.tp_bstart, big_min,
                           W.tp_bigcnt);
        hipLaunchKernelGGL(k_tp_big_scan, dim3(cus), dim3(1024), 0, s, W, nb, W.tp_bstart, big_min, W.tp_bigcnt);
        hipLaunchKernelGGL((k_tp_big_scatter<POS, PACK>), dim3(cus * 2), dim3(1024), 0, s, A, W, P.rb, nb,
                           W.tp_bstart, big_min, W.tp_bigcnt);
    }
    hipLaunchKernelGGL((k_tp_place<POS, PACK>), dim3(nb * kTpSub), dim3(256), 0, s, A, W, P.rb, nb,
                       big ? kBigSub : INT64_MAX);
    if (big) {
        hipLaunchKernelGGL(k_tp_sbig_count<PACK>, dim3(cus * 4), dim3(256), 0, s, W, P.rb, W.tp_bigcnt);
        hipLaunchKernelGGL(k_tp_sbig_scan, dim3(cus), dim3(1024), 0, s, A, W, P.rb, W.tp_bigcnt);
        hipLaunchKernelGGL((k_tp_sbig_scatter<POS, PACK>), dim3(cus * 2), dim3(1024), 0, s, A, W, P.rb, W.tp_bigcnt);
    }
}

hipError_t launch_transpose_buckets(const Csc& A, const Work& W, bool positions, hipStream_t s, int cus) {
    const TpPlan P = tp_plan(A.n, A.nnz);
    const int32_t nb = (int32_t)P.nb, nseg = (int32_t)P.nseg;
    hipLaunchKernelGGL(k_tp_tile_cols, dim3(cus * 8), dim3(256), 0, s, A, W, nseg);
    hipLaunchKernelGGL(k_tp_hist, dim3(nseg), dim3(256), 0, s, A, W, P.rb, nb, nseg, W.tp_cnt);
    // column scan in parts of S tiles (about 128 parts)
    const int32_t S = nseg / 128 + 1 > 32 ? nseg / 128 + 1 : 32;
    const int32_t nparts = (nseg + S - 1) / S;
    hipLaunchKernelGGL(k_tp_colsum, dim3(nparts), dim3(256), 0, s, W.tp_cnt, nb, nseg, S, W.tp_off);
    hipLaunchKernelGGL(k_tp_colscan, dim3(nb), dim3(64), 0, s, W.tp_off, nb, nparts, W.tp_btot, W.tp_bstart, A.nnz,
                       W.counters + kColDone);
    // a slot's offset in its bucket and a column share one word when they fit
    const bool pack = (int64_t)A.n <= ((int64_t)1 << (32 - P.rb));
    if (positions) {
        if (pack) launch_tp_scatter<true, true>(A, W, P, S, s);
        else launch_tp_scatter<true, false>(A, W, P, S, s);
    } else {
        if (pack) launch_tp_scatter<false, true>(A, W, P, S, s);
        else launch_tp_scatter<false, false>(A, W, P, S, s);
    }
    return hipGetLastError();
}

hipError_t launch_transpose_rest(const Csc& A, const Work& W, bool positions, bool big, hipStream_t s, int cus) {
    const TpPlan P = tp_plan(A.n, A.nnz);
    const bool pack = (int64_t)A.n <= ((int64_t)1 << (32 - P.rb));
    if (positions) {
        if (pack) launch_tp_rest<true, true>(A, W, P, big, s, cus);
        else launch_tp_rest<true, false>(A, W, P, big, s, cus);
    } else {
        if (pack) launch_tp_rest<false, true>(A, W, P, big, s, cus);
        else launch_tp_rest<false, false>(A, W, P, big, s, cus);
    }
    return hipGetLastError();
}

// Hash tables of the long row lists.  A row list never changes during a call
// (a flip moves it from one slot to another), so every list longer than
// kRowSetMin entries gets, once, a table in global memory mapping each of its
// columns to its place in the list (size pow2 >= 2 x length, load <= 1/2:
// the keys, then the values), and the probes of its roots find the closing
// edge with a load or two (and its CSC position through the list's stored
// positions) instead of a binary search of column m_i.  rtab[j] locates the
// table of the list at slot j and moves with rsl.  The tables take their
// words from a pool of nnz + 64 words, first come first served; a list that
// finds no room keeps rtab = -1 and the binary search.
struct GlobalCas32 {
    __device__ int32_t operator()(int32_t* p, int32_t e, int32_t d) const { return atomicCAS(p, e, d); }
};

// The long lists' tables are filled by the whole grid in units of kRowUnit
// (keys to clear, then entries to insert): one block lays out the units (a
// scan over the listed rows), and every block takes a contiguous range of
// units, finding its first list once by binary search.  The plan holds, per
// listed row q, the first clear unit, the first insert unit (each with the
// total after the last row) and the table's place in the pool: the inserts
// never read the table's place from rtab, which a failed insert clears.
constexpr int32_t kRowUnit = 2048;

__device__ __forceinline__ uint32_t rowset_size(int32_t len) {
    uint32_t size = 64;
    while ((int32_t)size < 2 * len) size <<= 1;
    return size;
}

__global__ __launch_bounds__(1024) void k_rowset_plan(Work W) {
    __shared__ int32_t wsum[32], carry[2];
    const int32_t nr = W.counters[kTabRows];
    int32_t* const cst = W.tab_plan;
    int32_t* const ist = cst + (nr + 1);
    int32_t* const toff = ist + (nr + 1);
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    if (t == 0) carry[0] = carry[1] = 0;
    __syncthreads();
    for (int32_t base = 0; base < nr; base += 1024) {  // block-uniform
        const int32_t q = base + t;
        int32_t cu = 0, iu = 0;
        if (q < nr) {
            const int32_t j = W.medium[q];
            const int32_t len = W.rsl[j].y;
            cu = (int32_t)(rowset_size(len) / kRowUnit);
            iu = (len + kRowUnit - 1) / kRowUnit;
            toff[q] = W.rtab[j];
        }
        const int64_t v = ((int64_t)cu << 32) | (uint32_t)iu;
        int64_t incl = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t x = __shfl_up(incl, o, 64);
            if (lane >= o) incl += x;
        }
        if (lane == 63) {
            wsum[2 * wave] = (int32_t)(incl >> 32);
            wsum[2 * wave + 1] = (int32_t)incl;
        }
        __syncthreads();
        int64_t pre = incl - v;
        for (int w = 0; w < wave; ++w) pre += ((int64_t)wsum[2 * w] << 32) + wsum[2 * w + 1];
        if (q < nr) {
            cst[q] = carry[0] + (int32_t)(pre >> 32);
            ist[q] = carry[1] + (int32_t)pre;
        }
        __syncthreads();
        if (t == 0) {
            for (int w = 0; w < 16; ++w) {
                carry[0] += wsum[2 * w];
                carry[1] += wsum[2 * w + 1];
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        cst[nr] = carry[0];
        ist[nr] = carry[1];
    }
}

// The last listed row whose first unit is at most u (first[0] = 0 <= u).
__device__ __forceinline__ int32_t rowset_row_of(const int32_t* first, int32_t nr, int32_t u) {
    int32_t lo = 0, hi = nr - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (first[mid] <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// fill = 0: clear the keys; fill = 1: insert the entries.
__global__ __launch_bounds__(256) void k_rowset_fill(Work W, int fill) {
    const int32_t nr = W.counters[kTabRows];
    if (nr == 0) return;
    const int32_t* const cst = W.tab_plan;
    const int32_t* const ist = cst + (nr + 1);
    const int32_t* const toff = ist + (nr + 1);
    const int32_t* const first = fill ? ist : cst;
    const int32_t total = first[nr];
    const int32_t per = (total + (int32_t)gridDim.x - 1) / (int32_t)gridDim.x;
    const int32_t u0 = (int32_t)blockIdx.x * per, u1 = u0 + per < total ? u0 + per : total;
    if (u0 >= u1) return;
    int32_t q = rowset_row_of(first, nr, u0);
    for (int32_t u = u0; u < u1; ++u) {  // block-uniform
        while (first[q + 1] <= u) ++q;
        const int32_t j = W.medium[q];
        int32_t* const tab = W.tabs + toff[q];
        const int32_t off = (u - first[q]) * kRowUnit;
        if (!fill) {
            for (int32_t x = threadIdx.x; x < kRowUnit; x += blockDim.x) tab[off + x] = -1;
            continue;
        }
        const int2 rl = W.rsl[j];
        const uint32_t size = rowset_size(rl.y);
        const int32_t end = off + kRowUnit < rl.y ? off + kRowUnit : rl.y;
        bool ok = true;
        for (int32_t x = off + threadIdx.x; x < end; x += blockDim.x)
            ok &= hash_insert(tab, tab + size, W.colidx[rl.x + x], x, size - 1, GlobalCas32{});
        // a list the table cannot take (impossible with a well-formed CSC)
        // keeps the binary search
        if (!ok) W.rtab[j] = -1;
    }
}

hipError_t launch_rowsets(const Csc& A, const Work& W, hipStream_t s, int cus) {
    if (!W.rtab) return hipSuccess;
    hipLaunchKernelGGL(k_rowset_plan, dim3(1), dim3(1024), 0, s, W);
    hipLaunchKernelGGL(k_rowset_fill, dim3(cus * 4), dim3(256), 0, s, W, 0);
    hipLaunchKernelGGL(k_rowset_fill, dim3(cus * 4), dim3(256), 0, s, W, 1);
    return hipGetLastError();
}

bool transpose_in_buckets(int64_t n, int64_t nnz) { return tp_plan(n, nnz).ok; }

hipError_t launch_transpose(const Csc& A, const Work& W, int32_t long_threshold, bool has_long,
                            bool positions, hipStream_t s, int cus) {
    const int64_t n = A.n;
    hipError_t e;
    if (tp_plan(A.n, A.nnz).ok) {
        // also fills mrk
        if ((e = launch_transpose_buckets(A, W, positions, s, cus)) != hipSuccess) return e;
        if ((e = launch_transpose_rest(A, W, positions, has_long, s, cus)) != hipSuccess) return e;
        return launch_rowsets(A, W, s, cus);
    } else {
        // very large matrices: counting sort with global atomics
        if ((e = hipMemsetAsync(W.rowcnt, 0, (size_t)n * sizeof(int32_t), s)) != hipSuccess) return e;
        if (A.nnz > 0) hipLaunchKernelGGL(k_row_count, dim3(cus * 8), dim3(256), 0, s, A, W.mr, W.rowcnt);
        const int64_t nb = (n + 2047) / 2048;
        hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(256), 0, s, W.rowcnt, n, W.rowptr,
                           W.scan_sums);
        hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, W.scan_sums, nb, W.rowptr + n);
        hipLaunchKernelGGL(k_scan_add, dim3(cus * 8), dim3(256), 0, s, W.rowptr, n, W.scan_sums);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipMemsetAsync(W.rowcnt, 0, (size_t)n * sizeof(int32_t), s)) != hipSuccess) return e;
        const unsigned blocks = (unsigned)((n * 16 + 255) / 256);
        hipLaunchKernelGGL(k_row_fill_short<16>, dim3(blocks), dim3(256), 0, s, A, W, long_threshold);
        if (has_long) hipLaunchKernelGGL(k_row_fill_long, dim3(cus * 8), dim3(256), 0, s, A, W);
        hipLaunchKernelGGL(k_slot_ptrs, dim3(cus * 8), dim3(256), 0, s, A, W);
    }
    if (A.nnz > 0) hipLaunchKernelGGL(k_mrk_fill, dim3(cus * 8), dim3(256), 0, s, A, W);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_rowsets(A, W, s, cus);
}

// After the flips of a round: the entries of every row whose mate changed get
// the new mate column (one block per flipped row; the rows with more than
// kHeavyRow entries, which k_apply lists, then eight at a time, each over
// an eighth of the grid).  In incremental mode the columns of those entries are marked
// for the next round: a root's Step-C result can change only if its own mate
// changed or one of its rows got a new mate (every value its gains read is
// otherwise the same), and the flipped columns themselves appear in the
// lists of their new rows.

__device__ __forceinline__ void refresh_entry(const Csc& A, const Work& W, int64_t x, int32_t m, int32_t row,
                                              int incremental, int next) {
    // entry {row, colidx[x]}: its CSC position is stored, or searched for
    const int64_t pos = W.cscpos ? (int64_t)W.cscpos[x] : find_row(A.col_ptr, A.row_idx, W.colidx[x], row);
    W.mrk[pos] = m;
    if (incremental) {
        const int32_t c = W.colidx[x];
        const bool first = __hip_atomic_load(&W.dirty[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
                           atomicExch(&W.dirty[c], 1) == 0;
        const int32_t q = wave_append(&W.counters[slot_word(next, kRoots)], first);
        if (first) W.dirty_list[q] = c;
    }
}

__global__ __launch_bounds__(256) void k_mrk_update(Csc A, Work W, int slot, int incremental) {
    if (round_over(W)) return;
    const int64_t nf = 2 * (int64_t)W.counters[slot_word(slot, kApplied)];
    const int next = (slot + 1) % kSlots;
    for (int64_t f = blockIdx.x; f < nf; f += gridDim.x) {
        const int32_t m = W.flips[2 * f + 1];   // new mate column of the flipped row
        const int2 rl = W.rsl[m];
        const int64_t b = rl.x;
        const int32_t len = rl.y;
        if (len > kHeavyRow) continue;  // block-uniform: below
        const int32_t row = W.mc[m];  // the row now matched to m owns the list
        for (int64_t x = b + threadIdx.x; x < b + len; x += blockDim.x)
            refresh_entry(A, W, x, m, row, incremental, next);
    }
    // the heavy rows: G groups of blocks, group g taking rows g, g + G, ...
    const int32_t nh = W.counters[slot_word(slot, kHeavy)];
    const int32_t G = gridDim.x >= 8 ? 8 : 1, ng = gridDim.x / G;
    const int32_t grp = blockIdx.x % G, gb = blockIdx.x / G;
    if (gb >= ng) return;
    const int64_t stride = (int64_t)ng * blockDim.x;
    for (int32_t h = grp; h < nh; h += G) {
        const int32_t m = W.heavy[h];
        const int2 rl = W.rsl[m];
        const int64_t b = rl.x, e = b + rl.y;
        const int32_t row = W.mc[m];
        for (int64_t x = b + (int64_t)gb * blockDim.x + threadIdx.x; x < e; x += stride)
            refresh_entry(A, W, x, m, row, incremental, next);
    }
}

// End of a round: record its statistics and, if it flipped nothing, raise
// the device flag that turns every later round kernel into a no-op (the
// loop's exit test of Algorithm 2, taken on the device so that the host can
// queue several rounds between two looks at the flag).
// The round's index is read on the device (rounds run so far), so that the
// same launches serve every batch of rounds with the same ring slots.
__global__ void k_round_end(Work W, int slot, int listed, int32_t n) {
    if (round_over(W)) return;
    const int32_t round = W.counters[kRoundsRun];
    const int32_t cand = W.counters[slot_word(slot, kCand)];
    const int32_t applied = W.counters[slot_word(slot, kApplied)];
    if (round < kMaxRoundStats) {
        W.round_stats[round] = cand;
        W.round_stats[kMaxRoundStats + round] = applied;
        W.round_stats[2 * kMaxRoundStats + round] = listed ? W.counters[slot_word(slot, kRoots)] : n;
    }
    *reinterpret_cast<unsigned long long*>(W.counters + kCycles) += (unsigned long long)applied;
    W.counters[kRoundsRun] = round + 1;
    if (applied == 0) W.counters[kDone] = cand > 0 ? 2 : 1;
}

hipError_t launch_round_end(const Work& W, int slot, bool listed, int32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_round_end, dim3(1), dim3(1), 0, s, W, slot, listed ? 1 : 0, n);
    return hipGetLastError();
}

hipError_t launch_mrk_update(const Csc& A, const Work& W, int slot, bool incremental, hipStream_t s, int cus) {
    hipLaunchKernelGGL(k_mrk_update, dim3(cus * 4), dim3(256), 0, s, A, W, slot, incremental ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Total weight: a perfect binary tree over the values padded with +0.0 to a
// power of two, pairs (2t, 2t+1) at every level.  A block sums an aligned run
// of kTreeBlock = 2048 leaves (exactly one subtree); the block sums form the
// next level, and the last level (<= 2048 values) runs in one block over
// exactly next_pow2(m) leaves.

__global__ __launch_bounds__(256) void k_tree_block(const double* __restrict__ x, int64_t m,
                                                    double* __restrict__ out, const int32_t* __restrict__ gate) {
    __shared__ double part[4];
    if (gate && *gate == 0) return;  // a gated sum runs only once the rounds have ended
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
                                                     double* __restrict__ out, const int32_t* __restrict__ gate) {
    __shared__ double a[kTreeBlock], b[kTreeBlock];
    if (gate && *gate == 0) return;
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

hipError_t launch_tree_sum(const double* x, int64_t m, const Work& W, double* out, hipStream_t s,
                           const int32_t* gate) {
    const double* cur = x;
    double* bufs[2] = {W.tree_a, W.tree_b};
    int which = 0;
    while (m > kTreeBlock) {
        const int64_t blocks = (m + kTreeBlock - 1) / kTreeBlock;
        hipLaunchKernelGGL(k_tree_block, dim3((unsigned)blocks), dim3(256), 0, s, cur, m, bufs[which], gate);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        cur = bufs[which];
        which ^= 1;
        m = blocks;
    }
    hipLaunchKernelGGL(k_tree_final, dim3(1), dim3(1024), 0, s, cur, m, out, gate);
    return hipGetLastError();
}

// dst[0..n) = src[0..n) once *gate is 1 (the output copy queued behind a
// batch of rounds before the host knows whether the batch ended them; the
// done flag is 1 when the rounds ended normally, 2 on a failed consistency
// check, after which the caller's output must stay untouched).
__global__ __launch_bounds__(256) void k_copy_gated(const int32_t* __restrict__ src, int32_t* __restrict__ dst,
                                                    int64_t n, const int32_t* __restrict__ gate) {
    if (*gate != 1) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t launch_copy_gated(const int32_t* src, int32_t* dst, int64_t n, const int32_t* gate, hipStream_t s,
                             int cus) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > (int64_t)cus * 8) blocks = (int64_t)cus * 8;
    hipLaunchKernelGGL(k_copy_gated, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n, gate);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Workspace layout (256-byte aligned sub-arrays).

static inline size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

size_t workspace_layout(int32_t n, int64_t nnz, char* base, Work* out, Mcm* mcm) {
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
    Work W{};
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
    W.chunk_col = (int32_t*)take(max_chunks * 4);
    W.part_g = (double*)take(max_chunks * 8);
    W.part_c = (int32_t*)take(max_chunks * 4);
    W.part_k = (int64_t*)take(max_chunks * 8);
    W.part_p = (int64_t*)take(max_chunks * 8);
    W.tree_a = (double*)take(tree1 * 8);
    W.tree_b = (double*)take(tree1 * 8);
    W.bitmap = (uint32_t*)take((Z + 1) / 32 * 4 + 8);
    // the run's report, read back as one range: result, per-round
    // statistics, then the counters (whose first words are the scalars)
    W.result = (double*)take(4 * 8);
    W.round_stats = (int32_t*)take(3 * kMaxRoundStats * 4);
    W.counters = (int32_t*)take(kCounterWords * 4);
    W.max_chunks = (int64_t)max_chunks;
    W.rowptr = (int64_t*)take((N + 1) * 8);
    W.rsl = (int2*)take(N * 8);
    W.cp32 = (int32_t*)take((N + 1) * 4);
    W.pm = (int32_t*)take(N * 4);
    W.colidx = (int32_t*)take(Z * 4 + 128);
    W.cscpos = (int32_t*)take(Z * 4);
    W.mrk = (int32_t*)take(Z * 4 + 128);
    W.rtab = (int32_t*)take(N * 4);
    W.tabs = (int32_t*)take((Z + 64) * 4);
    W.tab_plan = (int32_t*)take((Z / kRowSetMin + 2) * 3 * 4);
    W.rowcnt = (int32_t*)take(N * 4);
    W.scan_sums = (int64_t*)take((N / 2048 + 2) * 8);
    W.flips = (int32_t*)take(N * 4 * 4 / 2 + 16);
    W.dirty = (int32_t*)take(N * 4);
    W.dirty_list = (int32_t*)take(N * 4);
    W.medium = (int32_t*)take((N + kSpread * 64) * 4);
    W.heavy = (int32_t*)take(N * 4);
    const TpPlan P = tp_plan(n, nnz);
    const size_t tpm = P.ok ? (size_t)(P.nb * P.nseg) : 0;
    const size_t tpz = P.ok ? Z : 0;
    W.tile_col = (int32_t*)take(P.ok ? (size_t)(P.nseg + 1) * 4 : 0);
    W.tp_row = (int32_t*)take(tpz * 4);
    W.tp_col = (int32_t*)take(tpz * 4);
    W.tp_pos = (int32_t*)take(tpz * 4);
    W.tp_cnt = (int32_t*)take(tpm * 4);
    W.tp_off = (int64_t*)take((tpm + 1) * 8);
    W.tp_bstart = (int64_t*)take((kTpMaxBuckets + 1) * 8);
    W.tp_btot = (int64_t*)take(kTpMaxBuckets * 8);
    W.tp_sums = (int64_t*)take((tpm / 2048 + 2) * 8);
    W.tp_row2 = (int32_t*)take(tpz * 4);
    W.tp_col2 = (int32_t*)take(tpz * 4);
    W.tp_pos2 = (int32_t*)take(tpz * 4);
    W.tp_sub = (int64_t*)take(P.ok ? (size_t)(P.nb * 64 + 1) * 8 : 0);
    W.tp_bigcnt = (int32_t*)take(P.ok ? (size_t)(P.nseg + kTpMaxBuckets) * (kTpMaxRows / kTpSub) * 4 : 0);
    W.tp_biglist = (int32_t*)take(P.ok ? (size_t)kMaxBigSubs * 4 : 0);
    Mcm M;
    M.mc = (int32_t*)take(N * 4);
    M.mr = (int32_t*)take(N * 4);
    M.prop_row = (int32_t*)take(N * 4);
    M.prop_w = (double*)take(N * 8);
    M.rkey = (unsigned long long*)take(N * 8);
    M.racc = (int32_t*)take(N * 4);
    M.list = (int32_t*)take(N * 4);
    M.tree_row = (int32_t*)take(N * 4);
    M.tree_col = (int32_t*)take(N * 4);
    M.parent = (int32_t*)take(N * 4);
    M.end_row = (int32_t*)take(N * 4);
    M.pkey = (unsigned long long*)take(N * 8);
    M.touched = (int32_t*)take(N * 4);
    M.front_a = (int32_t*)take(N * 4);
    M.front_b = (int32_t*)take(N * 4);
    M.level = (int32_t*)take(N * 4);
    M.counters = (int32_t*)take(kMcmWords * 4);
    if (mcm) *mcm = M;
    W.mat_of_col = nullptr;
    W.item_flag = nullptr;
    W.item_cycles = nullptr;
    if (out) *out = W;
    return off;
}

}  // namespace hwpm
