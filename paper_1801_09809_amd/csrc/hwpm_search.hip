// HIP kernels of Steps A-C (arXiv 1801.09809, Section 5.3): for every root
// column j, every row i > m_j of column j and its closing edge {m_j, m_i},
// the gain of the alternating 4-cycle and the per-root winner.  Roots are
// binned by size: a tile of lanes per short root, a wave per medium root, a
// block per 1024-entry chunk of a long column.  Three probes of the closing
// edge give identical results: binary search of column m_i, and the row list
// of m_j from the matching-ordered transpose (per lane, or chunked).
#include "hwpm_device.h"

namespace hwpm {

// ---------------------------------------------------------------------------
// Steps A-C.  Short columns: a tile of T lanes per root column, lanes stride
// over the column (coalesced row_idx reads), each probes its own closing
// edge, the tile reduces to the Step-C winner with cross-lane shuffles.

template <int T>
__global__ __launch_bounds__(256) void k_search_short(Csc A, Work W, int32_t long_threshold,
                                                      int slot) {
    if (round_over(W)) return;
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
// a partial winner; k_merge_long reduces the partials of each column.  With
// the transposed lists and a row list of m_j of at most kLongHashMax entries
// the block first stores that list in an LDS hash table (column -> list
// position) and every probe is one lookup; otherwise each probe binary
// searches row m_j in column m_i.
constexpr int kLongHashMax = 2048;
constexpr int kLongHashSlots = 4096;
constexpr int kLongPre = kLongChunk / 256;  // chunk entries per thread

__global__ __launch_bounds__(256) void k_search_long(Csc A, Work W, int only_dirty, int transposed) {
    __shared__ double sg[4];
    __shared__ int32_t si[4], sc[4];
    __shared__ int64_t sk[4], sp[4];
    __shared__ int32_t hk[kLongHashSlots], hv[kLongHashSlots];
    if (round_over(W)) return;
    const int32_t total = W.counters[kNumChunks];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int32_t cid = blockIdx.x; cid < total; cid += gridDim.x) {
        const int32_t a = W.chunk_col[cid];  // long column of this chunk
        const int32_t j = W.long_list[a];
        if (only_dirty && W.dirty[j] == 0) continue;  // block-uniform: result kept
        const int64_t c0 = A.col_ptr[j];
        const int64_t lo = c0 + (int64_t)(cid - W.chunk_off[a]) * kLongChunk;
        const int64_t hi0 = A.col_ptr[j + 1];
        const int64_t hi = (lo + kLongChunk < hi0) ? lo + kLongChunk : hi0;
        const int32_t mj = W.mc[j];
        const double wmj = W.wm[j];
        Cand b{0.0, INT32_MAX, -1, -1, -1};
        const int32_t rlen = transposed ? W.rlen[j] : INT32_MAX;
        if (rlen <= kLongHashMax) {
            // the chunk's entries (kLongPre per thread) are loaded before the
            // table is built, so that both loads are in flight together
            int32_t iq[kLongPre], mq[kLongPre];
#pragma unroll
            for (int q = 0; q < kLongPre; ++q) {
                const int64_t k = lo + threadIdx.x + 256 * q;
                iq[q] = (k < hi) ? A.row_idx[k] : -1;
                mq[q] = (k < hi) ? W.mrk[k] : -1;
            }
            const int64_t rs = W.rstart[j];
            uint32_t size = 256;
            while ((int32_t)size < 2 * rlen) size <<= 1;
            const uint32_t mask = size - 1;
            for (uint32_t x = threadIdx.x; x < size; x += blockDim.x) hk[x] = -1;
            __syncthreads();
            for (int32_t x = threadIdx.x; x < rlen; x += blockDim.x) {
                const int32_t c = W.colidx[rs + x];
                uint32_t h = hash_col(c, mask);
                while (atomicCAS(&hk[h], -1, c) != -1) h = (h + 1) & mask;  // keys are distinct
                hv[h] = x;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kLongPre; ++q) {
                const int32_t i = iq[q], mi = mq[q];
                if (i <= mj) continue;  // also the slots past the chunk (i = -1)
                const int32_t qx = hash_find(hk, hv, mi, mask);
                if (qx < 0) continue;
                const int64_t k = lo + threadIdx.x + 256 * q;
                const int64_t p = W.cscpos ? (int64_t)W.cscpos[rs + qx] : find_row(A.col_ptr, A.row_idx, mi, mj);
                const double g = (A.w[k] + A.w[p]) - (W.wm[mi] + wmj);
                if (g > 0.0 && better(g, i, b.g, b.i)) {
                    b.g = g; b.i = i; b.c = mi; b.k = k; b.p = p;
                }
            }
        } else {
            // four entries per thread, their binary searches in lockstep
            const int32_t step = blockDim.x;
            for (int64_t k0 = lo + threadIdx.x; k0 < hi; k0 += 4 * (int64_t)step) {
                int32_t iq[4], cq[4], rq[4];
                int64_t pq[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t k = k0 + (int64_t)q * step;
                    iq[q] = (k < hi) ? A.row_idx[k] : -1;
                    cq[q] = (k < hi && iq[q] > mj) ? (transposed ? W.mrk[k] : W.mr[iq[q]]) : -1;
                    rq[q] = mj;
                }
                find_row_x4(A.col_ptr, A.row_idx, cq, rq, pq);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (pq[q] < 0) continue;
                    const int64_t k = k0 + (int64_t)q * step;
                    const double g = (A.w[k] + A.w[pq[q]]) - (W.wm[cq[q]] + wmj);
                    if (g > 0.0 && better(g, iq[q], b.g, b.i)) {
                        b.g = g; b.i = iq[q]; b.c = cq[q]; b.k = k; b.p = pq[q];
                    }
                }
            }
        }
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

__global__ void k_merge_long(Work W, int slot, int only_dirty) {
    if (round_over(W)) return;
    const int32_t nl = W.counters[kNumLong];
    for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nl; q += gridDim.x * blockDim.x) {
        if (only_dirty) {
            if (W.dirty[W.long_list[q]] == 0) continue;
            W.dirty[W.long_list[q]] = 0;
        }
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

// Steps A-C with the transposed probe, the GPU form of the marking trick of
// the sequential algorithm (Section 4): for root j the row list of m_j is
// read once per tile (contiguous) and every probe m_i of the tile is tested
// against it with T cross-lane rotations; the per-entry mate columns m_i are
// streamed from mrk (no gather).  Rows longer than kRowRotate fall back to the
// binary-search probe of column m_i.  Both give the same (hit, position).
constexpr int kRowRotate = 64;

template <int T>
__global__ __launch_bounds__(256) void k_search_rows(Csc A, Work W, int32_t long_threshold,
                                                     int slot) {
    if (round_over(W)) return;
    const int lane = threadIdx.x & (T - 1);
    const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / T;
    if (tile >= A.n) return;  // tile-uniform
    const int32_t j = (int32_t)tile;
    const int64_t lo = A.col_ptr[j], hi = A.col_ptr[j + 1];
    if (hi - lo > long_threshold) return;
    const int32_t mj = W.mc[j];
    const double wmj = W.wm[j];
    const int64_t rs = W.rstart[j];
    const int32_t rlen = W.rlen[j];
    Cand b{0.0, INT32_MAX, -1, -1, -1};
    if (rlen <= kRowRotate) {
        // row list of m_j, T entries per lane-chunk; -1 never equals a column
        int32_t cv0 = (lane < rlen) ? W.colidx[rs + lane] : -1;
        for (int64_t kc = lo; kc < hi; kc += T) {
            const int64_t k = kc + lane;
            int32_t i = -1, mi = -1;
            if (k < hi) {
                i = A.row_idx[k];
                if (i > mj) mi = W.mrk[k];
            }
            int32_t q = -1;
            for (int32_t rc = 0; rc < rlen; rc += T) {
                const int32_t cv = (rc == 0) ? cv0
                                             : ((rc + lane < rlen) ? W.colidx[rs + rc + lane] : -1);
#pragma unroll
                for (int sft = 0; sft < T; ++sft) {
                    const int src = (lane + sft) & (T - 1);
                    const int32_t v = __shfl(cv, src, T);
                    if (mi >= 0 && v == mi) q = rc + src;
                }
            }
            if (q >= 0) {
                const int64_t p = W.cscpos ? (int64_t)W.cscpos[rs + q] : find_row(A.col_ptr, A.row_idx, mi, mj);
                const double g = (A.w[k] + A.w[p]) - (W.wm[mi] + wmj);
                if (g > 0.0 && better(g, i, b.g, b.i)) {
                    b.g = g; b.i = i; b.c = mi; b.k = k; b.p = p;
                }
            }
        }
    } else {
        for (int64_t k = lo + lane; k < hi; k += T) {
            const int32_t i = A.row_idx[k];
            if (i <= mj) continue;
            const int32_t mi = W.mrk[k];
            const int64_t p = find_row(A.col_ptr, A.row_idx, mi, mj);
            if (p < 0) continue;
            const double g = (A.w[k] + A.w[p]) - (W.wm[mi] + wmj);
            if (g > 0.0 && better(g, i, b.g, b.i)) {
                b.g = g; b.i = i; b.c = mi; b.k = k; b.p = p;
            }
        }
    }
    reduce_best<T>(b);
    if (lane == 0) publish(W, j, b, slot);
}

// Steps A-C, transposed probe, chunked form: a tile of T lanes per root, each
// lane holding E entries of column j (i, m_i) and E entries of the row list
// of m_j, so one root of up to T*E entries in both lists is searched with all
// of its loads independent (one memory round trip per stage), and every probe
// is compared with the whole row list through T cross-lane exchanges.  Roots
// with a longer column or row list go to the wave-per-root kernel.
template <int T, int E>
__global__ __launch_bounds__(256) void k_search_chunk(Csc A, Work W, int32_t long_threshold,
                                                      int slot, const int32_t* __restrict__ roots,
                                                      int32_t cap) {
    if (round_over(W)) return;
    const int lane = threadIdx.x & (T - 1);
    // roots: this round's list (its length on the device; the grid covers
    // every column), else every column
    const int64_t ntiles = roots ? W.counters[slot_word(slot, kRoots)] : A.n;
    const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / T;
    if (tile >= ntiles) return;  // tile-uniform
    const int32_t j = roots ? roots[tile] : (int32_t)tile;
    // the root's values are read with its column bounds: one memory round
    // trip instead of two (wasted for the roots that return below).  The
    // empty asm statement takes all six as inputs, so the compiler issues
    // the six loads before it instead of sinking four of them past the
    // branches below (after the bounds' wait).
    const int32_t mj = W.mc[j];
    const double wmj = W.wm[j];
    const int64_t rs = W.rstart[j];
    const int32_t rlen = W.rlen[j];
    const int64_t lo = A.col_ptr[j], hi = A.col_ptr[j + 1];
    asm volatile("" ::"v"(mj), "v"(wmj), "v"(rs), "v"(rlen), "v"(lo), "v"(hi));
    const int64_t len = hi - lo;
    if (len > long_threshold) return;  // split kernel handles it
    if (roots && lane == 0) W.dirty[j] = 0;
    Cand b{0.0, INT32_MAX, -1, -1, -1};
    if (len > 1) {  // a single entry is the matched one: no cycle
        // a root too long for the tile goes to the wave-per-root kernel
        const bool handoff = len > T * E || rlen > T * E;
        const int sub = blockIdx.x & (kSpread - 1);
        const int32_t q = wave_append(&W.counters[spread_word(slot, sub)], handoff && lane == 0);
        if (handoff) {
            if (lane == 0) W.medium[(int64_t)sub * cap + q] = j;
            return;  // tile-uniform
        }
        {
            int32_t iv[E], mv[E], rv[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t k = lo + lane + T * e;
                iv[e] = (k < hi) ? A.row_idx[k] : -1;
                const int32_t x = lane + T * e;
                rv[e] = (x < rlen) ? W.colidx[rs + x] : -1;
            }
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t k = lo + lane + T * e;
                mv[e] = (iv[e] > mj) ? W.mrk[k] : -1;
            }
            int32_t qv[E];
#pragma unroll
            for (int e = 0; e < E; ++e) qv[e] = -1;
#pragma unroll
            for (int sft = 0; sft < T; ++sft) {
#pragma unroll
                for (int f = 0; f < E; ++f) {
                    const int32_t v = __shfl_xor(rv[f], sft, T);
                    const int32_t x = (lane ^ sft) + T * f;
#pragma unroll
                    for (int e = 0; e < E; ++e)
                        if (mv[e] >= 0 && v == mv[e]) qv[e] = x;
                }
            }
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (qv[e] >= 0) {
                    const int64_t k = lo + lane + T * e;
                    const int64_t p = W.cscpos ? (int64_t)W.cscpos[rs + qv[e]] : find_row(A.col_ptr, A.row_idx, mv[e], mj);
                    const double g = (A.w[k] + A.w[p]) - (W.wm[mv[e]] + wmj);
                    if (g > 0.0 && better(g, iv[e], b.g, b.i)) {
                        b.g = g; b.i = iv[e]; b.c = mv[e]; b.k = k; b.p = p;
                    }
                }
            }
        }
    }
    reduce_best<T>(b);
    if (lane == 0) publish(W, j, b, slot);
}

// Steps A-C for the roots a tile cannot hold (a column or a row list longer
// than T*E): one wave per root.  When the row list of m_j has at most
// kHashMax entries the wave stores it in an LDS hash table (column -> list
// position) and every probe m_i is one lookup (the marking trick of Section 4
// with a hash set for the mark array); longer lists take the binary search of
// row m_j in column m_i.  The 64 lanes stride over the column.
constexpr int kHashMax = 512;       // row-list entries a wave hashes
constexpr int kHashSlots = 1024;    // table size per wave (load factor <= 1/2)
constexpr int kHashPre = 4;         // column entries per lane loaded up front

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__global__ __launch_bounds__(256) void k_search_medium(Csc A, Work W, int slot, int32_t cap) {
    __shared__ int32_t keys[4][kHashSlots];
    __shared__ int32_t vals[4][kHashSlots];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t* hk = keys[wv];
    int32_t* hv = vals[wv];
    if (round_over(W)) return;
    const int32_t waves = gridDim.x * 4;
    const int32_t wid = blockIdx.x * 4 + wv;
    // the sub-lists read as one list (sub-list order, then position), dealt
    // round-robin to the waves: lane s holds the number of roots in
    // sub-lists 0..s, so the sub-list of a list index is one ballot
    static_assert(kSpread == 64, "one sub-list per lane");
    const int32_t len_s = W.counters[spread_word(slot, lane)];
    int32_t incl = len_s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    const int32_t total = __shfl(incl, 63, 64);
    for (int32_t item = wid; item < total; item += waves) {  // wave-uniform
        const int sub = (int)__popcll(__ballot(incl <= item));
        const int32_t at = item - __shfl(incl - len_s, sub, 64);
        const int32_t j = W.medium[(int64_t)sub * cap + at];
        const int64_t lo = A.col_ptr[j], hi = A.col_ptr[j + 1];
        const int32_t mj = W.mc[j];
        const double wmj = W.wm[j];
        const int64_t rs = W.rstart[j];
        const int32_t rlen = W.rlen[j];
        Cand b{0.0, INT32_MAX, -1, -1, -1};
        if (rlen <= kHashMax) {
            // the column's entries (at most 256: longer columns are split)
            // are loaded before the table is built, so that both loads are in
            // flight together
            int32_t iq[kHashPre], mq[kHashPre];
#pragma unroll
            for (int q = 0; q < kHashPre; ++q) {
                const int64_t k = lo + lane + 64 * q;
                iq[q] = (k < hi) ? A.row_idx[k] : -1;
                mq[q] = (k < hi) ? W.mrk[k] : -1;
            }
            uint32_t size = 64;
            while ((int32_t)size < 2 * rlen) size <<= 1;
            const uint32_t mask = size - 1;
            wave_lds_sync();  // the previous root's lookups are done
            for (uint32_t x = lane; x < size; x += 64) hk[x] = -1;
            wave_lds_sync();
            for (int32_t x = lane; x < rlen; x += 64) {
                const int32_t c = W.colidx[rs + x];
                uint32_t h = hash_col(c, mask);
                while (atomicCAS(&hk[h], -1, c) != -1) h = (h + 1) & mask;  // keys are distinct
                hv[h] = x;
            }
            wave_lds_sync();
            auto probe = [&](int64_t k, int32_t i, int32_t mi) {
                if (i <= mj) return;
                const int32_t qx = hash_find(hk, hv, mi, mask);
                if (qx < 0) return;
                const int64_t p = W.cscpos ? (int64_t)W.cscpos[rs + qx] : find_row(A.col_ptr, A.row_idx, mi, mj);
                const double g = (A.w[k] + A.w[p]) - (W.wm[mi] + wmj);
                if (g > 0.0 && better(g, i, b.g, b.i)) {
                    b.g = g; b.i = i; b.c = mi; b.k = k; b.p = p;
                }
            };
#pragma unroll
            for (int q = 0; q < kHashPre; ++q)
                if (iq[q] >= 0) probe(lo + lane + 64 * q, iq[q], mq[q]);
            for (int64_t k = lo + 64 * kHashPre + lane; k < hi; k += 64) probe(k, A.row_idx[k], W.mrk[k]);
        } else {
            // four entries per lane, their binary searches in lockstep
            for (int64_t k0 = lo + lane; k0 < hi; k0 += 4 * 64) {
                int32_t iq[4], cq[4], rq[4];
                int64_t pq[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t k = k0 + 64 * q;
                    iq[q] = (k < hi) ? A.row_idx[k] : -1;
                    cq[q] = (k < hi && iq[q] > mj) ? W.mrk[k] : -1;
                    rq[q] = mj;
                }
                find_row_x4(A.col_ptr, A.row_idx, cq, rq, pq);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (pq[q] < 0) continue;
                    const int64_t k = k0 + 64 * q;
                    const double g = (A.w[k] + A.w[pq[q]]) - (W.wm[cq[q]] + wmj);
                    if (g > 0.0 && better(g, iq[q], b.g, b.i)) {
                        b.g = g; b.i = iq[q]; b.c = cq[q]; b.k = k; b.p = pq[q];
                    }
                }
            }
        }
        reduce_best<64>(b);
        if (lane == 0) publish(W, j, b, slot);
    }
}

// Steps A-C, transposed probe, vector form: a quad of lanes per root; each
// stream (row indices, mate columns, the row list of m_j) is read as the
// 32-entry window that starts at the 16-byte boundary below the segment, one
// 16-byte load per lane and half, all independent.  Entries outside the
// segment are masked.  A segment that does not fit its window (or a window
// that would pass the end of row_idx) takes the generic path.
__device__ __forceinline__ int4 ld4(const int32_t* p) { return *reinterpret_cast<const int4*>(p); }

__global__ __launch_bounds__(256) void k_search_vec(Csc A, Work W, int32_t long_threshold, int slot,
                                                    const int32_t* __restrict__ roots, int32_t cap) {
    constexpr int T = 4, E = 8;
    if (round_over(W)) return;
    const int lane = threadIdx.x & 3;
    const int64_t ntiles = roots ? W.counters[slot_word(slot, kRoots)] : A.n;
    const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 2;
    if (tile >= ntiles) return;  // tile-uniform
    const int32_t j = roots ? roots[tile] : (int32_t)tile;
    // the root's values are read with its column bounds (as in k_search_chunk)
    const int32_t mj = W.mc[j];
    const double wmj = W.wm[j];
    const int64_t rs = W.rstart[j];
    const int32_t rlen = W.rlen[j];
    const int64_t lo = A.col_ptr[j], hi = A.col_ptr[j + 1];
    asm volatile("" ::"v"(mj), "v"(wmj), "v"(rs), "v"(rlen), "v"(lo), "v"(hi));
    const int64_t len = hi - lo;
    if (len > long_threshold) return;  // split kernel handles it
    if (roots && lane == 0) W.dirty[j] = 0;
    Cand b{0.0, INT32_MAX, -1, -1, -1};
    if (len > 1) {
        const int64_t cb = lo & ~(int64_t)3, rb = rs & ~(int64_t)3;
        // a segment that does not fit its window goes to the wave-per-root kernel
        const bool handoff = !(hi <= cb + 32 && rs + rlen <= rb + 32 && cb + 32 <= A.nnz);
        const int sub = blockIdx.x & (kSpread - 1);
        const int32_t q = wave_append(&W.counters[spread_word(slot, sub)], handoff && lane == 0);
        if (handoff) {
            if (lane == 0) W.medium[(int64_t)sub * cap + q] = j;
            return;  // tile-uniform
        }
        {
            const int4 i0 = ld4(A.row_idx + cb + 4 * lane), i1 = ld4(A.row_idx + cb + 16 + 4 * lane);
            const int4 m0 = ld4(W.mrk + cb + 4 * lane), m1 = ld4(W.mrk + cb + 16 + 4 * lane);
            const int4 r0 = ld4(W.colidx + rb + 4 * lane), r1 = ld4(W.colidx + rb + 16 + 4 * lane);
            int32_t iv[E] = {i0.x, i0.y, i0.z, i0.w, i1.x, i1.y, i1.z, i1.w};
            int32_t mv[E] = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
            int32_t rv[E] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t k = cb + 16 * (e >> 2) + 4 * lane + (e & 3);
                const bool in = k >= lo && k < hi;
                if (!(in && iv[e] > mj)) mv[e] = -1;
                const int64_t x = rb + 16 * (e >> 2) + 4 * lane + (e & 3);
                if (x < rs || x >= rs + rlen) rv[e] = -1;
            }
            int32_t qv[E];
#pragma unroll
            for (int e = 0; e < E; ++e) qv[e] = -1;
#pragma unroll
            for (int sft = 0; sft < T; ++sft) {
#pragma unroll
                for (int f = 0; f < E; ++f) {
                    const int32_t v = __shfl_xor(rv[f], sft, T);
                    const int32_t x = 16 * (f >> 2) + 4 * (lane ^ sft) + (f & 3);
#pragma unroll
                    for (int e = 0; e < E; ++e)
                        if (mv[e] >= 0 && v == mv[e]) qv[e] = x;
                }
            }
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (qv[e] >= 0) {
                    const int64_t k = cb + 16 * (e >> 2) + 4 * lane + (e & 3);
                    const int64_t p = W.cscpos ? (int64_t)W.cscpos[rb + qv[e]] : find_row(A.col_ptr, A.row_idx, mv[e], mj);
                    const double g = (A.w[k] + A.w[p]) - (W.wm[mv[e]] + wmj);
                    if (g > 0.0 && better(g, iv[e], b.g, b.i)) {
                        b.g = g; b.i = iv[e]; b.c = mv[e]; b.k = k; b.p = p;
                    }
                }
            }
        }
    }
    reduce_best<T>(b);
    if (lane == 0) publish(W, j, b, slot);
}

hipError_t launch_search(const Csc& A, const Work& W, int tile_width, int32_t long_threshold,
                         int slot, bool has_long, int probe, bool listed, bool incremental, hipStream_t s,
                         int cus) {
    // a listed round's length is on the device: the grid covers every column
    // and the tiles past the list's end return at once
    const int64_t all_blocks = ((int64_t)A.n * tile_width + 255) / 256;
    const unsigned blocks = (unsigned)(all_blocks > 0 ? all_blocks : 1);
    const int32_t* roots = listed ? W.dirty_list : nullptr;
    const bool transposed = probe == 2;
#define HWPM_SEARCH(TW)                                                                     \
    if (transposed)                                                                         \
        hipLaunchKernelGGL(k_search_rows<TW>, dim3(blocks), dim3(256), 0, s, A, W,          \
                           long_threshold, slot);                                           \
    else                                                                                    \
        hipLaunchKernelGGL(k_search_short<TW>, dim3(blocks), dim3(256), 0, s, A, W,         \
                           long_threshold, slot);
    // hand-off sub-list capacity: the roots of the blocks that share a
    // sub-list (kSpread sub-lists hold at most n + 4095 roots in all)
    int32_t cap = 0;
    if (probe == 4) {
        const int64_t vall = ((int64_t)A.n * 4 + 255) / 256;
        const unsigned vblocks = (unsigned)(vall > 0 ? vall : 1);
        cap = (int32_t)((vblocks + kSpread - 1) / kSpread * (256 / 4));
        hipLaunchKernelGGL(k_search_vec, dim3(vblocks), dim3(256), 0, s, A, W, long_threshold, slot, roots, cap);
    } else if (probe == 3) {
        cap = (int32_t)((blocks + kSpread - 1) / kSpread * (256 / tile_width));
        switch (tile_width) {
            case 4: hipLaunchKernelGGL((k_search_chunk<4, 8>), dim3(blocks), dim3(256), 0, s, A, W, long_threshold, slot, roots, cap); break;
            case 8: hipLaunchKernelGGL((k_search_chunk<8, 4>), dim3(blocks), dim3(256), 0, s, A, W, long_threshold, slot, roots, cap); break;
            case 16: hipLaunchKernelGGL((k_search_chunk<16, 2>), dim3(blocks), dim3(256), 0, s, A, W, long_threshold, slot, roots, cap); break;
            case 32: hipLaunchKernelGGL((k_search_chunk<32, 1>), dim3(blocks), dim3(256), 0, s, A, W, long_threshold, slot, roots, cap); break;
            default: return hipErrorInvalidValue;
        }
    } else switch (tile_width) {
        case 4: HWPM_SEARCH(4) break;
        case 8: HWPM_SEARCH(8) break;
        case 16: HWPM_SEARCH(16) break;
        case 32: HWPM_SEARCH(32) break;
        case 64: HWPM_SEARCH(64) break;
        default: return hipErrorInvalidValue;
    }
#undef HWPM_SEARCH
    if (probe >= 3) hipLaunchKernelGGL(k_search_medium, dim3(cus * 8), dim3(256), 0, s, A, W, slot, cap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !has_long) return e;
    const int only_dirty = (listed && incremental) ? 1 : 0;
    hipLaunchKernelGGL(k_search_long, dim3(cus * 8), dim3(256), 0, s, A, W, only_dirty, probe >= 2 ? 1 : 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_merge_long, dim3(64), dim3(256), 0, s, W, slot, only_dirty);
    return hipGetLastError();
}

}  // namespace hwpm
