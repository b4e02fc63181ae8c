// HIP kernels of Steps A-C (arXiv 1801.09809, Section 5.3): for every root
// column j, every row i > m_j of column j and its closing edge {m_j, m_i},
// the gain of the alternating 4-cycle and the per-root winner.
//
// Roots are binned by size: a tile of lanes per short root, a wave per
// medium root, a block per 2048-entry chunk of a long column.  The closing
// edge is probed by binary search of column m_i (probe 1) or, the GPU form of
// the marking trick of Section 4, by testing m_i against the row list of m_j
// from the matching-ordered transpose (probes 2-5).  Every probe gives the
// same (hit, position), so results never depend on the choice.
//
// With the transposed lists the search reads no row indices at all: the rows
// i > m_j of column j are exactly the positions after the matched entry
// (rows increase along a column), whose position pm[j] is kept up to date by
// the flips; each such entry's m_i is streamed from mrk; candidates are
// keyed by position, and the winner's row is read once, when it is published.
#include "hwpm_device.h"

namespace hwpm {

// ---------------------------------------------------------------------------
// Probe 1.  Short columns: a tile of T lanes per root column, lanes stride
// over the column (coalesced row_idx reads), each probes its own closing edge
// by binary search, the tile reduces to the Step-C winner with shuffles.

template <int T>
__global__ __launch_bounds__(256) void k_search_short(Csc A, Work W, int32_t long_threshold) {
    if (round_over(W)) return;
    const int lane = threadIdx.x & (T - 1);
    const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / T;
    if (tile >= A.n) return;  // tile-uniform
    const int32_t j = (int32_t)tile;
    const int64_t lo = A.col_ptr[j], hi = A.col_ptr[j + 1];
    if (hi - lo > long_threshold) return;  // split kernel handles it
    const int32_t mj = W.mc[j];
    const double wmj = W.wm[j];
    Cand b{0.0, kNoPos, -1, -1};
    for (int64_t k = lo + lane; k < hi; k += T) try_entry(A, W, k, mj, wmj, b);
    reduce_best<T>(b);
    if (lane == 0) publish(A, W, j, b);
}

// ---------------------------------------------------------------------------
// Long columns: each block takes kLongChunk entries of one column and writes
// a partial winner; k_merge_long reduces the partials of each column.  With
// the transposed lists and a row list of m_j of at most kLongHashMax entries
// the block first stores that list in an LDS hash set (column -> list
// position) and every probe is one lookup; otherwise (or if the set cannot
// take the list) each probe binary-searches row m_j in column m_i.
constexpr int kLongHashMax = 2048;
constexpr int kLongHashSlots = 4096;
constexpr int kLongPre = kLongChunk / 256;  // chunk entries per thread
static_assert(kLongHashSlots >= 2 * kLongHashMax, "long-column hash set at most half full");

__global__ __launch_bounds__(256) void k_search_long(Csc A, Work W, int only_dirty, int transposed) {
    __shared__ double sg[4];
    __shared__ int64_t sk[4], sp[4];
    __shared__ int32_t sc[4];
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
        // transposed: the chunk's entries after the matched one; else every
        // entry, pruned by row below
        const int64_t start = transposed ? ((int64_t)W.pm[j] + 1 > lo ? (int64_t)W.pm[j] + 1 : lo) : lo;
        Cand b{0.0, kNoPos, -1, -1};
        const int2 rl = transposed ? W.rsl[j] : make_int2(0, INT32_MAX);
        bool hashed = start < hi && rl.y <= kLongHashMax;  // block-uniform
        if (hashed) {
            // the chunk's mate columns (kLongPre per thread) are loaded
            // before the set is built, so that both loads are in flight together
            int32_t mq[kLongPre];
#pragma unroll
            for (int q = 0; q < kLongPre; ++q) {
                const int64_t k = lo + threadIdx.x + 256 * q;
                mq[q] = (k >= start && k < hi) ? W.mrk[k] : -1;
            }
            uint32_t size = 256;
            while ((int32_t)size < 2 * rl.y) size <<= 1;
            const uint32_t mask = size - 1;
            for (uint32_t x = threadIdx.x; x < size; x += blockDim.x) hk[x] = -1;
            __syncthreads();
            bool ok = true;
            for (int32_t x = threadIdx.x; x < rl.y; x += blockDim.x)
                ok &= hash_insert(hk, hv, W.colidx[rl.x + x], x, mask, LdsCas32{});
            hashed = !__syncthreads_or(!ok);  // a list the set cannot take: binary search
            if (hashed) {
#pragma unroll
                for (int q = 0; q < kLongPre; ++q) {
                    const int32_t mi = mq[q];
                    if (mi < 0) continue;
                    const int32_t qx = hash_find(hk, hv, mi, mask);
                    if (qx < 0) continue;
                    const int64_t k = lo + threadIdx.x + 256 * q;
                    const int64_t p = W.cscpos ? (int64_t)W.cscpos[rl.x + qx] : find_row(A.col_ptr, A.row_idx, mi, mj);
                    if (p >= 0) offer(b, (A.w[k] + A.w[p]) - (W.wm[mi] + W.wm[j]), k, mi, p);
                }
            }
            __syncthreads();  // the set is rebuilt for the next chunk
        }
        const int32_t tb = transposed && !hashed && W.rtab ? W.rtab[j] : -1;  // block-uniform
        if (!hashed && start < hi && tb >= 0) {
            // the list's hash table: a probe that hits reads its position
            // (or, without stored positions, searches for it)
            uint32_t size = 64;
            while ((int32_t)size < 2 * rl.y) size <<= 1;
            const int32_t* tab = W.tabs + tb;
            for (int64_t k0 = start + threadIdx.x; k0 < hi; k0 += 4 * (int64_t)blockDim.x) {
                int32_t cq[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t k = k0 + (int64_t)q * blockDim.x;
                    cq[q] = (k < hi) ? W.mrk[k] : -1;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int32_t qx = cq[q] < 0 ? -1 : hash_find(tab, tab + size, cq[q], size - 1);
                    if (qx < 0) continue;
                    const int64_t k = k0 + (int64_t)q * blockDim.x;
                    const int64_t p = W.cscpos ? (int64_t)W.cscpos[rl.x + qx] : find_row(A.col_ptr, A.row_idx, cq[q], mj);
                    if (p >= 0) offer(b, (A.w[k] + A.w[p]) - (W.wm[cq[q]] + W.wm[j]), k, cq[q], p);
                }
            }
        } else if (!hashed && start < hi) {
            // four entries per thread, their binary searches in lockstep
            const int32_t step = blockDim.x;
            for (int64_t k0 = start + threadIdx.x; k0 < hi; k0 += 4 * (int64_t)step) {
                int32_t cq[4], rq[4];
                int64_t pq[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t k = k0 + (int64_t)q * step;
                    if (transposed) {
                        cq[q] = (k < hi) ? W.mrk[k] : -1;
                    } else {
                        const int32_t i = (k < hi) ? A.row_idx[k] : -1;
                        cq[q] = (i > mj) ? W.mr[i] : -1;
                    }
                    rq[q] = mj;
                }
                find_row_x4(A.col_ptr, A.row_idx, cq, rq, pq);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (pq[q] < 0) continue;
                    const int64_t k = k0 + (int64_t)q * step;
                    offer(b, (A.w[k] + A.w[pq[q]]) - (W.wm[cq[q]] + W.wm[j]), k, cq[q], pq[q]);
                }
            }
        }
        reduce_best<64>(b);
        if (lane == 0) {
            sg[wave] = b.g; sk[wave] = b.k; sc[wave] = b.c; sp[wave] = b.p;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int u = 1; u < 4; ++u) {
                if (better(sg[u], sk[u], b.g, b.k)) {
                    b.g = sg[u]; b.k = sk[u]; b.c = sc[u]; b.p = sp[u];
                }
            }
            W.part_g[cid] = b.g; W.part_k[cid] = b.k; W.part_c[cid] = b.c; W.part_p[cid] = b.p;
        }
        __syncthreads();
    }
}

__global__ void k_merge_long(Csc A, Work W, int only_dirty) {
    if (round_over(W)) return;
    const int32_t nl = W.counters[kNumLong];
    for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nl; q += gridDim.x * blockDim.x) {
        if (only_dirty) {
            if (W.dirty[W.long_list[q]] == 0) continue;
            W.dirty[W.long_list[q]] = 0;
        }
        Cand b{0.0, kNoPos, -1, -1};
        for (int64_t cid = W.chunk_off[q]; cid < W.chunk_off[q + 1]; ++cid) {
            if (better(W.part_g[cid], W.part_k[cid], b.g, b.k)) {
                b.g = W.part_g[cid]; b.k = W.part_k[cid]; b.c = W.part_c[cid]; b.p = W.part_p[cid];
            }
        }
        publish(A, W, W.long_list[q], b);
    }
}

// ---------------------------------------------------------------------------
// Probe 2: transposed lists, one entry per lane.  For root j the row list of
// m_j is read once per tile (contiguous) and every probe m_i of the tile is
// tested against it with T cross-lane rotations.  Rows longer than kRowRotate
// fall back to the binary-search probe of column m_i.
constexpr int kRowRotate = 64;

template <int T>
__global__ __launch_bounds__(256) void k_search_rows(Csc A, Work W, int32_t long_threshold) {
    if (round_over(W)) return;
    const int lane = threadIdx.x & (T - 1);
    const int64_t tile = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / T;
    if (tile >= A.n) return;  // tile-uniform
    const int32_t j = (int32_t)tile;
    const int32_t lo = W.cp32[j], hi = W.cp32[j + 1];
    if (hi - lo > long_threshold) return;
    const int32_t s0 = W.pm[j] + 1;  // rows i > m_j: the positions after the matched entry
    const int2 rl = W.rsl[j];
    Cand b{0.0, kNoPos, -1, -1};
    if (rl.y <= kRowRotate) {
        // row list of m_j, T entries per lane-chunk; -1 never equals a column
        const int32_t cv0 = (lane < rl.y) ? W.colidx[rl.x + lane] : -1;
        for (int32_t kc = s0; kc < hi; kc += T) {  // tile-uniform trip count
            const int32_t k = kc + lane;
            const int32_t mi = (k < hi) ? W.mrk[k] : -2;
            int32_t q = -1;
            for (int32_t rc = 0; rc < rl.y; rc += T) {
                const int32_t cv = (rc == 0) ? cv0 : ((rc + lane < rl.y) ? W.colidx[rl.x + rc + lane] : -1);
#pragma unroll
                for (int sft = 0; sft < T; ++sft) {
                    const int src = (lane + sft) & (T - 1);
                    if (__shfl(cv, src, T) == mi) q = rc + src;
                }
            }
            if (q >= 0) {
                const int64_t p = W.cscpos ? (int64_t)W.cscpos[rl.x + q] : find_row(A.col_ptr, A.row_idx, mi, W.mc[j]);
                if (p >= 0) offer(b, (A.w[k] + A.w[p]) - (W.wm[mi] + W.wm[j]), k, mi, p);
            }
        }
    } else {
        const int32_t mj = W.mc[j];
        for (int32_t k = s0 + lane; k < hi; k += T) {
            const int32_t mi = W.mrk[k];
            const int64_t p = find_row(A.col_ptr, A.row_idx, mi, mj);
            if (p < 0) continue;
            offer(b, (A.w[k] + A.w[p]) - (W.wm[mi] + W.wm[j]), k, mi, p);
        }
    }
    reduce_best<T>(b);
    if (lane == 0) publish(A, W, j, b);
}

// ---------------------------------------------------------------------------
// Roots a tile cannot hold go to the wave-per-root kernel through kSpread
// sub-lists per round; sub-list s of a round holds at most `cap` roots, at
// medium[s * cap ...).
__device__ __forceinline__ void hand_off(const Work& W, int slot, int sub, int32_t cap, int32_t j, bool want) {
    const int32_t q = wave_append(&W.counters[spread_word(slot, sub)], want);
    if (want) W.medium[(int64_t)sub * cap + q] = j;
}

// Exchanges inside a tile of T lanes.  With 4-lane tiles they are DPP quad
// permutations (a VALU move, no trip through the LDS crossbar).
template <int T>
__device__ __forceinline__ int32_t tile_xor(int32_t v, int sft) {
    if constexpr (T == 4) {
        switch (sft) {
            case 0: return v;
            case 1: return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
            case 2: return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
            default: return __builtin_amdgcn_mov_dpp(v, 0x1B, 0xF, 0xF, false);  // quad_perm [3,2,1,0]
        }
    } else {
        return __shfl_xor(v, sft, T);
    }
}

template <int T>
__device__ __forceinline__ int32_t tile_bcast(int32_t v, int src) {
    if constexpr (T == 4) {
        switch (src) {
            case 0: return __builtin_amdgcn_mov_dpp(v, 0x00, 0xF, 0xF, false);  // quad_perm [0,0,0,0]
            case 1: return __builtin_amdgcn_mov_dpp(v, 0x55, 0xF, 0xF, false);  // quad_perm [1,1,1,1]
            case 2: return __builtin_amdgcn_mov_dpp(v, 0xAA, 0xF, 0xF, false);  // quad_perm [2,2,2,2]
            default: return __builtin_amdgcn_mov_dpp(v, 0xFF, 0xF, 0xF, false);  // quad_perm [3,3,3,3]
        }
    } else {
        return __shfl(v, src, T);
    }
}

// OR over the tile, in every lane of the tile.  With 4-lane tiles each step
// is one OR with a DPP quad-permuted operand.
template <int T>
__device__ __forceinline__ uint32_t tile_or(uint32_t v) {
    if constexpr (T == 4) {
        v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]
        v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
    } else {
#pragma unroll
        for (int sft = 1; sft < T; sft <<= 1) v |= (uint32_t)__shfl_xor((int32_t)v, sft, T);
    }
    return v;
}

// Bit T t of the result: some bit of tile t of the lane mask m is set; the
// other bits are clear.
template <int T>
__device__ __forceinline__ uint64_t tile_any(uint64_t m) {
#pragma unroll
    for (int sft = 1; sft < T; sft <<= 1) m |= m >> sft;
    constexpr uint64_t first = T == 4 ? 0x1111111111111111ull : T == 8 ? 0x0101010101010101ull
                             : T == 16 ? 0x0001000100010001ull : T == 32 ? 0x0000000100000001ull : 1ull;
    return m & first;
}

// Largest value of the tile, in every lane of the tile.
template <int T>
__device__ __forceinline__ int32_t tile_max(int32_t v) {
#pragma unroll
    for (int sft = 1; sft < T; sft <<= 1) v = max(v, tile_xor<T>(v, sft));
    return v;
}

// Largest of non-negative values over the wave, as a wave-uniform (scalar)
// value: DPP row shifts give every lane the maximum of its row of 16 up to
// itself, two row broadcasts carry the rows' maxima into lane 63.  Lanes
// without a source read 0, the identity of the unsigned maximum, so each
// step is one maximum with a DPP operand.  All lanes must be active.
__device__ __forceinline__ int32_t wave_max(int32_t x) {
    uint32_t v = (uint32_t)x;
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x111, 0xF, 0xF, true));  // row_shr:1
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x112, 0xF, 0xF, true));  // row_shr:2
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x114, 0xF, 0xF, true));  // row_shr:4
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x118, 0xF, 0xF, true));  // row_shr:8
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x142, 0xA, 0xF, false));  // row_bcast:15
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)v, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return (int32_t)__builtin_amdgcn_readlane((int32_t)v, 63);
}

// Element idx of an array of at most 2^32 bytes.  With O32 the byte offset
// is a 32-bit value added to the array's base, so the load takes the base
// from scalar registers and a 32-bit offset per lane, with no 64-bit address
// arithmetic in the vector unit (the tile kernels are bound by vector
// instruction issue).
template <bool O32, typename V>
__device__ __forceinline__ V ld_at(const V* base, int32_t idx) {
    if constexpr (O32)
        return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) +
                                           (uint32_t)idx * (uint32_t)sizeof(V));
    else
        return base[idx];
}

// The element at byte offset off of an array of at most 2^32 bytes.
template <typename V>
__device__ __forceinline__ V ld_byte(const V* base, uint32_t off) {
    return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + off);
}

// The per-root values of a tile kernel, read together (one memory round trip).
struct RootView {
    int32_t j, s0, slen;  // root, first position after the matched entry, suffix length
    int2 rl;              // row list of m_j: (start, length)
    bool own;             // a short root of this kernel (long columns: the split kernel)
};

template <bool O32 = false>
__device__ __forceinline__ RootView load_root(const Work& W, int64_t t, int64_t ntiles, const int32_t* roots,
                                              int32_t long_threshold) {
    RootView r;
    const bool in = t < ntiles;
    r.j = in ? (roots ? ld_at<O32>(roots, (int32_t)t) : (int32_t)t) : 0;
    const int32_t lo = ld_at<O32>(W.cp32, r.j), hi = ld_at<O32>(W.cp32, r.j + 1), pmj = ld_at<O32>(W.pm, r.j);
    r.rl = ld_at<O32>(W.rsl, r.j);
    r.own = in && hi - lo <= long_threshold;
    r.s0 = pmj + 1;  // rows i > m_j: the positions after the matched entry
    r.slen = r.own ? hi - r.s0 : 0;
    return r;
}

// Probe 4: transposed lists, cross-lane form: a tile of T lanes per root,
// each lane holding E entries of the pruned suffix of column j (their m_i)
// and E entries of the row list of m_j, every probe compared with the whole
// row list through T cross-lane exchanges.  The comparisons stop at the
// longest suffix and row list of the wave.  Roots with a longer suffix or row
// list than T * E are handed off.
template <int T, int E>
__global__ __launch_bounds__(256) void k_search_chunk(Csc A, Work W, int32_t long_threshold,
                                                      int slot, const int32_t* __restrict__ roots,
                                                      int32_t cap) {
    if (round_over(W)) return;
    const int lane = threadIdx.x & (T - 1);
    // roots: this round's list (its length on the device; the grid covers
    // every column), else every column
    const int64_t ntiles = roots ? W.counters[slot_word(slot, kRoots)] : A.n;
    const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / T;
    if (((int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63)) / T >= ntiles) return;  // wave-uniform
    const RootView r = load_root(W, t, ntiles, roots, long_threshold);
    if (r.own && roots && lane == 0) W.dirty[r.j] = 0;
    const bool handoff = r.slen > 0 && (r.slen > T * E || r.rl.y > T * E);
    hand_off(W, slot, blockIdx.x & (kSpread - 1), cap, r.j, handoff && lane == 0);
    const bool search = r.slen > 0 && !handoff;
    int32_t mv[E], rv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int32_t x = lane + T * e;
        mv[e] = (search && x < r.slen) ? W.mrk[r.s0 + x] : -1;
        rv[e] = (search && x < r.rl.y) ? W.colidx[r.rl.x + x] : -2;  // -1 / -2 never match each other
    }
    const int32_t e_lim = (wave_max(search ? r.slen : 0) + T - 1) / T;
    const int32_t f_lim = (wave_max(search ? r.rl.y : 0) + T - 1) / T;
    int32_t qv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) qv[e] = -1;
#pragma unroll
    for (int sft = 0; sft < T; ++sft) {
#pragma unroll
        for (int f = 0; f < E; ++f) {
            if (f >= f_lim) break;  // wave-uniform
            const int32_t v = tile_xor<T>(rv[f], sft);
            const int32_t x = (lane ^ sft) + T * f;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (e >= e_lim) break;  // wave-uniform
                if (v == mv[e]) qv[e] = x;
            }
        }
    }
    Cand b{0.0, kNoPos, -1, -1};
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (qv[e] >= 0) {
            const int32_t k = r.s0 + lane + T * e;
            const int64_t p = W.cscpos ? (int64_t)W.cscpos[r.rl.x + qv[e]] : find_row(A.col_ptr, A.row_idx, mv[e], W.mc[r.j]);
            if (p >= 0) offer(b, (A.w[k] + A.w[p]) - (W.wm[mv[e]] + W.wm[r.j]), k, mv[e], p);
        }
    }
    if (__ballot(b.k != kNoPos)) reduce_best<T>(b);  // wave-uniform: most waves have no candidate
    if (r.own && !handoff && lane == 0) publish(A, W, r.j, b);
}

// Probes 3 and 5: transposed lists, filter form (the default).  A tile of T
// lanes per root loads the pruned suffix of column j (E mate columns per
// lane) and the row list of m_j (E columns per lane), all loads independent.
// The tile ORs its row list into a two-word filter (one bit per 64-bit word,
// from two fields of one hash of the column), and each probe m_i whose two bits
// are both set is compared exactly with the row list: the tile's passed
// probes are broadcast in turn and every lane compares each with its own part
// of the list (with positions kept, a tile maximum returns the place; without
// them only membership is needed, taken in lane masks); the others are
// certain misses.  With about 17 columns in a row list a miss passes the
// filter about 5 % of the time, so on matrices whose probes mostly miss the
// exact comparisons shrink from every pair to a few probes per wave.  Roots
// whose suffix or row list exceeds T * E entries are handed off.
// One multiplicative hash of the column's low 24 bits (a full-rate 24-bit
// multiply); its bits 26-31 and 20-25 pick the bits of the two filter words.
// Columns that agree in their low 24 bits share their bits, which can only
// let more probes through to the exact comparison.
__device__ __forceinline__ uint32_t filter_hash(int32_t c) { return __umul24((uint32_t)c, 0x9E3779u); }

// A root whose suffix and row list exceed the tile but fit the wave's 64
// lanes: the whole wave searches it, one suffix entry and one list entry per
// lane, every list entry broadcast in turn.  j is wave-uniform, so its values
// come in through scalar loads; all lanes must be active.
__device__ __forceinline__ void search_wide(const Csc& A, const Work& W, int32_t j, int l64) {
    const int32_t s0 = W.pm[j] + 1, slen = W.cp32[j + 1] - s0;
    const int2 rl = W.rsl[j];
    const int32_t mi = l64 < slen ? W.mrk[s0 + l64] : -1;
    const int32_t cv = l64 < rl.y ? W.colidx[rl.x + l64] : -2;
    int32_t q = -1;
    for (int32_t x = 0; x < rl.y; ++x)  // wave-uniform trip count
        if (__builtin_amdgcn_readlane(cv, x) == mi) q = x;
    Cand b{0.0, kNoPos, -1, -1};
    if (q >= 0) {
        const int32_t k = s0 + l64;
        const int64_t p = W.cscpos ? (int64_t)W.cscpos[rl.x + q] : find_row(A.col_ptr, A.row_idx, mi, W.mc[j]);
        if (p >= 0) offer(b, (A.w[k] + A.w[p]) - (W.wm[mi] + W.wm[j]), k, mi, p);
    }
    if (__ballot(b.k != kNoPos)) reduce_best<64>(b);
    if (l64 == 0) publish(A, W, j, b);
}

// Roots of one wave searched by the whole wave when they are this few;
// more than that go to the wave-per-root kernel, which runs them in
// parallel.  Only 4-lane tiles take them: on wider tiles the extra code
// slowed the tile path itself by more than it saved (measured on the 27-point
// stencil, whose roots all fit the tile).
template <int T>
constexpr int kWideMax = T == 4 ? 2 : 0;

// Steps A-C of one group of 64 / T roots (a tile per root); see below.
template <int T, int E, bool O32, bool POS>
__device__ __forceinline__ void search_group(const Csc& A, const Work& W, const RootView& r, int slot, int sub,
                                             int32_t cap, bool listed) {
    const int l64 = threadIdx.x & 63;
    const int lane = l64 & (T - 1);
    if (r.own && listed && lane == 0) W.dirty[r.j] = 0;
    // too long for the tile: the wave searches it when both lists fit 64
    // lanes and the wave has at most kWideMax such roots, else the
    // wave-per-root kernel does
    const bool big = r.slen > 0 && (r.slen > T * E || r.rl.y > T * E);
    uint64_t wm = __ballot(big && r.slen <= 64 && r.rl.y <= 64 && lane == 0);
    if (__popcll(wm) > kWideMax<T>) wm = 0;  // wave-uniform
    const bool wide = (wm >> l64) & 1u;
    hand_off(W, slot, sub, cap, r.j, big && !wide && lane == 0);
    const bool search = r.slen > 0 && !big;
    // loads, only as far as the wave's longest suffix and row list go,
    // indices clamped to the last entry of the segment: a lane's entries past
    // the end repeat that entry (an empty suffix reads the matched entry; a
    // row list always holds the matched entry of its row)
    const int32_t e_lim = (wave_max(search ? r.slen : 0) + T - 1) / T;
    const int32_t f_lim = (wave_max(search ? r.rl.y : 0) + T - 1) / T;
    int32_t mv[E], rv[E];
    if constexpr (O32) {  // byte offsets
        const uint32_t m0 = (uint32_t)(r.s0 + lane) * 4u, m1 = (uint32_t)(r.s0 + r.slen - 1) * 4u;
        const uint32_t c0 = (uint32_t)(r.rl.x + lane) * 4u, c1 = (uint32_t)(r.rl.x + r.rl.y - 1) * 4u;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            mv[e] = e < e_lim ? ld_byte(W.mrk, min(m0 + 4u * T * e, m1)) : -1;
            rv[e] = e < f_lim ? ld_byte(W.colidx, min(c0 + 4u * T * e, c1)) : -2;
        }
    } else {
        const int64_t m1 = (int64_t)r.s0 + r.slen - 1, c1 = (int64_t)r.rl.x + r.rl.y - 1;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            mv[e] = e < e_lim ? W.mrk[min((int64_t)r.s0 + lane + T * e, m1)] : -1;
            rv[e] = e < f_lim ? W.colidx[min((int64_t)r.rl.x + lane + T * e, c1)] : -2;
        }
    }
    // the filter of the row list (the repeated last entry adds no bits)
    uint64_t f1 = 0, f2 = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (e >= f_lim) break;  // wave-uniform
        const uint32_t h = filter_hash(rv[e]);
        f1 |= 1ull << (h >> 26);
        f2 |= 1ull << ((h >> 20) & 63);
    }
    f1 = ((uint64_t)tile_or<T>((uint32_t)(f1 >> 32)) << 32) | tile_or<T>((uint32_t)f1);
    f2 = ((uint64_t)tile_or<T>((uint32_t)(f2 >> 32)) << 32) | tile_or<T>((uint32_t)f2);
    // the probes against it; a lane's own probes are its first nm entries
    const int32_t nm = search && r.slen > lane ? (r.slen - lane + T - 1) / T : 0;
    uint32_t pending = 0;  // bit e: probe e passed the filter
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (e >= e_lim) break;  // wave-uniform
        const uint32_t h = filter_hash(mv[e]);
        pending |= (uint32_t)((f1 >> (h >> 26)) & (f2 >> ((h >> 20) & 63)) & 1u) << e;
    }
    pending &= (1u << nm) - 1u;
    Cand b{0.0, kNoPos, -1, -1};
    while (__ballot(pending != 0)) {  // wave-uniform: one passed probe per lane at a time
        const int e = pending ? __builtin_ctz(pending) : -1;
        pending &= pending - 1;
        int32_t mi = -1;
#pragma unroll
        for (int u = 0; u < E; ++u)
            if (u == e) mi = mv[u];
        if constexpr (!POS) {
            // membership only (the closing edge is then found in column m_i):
            // the tile's probes, each compared by every lane with its own part
            // of the row list into one lane mask per probe; bit T t + src of
            // `held` says whether tile t holds the probe of its lane src
            uint64_t held = 0;
#pragma unroll
            for (int src = 0; src < T; ++src) {
                const int32_t ps = tile_bcast<T>(mi, src);
                uint64_t m = 0;
#pragma unroll
                for (int f = 0; f < E; ++f) m |= __ballot(rv[f] == ps);
                held |= tile_any<T>(m) << src;
            }
            if ((held >> l64) & 1u) {
                const int32_t k = r.s0 + lane + T * e;
                const int64_t p = find_row(A.col_ptr, A.row_idx, mi, W.mc[r.j]);
                if (p >= 0) offer(b, (A.w[k] + A.w[p]) - (W.wm[mi] + W.wm[r.j]), k, mi, p);
            }
            continue;
        }
        // the tile's probes, each compared by every lane with its own part
        // of the row list; the matching place comes back to the probe's lane
        // (a match with a repeat of the list's last entry lies past the
        // list's end and stands for that last entry)
        int32_t q = -1;
#pragma unroll
        for (int src = 0; src < T; ++src) {
            const int32_t ps = tile_bcast<T>(mi, src);
            int32_t xs = -1;
#pragma unroll
            for (int f = 0; f < E; ++f)
                if (rv[f] == ps) xs = lane + T * f;
            xs = tile_max<T>(xs);
            if (lane == src) q = xs;
        }
        if (q >= 0) {
            q = min(q, r.rl.y - 1);
            const int32_t k = r.s0 + lane + T * e;
            const int64_t p = W.cscpos[r.rl.x + q];
            if (p >= 0) offer(b, (A.w[k] + A.w[p]) - (W.wm[mi] + W.wm[r.j]), k, mi, p);
        }
    }
    if (__ballot(b.k != kNoPos)) reduce_best<T>(b);  // wave-uniform: most waves have no candidate
    if (r.own && !big && lane == 0) publish(A, W, r.j, b);
    // the group's wide roots, one after the other
    for (; wm; wm &= wm - 1)  // wave-uniform
        search_wide(A, W, __builtin_amdgcn_readlane(r.j, __builtin_ctzll(wm)), l64);
}

// One group of 64 / T roots per wave.  O32: every array the tiles index holds
// at most 2^32 bytes (nnz < 2^30, n < 2^28).  POS: the row lists carry the
// CSC positions of their entries.
template <int T, int E, bool O32, bool POS>
__global__ __launch_bounds__(256, 8) void k_search_filter(Csc A, Work W, int32_t long_threshold, int slot,
                                                          const int32_t* __restrict__ roots, int32_t cap) {
    constexpr int kTiles = 64 / T;
    if (round_over(W)) return;
    const int64_t ntiles = roots ? W.counters[slot_word(slot, kRoots)] : A.n;
    const int64_t grp = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (grp * kTiles >= ntiles) return;  // wave-uniform
    const RootView r = load_root<O32>(W, grp * kTiles + (threadIdx.x & 63) / T, ntiles, roots, long_threshold);
    search_group<T, E, O32, POS>(A, W, r, slot, (int)(blockIdx.x & (kSpread - 1)), cap, roots != nullptr);
}

// ---------------------------------------------------------------------------
// Steps A-C for the roots a tile cannot hold (a pruned suffix or a row list
// longer than the tile): one wave per root.  When the row list of m_j has at
// most kHashMax entries the wave stores it in an LDS hash set (column -> list
// position) and every probe m_i is one lookup (the marking trick of Section 4
// with a hash set for the mark array); longer lists, or a list the set cannot
// take, use the binary search of row m_j in column m_i.  The 64 lanes stride
// over the suffix of the column.
constexpr int kHashMax = 512;       // row-list entries a wave hashes
constexpr int kHashSlots = 1024;    // set size per wave (load factor <= 1/2)
constexpr int kHashPre = 4;         // column entries per lane loaded up front
static_assert(kHashSlots >= 2 * kHashMax, "wave hash set at most half full");

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
        const int32_t hi = W.cp32[j + 1];
        const int32_t s0 = W.pm[j] + 1;  // rows i > m_j: positions after the matched entry
        const int2 rl = W.rsl[j];
        Cand b{0.0, kNoPos, -1, -1};
        bool hashed = rl.y <= kHashMax;  // wave-uniform
        if (hashed) {
            // the suffix's first entries (at most 256 entries in all: longer
            // columns are split) are loaded before the set is built, so that
            // both loads are in flight together
            int32_t mq[kHashPre];
#pragma unroll
            for (int q = 0; q < kHashPre; ++q) {
                const int32_t k = s0 + lane + 64 * q;
                mq[q] = (k < hi) ? W.mrk[k] : -1;
            }
            uint32_t size = 64;
            while ((int32_t)size < 2 * rl.y) size <<= 1;
            const uint32_t mask = size - 1;
            wave_lds_sync();  // the previous root's lookups are done
            for (uint32_t x = lane; x < size; x += 64) hk[x] = -1;
            wave_lds_sync();
            bool ok = true;
            for (int32_t x = lane; x < rl.y; x += 64)
                ok &= hash_insert(hk, hv, W.colidx[rl.x + x], x, mask, LdsCas32{});
            wave_lds_sync();
            hashed = __ballot(!ok) == 0ull;
            if (hashed) {
                auto probe = [&](int32_t k, int32_t mi) {
                    const int32_t qx = hash_find(hk, hv, mi, mask);
                    if (qx < 0) return;
                    const int64_t p = W.cscpos ? (int64_t)W.cscpos[rl.x + qx] : find_row(A.col_ptr, A.row_idx, mi, W.mc[j]);
                    if (p >= 0) offer(b, (A.w[k] + A.w[p]) - (W.wm[mi] + W.wm[j]), k, mi, p);
                };
#pragma unroll
                for (int q = 0; q < kHashPre; ++q)
                    if (mq[q] >= 0) probe(s0 + lane + 64 * q, mq[q]);
                for (int32_t k = s0 + 64 * kHashPre + lane; k < hi; k += 64) probe(k, W.mrk[k]);
            }
        }
        const int32_t tb = hashed || !W.rtab ? -1 : W.rtab[j];  // wave-uniform
        if (!hashed && tb >= 0) {
            // the list's hash table: a probe that hits reads its position
            // (or, without stored positions, searches for it)
            const int32_t mj = W.mc[j];
            uint32_t size = 64;
            while ((int32_t)size < 2 * rl.y) size <<= 1;
            const int32_t* tab = W.tabs + tb;
            for (int32_t k0 = s0 + lane; k0 < hi; k0 += 4 * 64) {
                int32_t cq[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int32_t k = k0 + 64 * q;
                    cq[q] = (k < hi) ? W.mrk[k] : -1;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int32_t qx = cq[q] < 0 ? -1 : hash_find(tab, tab + size, cq[q], size - 1);
                    if (qx < 0) continue;
                    const int32_t k = k0 + 64 * q;
                    const int64_t p = W.cscpos ? (int64_t)W.cscpos[rl.x + qx] : find_row(A.col_ptr, A.row_idx, cq[q], mj);
                    if (p >= 0) offer(b, (A.w[k] + A.w[p]) - (W.wm[cq[q]] + W.wm[j]), k, cq[q], p);
                }
            }
        } else if (!hashed) {
            // four entries per lane, their binary searches in lockstep
            const int32_t mj = W.mc[j];
            for (int32_t k0 = s0 + lane; k0 < hi; k0 += 4 * 64) {
                int32_t cq[4], rq[4];
                int64_t pq[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int32_t k = k0 + 64 * q;
                    cq[q] = (k < hi) ? W.mrk[k] : -1;
                    rq[q] = mj;
                }
                find_row_x4(A.col_ptr, A.row_idx, cq, rq, pq);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (pq[q] < 0) continue;
                    const int32_t k = k0 + 64 * q;
                    offer(b, (A.w[k] + A.w[pq[q]]) - (W.wm[cq[q]] + W.wm[j]), k, cq[q], pq[q]);
                }
            }
        }
        reduce_best<64>(b);
        if (lane == 0) publish(A, W, j, b);
    }
}

template <bool O32, bool POS>
static hipError_t launch_filter(const Csc& A, const Work& W, int tile_width, unsigned blocks, int32_t long_threshold,
                                int slot, const int32_t* roots, int32_t cap, hipStream_t s) {
    switch (tile_width) {
        case 4: hipLaunchKernelGGL((k_search_filter<4, 8, O32, POS>), dim3(blocks), dim3(256), 0, s, A, W, long_threshold, slot, roots, cap); break;
        case 8: hipLaunchKernelGGL((k_search_filter<8, 4, O32, POS>), dim3(blocks), dim3(256), 0, s, A, W, long_threshold, slot, roots, cap); break;
        case 16: hipLaunchKernelGGL((k_search_filter<16, 2, O32, POS>), dim3(blocks), dim3(256), 0, s, A, W, long_threshold, slot, roots, cap); break;
        case 32: hipLaunchKernelGGL((k_search_filter<32, 1, O32, POS>), dim3(blocks), dim3(256), 0, s, A, W, long_threshold, slot, roots, cap); break;
        default: return hipErrorInvalidValue;
    }
    return hipSuccess;
}

hipError_t launch_search(const Csc& A, const Work& W, int tile_width, int32_t long_threshold,
                         int slot, bool has_long, int probe, bool listed, bool incremental, hipStream_t s,
                         int cus) {
    // a listed round's length is on the device: the grid covers every column
    // and the tiles past the list's end return at once
    const int64_t all_blocks = ((int64_t)A.n * tile_width + 255) / 256;
    const unsigned blocks = (unsigned)(all_blocks > 0 ? all_blocks : 1);
    const int32_t* roots = listed ? W.dirty_list : nullptr;
    int32_t cap = 0;
    if (probe == 1) {
        switch (tile_width) {
            case 4: hipLaunchKernelGGL(k_search_short<4>, dim3(blocks), dim3(256), 0, s, A, W, long_threshold); break;
            case 8: hipLaunchKernelGGL(k_search_short<8>, dim3(blocks), dim3(256), 0, s, A, W, long_threshold); break;
            case 16: hipLaunchKernelGGL(k_search_short<16>, dim3(blocks), dim3(256), 0, s, A, W, long_threshold); break;
            case 32: hipLaunchKernelGGL(k_search_short<32>, dim3(blocks), dim3(256), 0, s, A, W, long_threshold); break;
            case 64: hipLaunchKernelGGL(k_search_short<64>, dim3(blocks), dim3(256), 0, s, A, W, long_threshold); break;
            default: return hipErrorInvalidValue;
        }
    } else if (probe == 2) {
        switch (tile_width) {
            case 4: hipLaunchKernelGGL(k_search_rows<4>, dim3(blocks), dim3(256), 0, s, A, W, long_threshold); break;
            case 8: hipLaunchKernelGGL(k_search_rows<8>, dim3(blocks), dim3(256), 0, s, A, W, long_threshold); break;
            case 16: hipLaunchKernelGGL(k_search_rows<16>, dim3(blocks), dim3(256), 0, s, A, W, long_threshold); break;
            case 32: hipLaunchKernelGGL(k_search_rows<32>, dim3(blocks), dim3(256), 0, s, A, W, long_threshold); break;
            case 64: hipLaunchKernelGGL(k_search_rows<64>, dim3(blocks), dim3(256), 0, s, A, W, long_threshold); break;
            default: return hipErrorInvalidValue;
        }
    } else if (probe == 4) {
        // hand-off sub-lists by block: the roots of the blocks that share a
        // sub-list (kSpread sub-lists hold at most n + 4095 roots in all)
        cap = (int32_t)((blocks + kSpread - 1) / kSpread * (256 / tile_width));
        switch (tile_width) {
            case 4: hipLaunchKernelGGL((k_search_chunk<4, 8>), dim3(blocks), dim3(256), 0, s, A, W, long_threshold, slot, roots, cap); break;
            case 8: hipLaunchKernelGGL((k_search_chunk<8, 4>), dim3(blocks), dim3(256), 0, s, A, W, long_threshold, slot, roots, cap); break;
            case 16: hipLaunchKernelGGL((k_search_chunk<16, 2>), dim3(blocks), dim3(256), 0, s, A, W, long_threshold, slot, roots, cap); break;
            case 32: hipLaunchKernelGGL((k_search_chunk<32, 1>), dim3(blocks), dim3(256), 0, s, A, W, long_threshold, slot, roots, cap); break;
            default: return hipErrorInvalidValue;
        }
    } else {  // probes 3 and 5 (the row lists with or without positions)
        cap = (int32_t)((blocks + kSpread - 1) / kSpread * (256 / tile_width));
        const bool o32 = A.nnz < ((int64_t)1 << 30) && A.n < (1 << 28);
        const bool pos = W.cscpos != nullptr;
        const hipError_t e =
            o32 ? (pos ? launch_filter<true, true>(A, W, tile_width, blocks, long_threshold, slot, roots, cap, s)
                       : launch_filter<true, false>(A, W, tile_width, blocks, long_threshold, slot, roots, cap, s))
                : (pos ? launch_filter<false, true>(A, W, tile_width, blocks, long_threshold, slot, roots, cap, s)
                       : launch_filter<false, false>(A, W, tile_width, blocks, long_threshold, slot, roots, cap, s));
        if (e != hipSuccess) return e;
    }
    if (probe >= 3) hipLaunchKernelGGL(k_search_medium, dim3(cus * 8), dim3(256), 0, s, A, W, slot, cap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !has_long) return e;
    const int only_dirty = (listed && incremental) ? 1 : 0;
    hipLaunchKernelGGL(k_search_long, dim3(cus * 8), dim3(256), 0, s, A, W, only_dirty, probe >= 2 ? 1 : 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_merge_long, dim3(64), dim3(256), 0, s, A, W, only_dirty);
    return hipGetLastError();
}

}  // namespace hwpm
