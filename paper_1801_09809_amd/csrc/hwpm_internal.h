// Internal declarations shared by the HIP kernels and the C-ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hwpm {

constexpr int32_t kNoRoot = 0x7fffffff;   // empty Step-D slot
constexpr int kSlots = 8;                  // ring of per-round counter pairs
constexpr int kLongChunk = 2048;           // entries per block in the long-column search
constexpr int kTreeBlock = 2048;           // leaves summed by one tree-sum block
constexpr int kMaxRoundStats = 512;        // rounds with per-round statistics

// Counter words (int32) at the start of the counter area.
enum CounterWord : int {
    kErrCsc = 0,       // CSC validation flags
    kErrMatch = 1,     // matching validation flags
    kNumLong = 2,      // number of long columns
    kNumChunks = 3,    // chunks of the long-column search
    kDone = 4,         // 0 while rounds run; 1 after a round that flipped nothing;
                       // 2 if that round had candidates (a broken invariant)
    kRoundsRun = 5,    // search passes run so far
    kCycles = 6,       // u64 in words 6-7: cycles flipped in all rounds
    kRoundBase = 8,    // per-round words, kSlotWords per slot of the ring
    kTabUsed = 72,     // u64 in words 72-73: pool words taken by the row-list hash tables
    kTabRows = 74,     // row lists that got a hash table
    kColDone = 75,     // buckets whose column scan has finished (the transpose's part 2)
    kBigSubs = 76,     // oversized sub-buckets listed for the grid-wide placement
    kSpreadBase = 128, // sub-list counters of the wave-per-root hand-off (below)
};

// Per-round words of one ring slot.
enum SlotWord : int {
    kCand = 0,         // roots with a Step-C winner
    kApplied = 1,      // cycles flipped
    kRoots = 2,        // roots to search in this round (incremental mode)
    kHeavy = 4,        // flipped rows whose mate columns are refreshed by the whole grid
    kSlotWords = 8,
};

__host__ __device__ inline int slot_word(int slot, int w) { return kRoundBase + kSlotWords * slot + w; }

// The roots the tile kernels hand to the wave-per-root kernel go to kSpread
// sub-lists per round (by block index), each with its own counter in its own
// 128-byte line: appends from the whole grid would otherwise queue on one
// counter address.  Sub-list s of a round holds at most `cap` roots, at
// medium[s * cap ...).
constexpr int kSpread = 64;

// Row lists longer than this get a hash table in global memory (column ->
// place in the list; built once per call, after the transpose).
constexpr int kRowSetMin = 2048;
// Sub-buckets listed for the grid-wide placement, at most (the rest are
// placed by one block each).
constexpr int kMaxBigSubs = 1024;
// Flipped rows with more entries than this get their mate columns refreshed
// by the whole grid rather than one block.
constexpr int32_t kHeavyRow = 4096;
constexpr int kSpreadStride = 32;  // words between two sub-list counters
constexpr int kCounterWords = kSpreadBase + kSlots * kSpread * kSpreadStride;
__host__ __device__ inline int spread_word(int slot, int s) {
    return kSpreadBase + (slot * kSpread + s) * kSpreadStride;
}

// Append to a device list whose length is *counter: every active lane of the
// wave with want set gets its own slot (returned; -1 for the others), and
// the wave adds to the counter once.  Many lanes appending at once would
// otherwise queue on the one counter address.  All active lanes of the wave
// must call it together.
__device__ __forceinline__ int32_t wave_append(int32_t* counter, bool want) {
    const unsigned long long m = __ballot(want);
    if (m == 0ull) return -1;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll(m) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, (int32_t)__popcll(m));
    base = __shfl(base, leader, 64);
    return want ? base + (int32_t)__popcll(m & ((1ull << lane) - 1ull)) : -1;
}

// Matrix in CSC form (device pointers).
struct Csc {
    int32_t n;
    int64_t nnz;
    const int64_t* col_ptr;
    const int32_t* row_idx;
    const double* w;
};

// Device arrays carved from the caller's workspace.
struct Work {
    int32_t* mr;        // m_i: column matched to row i
    int32_t* mc;        // m_j: row matched to column j
    double* wm;         // w(m_j, j)
    double* best_g;     // Step-C winner of root j: gain
    int32_t* best_i;    //   row i (-1: none)
    int32_t* best_c;    //   other column c = m_i
    int64_t* best_k;    //   position of {i, j}
    int64_t* best_p;    //   position of {m_j, m_i}
    unsigned long long* dgain;  // Step D: max gain bits per column
    int32_t* droot;     // Step D: smallest root among the max-gain ones
    int32_t* cand;      // compacted list of roots with a Step-C winner
    int32_t* long_list; // columns searched by the split kernel
    int64_t* chunk_off; // chunk prefix per long column (n_long + 1)
    int32_t* chunk_col; // long column (index into long_list) of every chunk
    double* part_g;     // per-chunk partial winners (position keyed)
    int32_t* part_c;
    int64_t* part_k;
    int64_t* part_p;
    double* tree_a;     // tree-sum partials
    double* tree_b;
    uint32_t* bitmap;   // column-start bitmap for CSC validation
    int32_t* counters;  // kCounterWords
    double* result;     // [0] = total, [1] = initial weight
    int64_t max_chunks;
    // pattern transpose (row lists) and per-entry mate columns, for the
    // transposed probe
    int64_t* rowptr;    // n + 1: row lists laid out by the column matched to
                        // each row when the call starts (slot order)
    int2* rsl;          // n: (start, length) of the row list of the row matched to column j
    int32_t* cp32;      // n + 1: 32-bit copy of col_ptr (transposed probes, nnz < 2^31)
    int32_t* pm;        // n: CSC position of column j's matched entry {m_j, j} (transposed
                        // probes): the rows i > m_j of column j are the positions after it
    int32_t* colidx;    // nnz: columns of each row (any order within a row)
    int32_t* cscpos;    // nnz: CSC position of each row-list entry (transposed probes need nnz < 2^31);
                        // null when the lists are built without positions (probe 5)
    int32_t* mrk;       // nnz: m_i of the row of CSC entry k
    int32_t* rtab;      // n: offset in tabs of the hash table of the row list at slot j (-1: none);
                        // moves with rsl; null when the solve keeps no tables
    int32_t* tabs;      // nnz + 64: pool of the hash tables of the long row lists (keys, then values)
    int32_t* tab_plan;  // 3 (nnz / kRowSetMin + 2): the tables' fill plan (first units, places)
    int32_t* rowcnt;    // n: row counts, then fill cursors
    int64_t* scan_sums; // block sums of the row-count scan
    int32_t* flips;     // 4 per flipped cycle: (i, new mate j), (l, new mate c)
    int32_t* dirty;     // n: root must be searched again (incremental mode)
    int32_t* dirty_list;// n: the roots to search next round
    int32_t* medium;    // n + kSpread * 64: roots for the wave-per-root search (this round), in sub-lists
    int32_t* heavy;     // n: new mate columns of the flipped rows with long lists (this round)
    int32_t* round_stats; // 3 x kMaxRoundStats: candidates, flips, roots searched
    // staging of the bucketed transpose
    int32_t* tile_col;  // first column of every pass-1 tile (the column holding its first entry)
    int32_t* tp_row;
    int32_t* tp_col;
    int32_t* tp_pos;
    int32_t* tp_cnt;    // tile-major (tile, bucket) counts, then their scan inside each part of tiles
    int64_t* tp_off;    // per (part of tiles, bucket): where its entries of that bucket begin,
                        // counted from the bucket's start
    int64_t* tp_bstart; // bucket starts (+ nnz)
    int64_t* tp_btot;   // bucket totals
    int64_t* tp_sums;
    int32_t* tp_row2;   // pass-2 output, grouped by sub-bucket
    int32_t* tp_col2;
    int32_t* tp_pos2;
    int64_t* tp_sub;    // start of every sub-bucket (+ total)
    int32_t* tp_bigcnt; // oversized buckets (kTpSub) or sub-buckets (kSubSlots): counts, then places, per tile
    int32_t* tp_biglist; // oversized sub-buckets (at most kMaxBigSubs)
    // batched solves (nullptr otherwise): the block of every packed column and
    // per-block flip flags / counts
    const int32_t* mat_of_col;
    int32_t* item_flag;
    unsigned long long* item_cycles;
};

// One matrix of a batch: its caller-owned device arrays and its place in the
// packed block-diagonal matrix.
struct BatchItem {
    const int64_t* col_ptr;
    const int32_t* row_idx;
    const double* w;
    const int32_t* mate_in;   // improve: starting matching; match: unused
    int32_t* perm_out;
    int64_t n;
    int64_t nnz;
    int64_t col_off;          // first packed column (= first packed row)
    int64_t nnz_off;          // first packed entry
};

// Device-side tables of a batch (carved from the workspace; filled by the host).
struct BatchPlan {
    int32_t count;
    int64_t n_tot, nnz_tot;
    BatchItem* items;
    int32_t* col_chunk_item; int64_t* col_chunk_first; int32_t ncol_chunks;
    int32_t* ent_chunk_item; int64_t* ent_chunk_first; int32_t nent_chunks;
    int32_t* run_item; int64_t* run_first; int32_t nruns;
    int64_t* item_run0;       // first tree run of every item
    double* partial;          // tree run sums
    int64_t* col_ptr;         // packed matrix
    int32_t* row_idx;
    double* w;
    int32_t* mate;
    int32_t* mat_of_col;
    int32_t* item_flag;
    int32_t* item_rounds;
    unsigned long long* item_cycles;
    int32_t* item_unmatched;
    int32_t* item_err;        // [0]: malformed input flags
    double* item_total;
    double* item_init;
};

// Counter words of the matching phase.
enum McmWord : int {
    kMcmProposals = 0,
    kMcmListLen = 1,
    kMcmFrontier = 2,
    kMcmNext = 3,
    kMcmLevelLen = 4,
    kMcmAugmented = 5,
    kMcmDone = 8,         // greedy: a round found no proposal (later rounds do nothing)
    kMcmRounds = 9,       // greedy: proposal rounds run
    kMcmLevels = 10,      // BFS: levels with a nonempty frontier
    kMcmWords = 16,
};

// Device arrays of the initial-matching phase (greedy + multi-source BFS).
struct Mcm {
    int32_t* mc;        // column -> row (-1: unmatched)
    int32_t* mr;        // row -> column (-1: unmatched)
    int32_t* prop_row;  // greedy: row proposed to
    double* prop_w;     // greedy: its weight
    unsigned long long* rkey;  // greedy: max proposal key per row
    int32_t* racc;      // greedy: accepted proposer per row
    int32_t* list;      // greedy: proposing columns
    int32_t* tree_row;  // BFS: tree (root column) of each visited row, -1
    int32_t* tree_col;  // BFS: tree of each frontier column
    int32_t* parent;    // BFS: parent column of each visited row
    int32_t* end_row;   // BFS: chosen endpoint per tree (root column)
    unsigned long long* pkey;  // BFS: max parent key per row
    int32_t* touched;   // BFS: row listed in the current level
    int32_t* front_a;   // BFS: frontier buffers
    int32_t* front_b;
    int32_t* level;     // BFS: rows of the current level
    int32_t* counters;  // kMcmWords
};

size_t workspace_layout(int32_t n, int64_t nnz, char* base, Work* out, Mcm* mcm = nullptr);

// Launch wrappers (all asynchronous on `s`; return the launch status).
hipError_t launch_check_csc(const Csc& A, const Work& W, hipStream_t s, int cus);
hipError_t launch_init_match(const Csc& A, const Work& W, const int32_t* mate_in,
                             int32_t long_threshold, hipStream_t s);
hipError_t launch_long_chunks(const Work& W, const Csc& A, hipStream_t s);
hipError_t launch_search(const Csc& A, const Work& W, int tile_width, int32_t long_threshold,
                         int slot, bool has_long, int probe, bool listed, bool incremental, hipStream_t s,
                         int cus);
hipError_t launch_round_end(const Work& W, int slot, bool listed, int32_t n, hipStream_t s);
hipError_t launch_collect(const Csc& A, const Work& W, int slot, hipStream_t s, int cus);
hipError_t launch_transpose(const Csc& A, const Work& W, int32_t long_threshold, bool has_long,
                            bool positions, hipStream_t s, int cus);
// The bucket transpose (it also fills mrk) works for this size; it is the
// one that can go without positions.  launch_transpose_buckets queues its
// first pass (up to the bucket scatter), launch_transpose_rest the others
// (with big, oversized buckets are split by the whole grid); the long
// lists' hash tables are filled by launch_rowsets (when W.rtab is set).
// Its kernels return at once if the matching check failed.
bool transpose_in_buckets(int64_t n, int64_t nnz);
hipError_t launch_transpose_buckets(const Csc& A, const Work& W, bool positions, hipStream_t s, int cus);
hipError_t launch_transpose_rest(const Csc& A, const Work& W, bool positions, bool big, hipStream_t s, int cus);
hipError_t launch_rowsets(const Csc& A, const Work& W, hipStream_t s, int cus);
hipError_t launch_mrk_update(const Csc& A, const Work& W, int slot, bool incremental, hipStream_t s, int cus);
hipError_t launch_resolve(const Work& W, int slot, hipStream_t s, int cus);
hipError_t launch_apply(const Csc& A, const Work& W, int slot, bool transposed, hipStream_t s,
                        int cus);
// gate: null, or a device flag; the sum then runs only if the flag is nonzero
hipError_t launch_tree_sum(const double* x, int64_t m, const Work& W, double* out, hipStream_t s,
                           const int32_t* gate = nullptr);
hipError_t launch_copy_gated(const int32_t* src, int32_t* dst, int64_t n, const int32_t* gate, hipStream_t s,
                             int cus);
hipError_t launch_mcm_init(const Csc& A, const Mcm& M, const Work& W, int32_t long_threshold,
                           hipStream_t s, int cus);
hipError_t launch_greedy_round(const Csc& A, const Mcm& M, const Work& W, int heavy,
                               int32_t long_threshold, bool has_long, hipStream_t s, int cus);
hipError_t launch_bfs_roots(const Csc& A, const Mcm& M, hipStream_t s, int cus);
hipError_t launch_bfs_level(const Csc& A, const Mcm& M, int level, int heavy, hipStream_t s, int cus);
hipError_t launch_bfs_augment(const Csc& A, const Mcm& M, hipStream_t s, int cus);
hipError_t launch_pack(const BatchPlan& P, bool with_mates, hipStream_t s, int cus);
// skip (nullable): blocks with skip[b] != 0 keep their perm_out untouched.
hipError_t launch_unpack(const BatchPlan& P, const int32_t* mc, hipStream_t s, int cus,
                         const int32_t* skip = nullptr);
hipError_t launch_seg_tree(const BatchPlan& P, const double* x, double* out, hipStream_t s, int cus);
hipError_t launch_item_rounds(const BatchPlan& P, const int32_t* done, hipStream_t s);
hipError_t launch_item_unmatched(const BatchPlan& P, const int32_t* mc, hipStream_t s, int cus);

}  // namespace hwpm
