// Internal declarations shared by the HIP kernels and the C-ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hwpm {

constexpr int32_t kNoRoot = 0x7fffffff;   // empty Step-D slot
constexpr int kSlots = 8;                  // ring of per-round counter pairs
constexpr int kLongChunk = 1024;           // entries per block in the long-column search
constexpr int kTreeBlock = 2048;           // leaves summed by one tree-sum block

// Counter words (int32) at the start of the counter area.
enum CounterWord : int {
    kErrCsc = 0,       // CSC validation flags
    kErrMatch = 1,     // matching validation flags
    kNumLong = 2,      // number of long columns
    kNumChunks = 3,    // chunks of the long-column search
    kRoundBase = 8,    // [kRoundBase + 2*slot] = candidates, [+1] = applied
    kCounterWords = 64,
};

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
    double* part_g;     // per-chunk partial winners
    int32_t* part_i;
    int32_t* part_c;
    int64_t* part_k;
    int64_t* part_p;
    double* tree_a;     // tree-sum partials
    double* tree_b;
    uint32_t* bitmap;   // column-start bitmap for CSC validation
    int32_t* counters;  // kCounterWords
    double* result;     // [0] = total, [1] = initial weight
    int64_t max_chunks;
};

size_t workspace_layout(int32_t n, int64_t nnz, char* base, Work* out);

// Launch wrappers (all asynchronous on `s`; return the launch status).
hipError_t launch_check_csc(const Csc& A, const Work& W, hipStream_t s, int cus);
hipError_t launch_init_match(const Csc& A, const Work& W, const int32_t* mate_in,
                             int32_t long_threshold, hipStream_t s);
hipError_t launch_long_chunks(const Work& W, const Csc& A, hipStream_t s);
hipError_t launch_search(const Csc& A, const Work& W, int tile_width, int32_t long_threshold,
                         int slot, bool has_long, hipStream_t s, int cus);
hipError_t launch_resolve(const Work& W, int slot, hipStream_t s, int cus);
hipError_t launch_apply(const Csc& A, const Work& W, int slot, hipStream_t s, int cus);
hipError_t launch_tree_sum(const double* x, int64_t m, const Work& W, double* out, hipStream_t s);

}  // namespace hwpm
