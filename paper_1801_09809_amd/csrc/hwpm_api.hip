// C ABI of libhwpm.so (declared in include/hwpm.h): argument checks, the
// workspace carve-up, and the host round loop that launches the kernels of
// hwpm_kernels.hip and reads back two counters per round.
#include <chrono>
#include <mutex>
#include <new>
#include <vector>
#include <string.h>

#include "hwpm.h"
#include "hwpm_internal.h"
#include "hwpm_serving.h"

using namespace hwpm;

struct hwpm_handle_s {
    int device;
    hipStream_t stream;
    int cus;
    void* scratch;        // this device's copy of the static workspace (hwpm_improve_static), or null
    hipStream_t cap;      // private stream that repeated batches of launches are captured on
    bool has_tune;        // batches resolve default launch configurations from `tune`
    hwpm_tune_table tune;
    int32_t* host;        // pinned host buffer for counter / result readback
    // 0-7: stage events; 8 + 4*b .. 8 + 4*b + 3: the stages of the b-th
    // round of a batch of queued rounds
    hipEvent_t ev[8 + 8 * kSlots];  // 8 stage events, two sets of 4 per round of a batch
    // the set-up readback done (with the system-scope release, so the host
    // may read what the copies before it wrote) while later work still runs
    hipEvent_t ready;
};

namespace {

constexpr int kDefaultTile = 4;
constexpr int kDefaultProbe = 3;
constexpr int32_t kLongThreshold = 256;   // longer columns use the split search
// The report of a run is one range of the workspace, read back with one
// copy into the pinned buffer at int32 index kHostReport: the results
// (W.result), the per-round statistics (W.round_stats) and the first
// kReportCounters counter words (the workspace lays them out in that order).
constexpr int kReportCounters = 8;
static_assert(kErrMatch < kReportCounters && kNumLong < kReportCounters && kCycles + 2 <= kReportCounters,
              "report counter words");
constexpr int kHostReport = 64;
constexpr size_t kReportMaxBytes = 256 + 3 * kMaxRoundStats * sizeof(int32_t) + 256;
constexpr size_t kHostBytes = kHostReport * sizeof(int32_t) + kReportMaxBytes;

// Where the report's parts sit, in bytes from W.result.
struct Report {
    size_t stats, counters, bytes;  // bytes: up to the end of the counter words read
};
Report report_of(const Work& W) {
    Report r;
    r.stats = (size_t)((const char*)W.round_stats - (const char*)W.result);
    r.counters = (size_t)((const char*)W.counters - (const char*)W.result);
    r.bytes = r.counters + kReportCounters * sizeof(int32_t);
    return r;
}
constexpr int64_t kMaxNnz = (int64_t)1 << 40;

// The workspace of hwpm_improve_static: a fixed device array, one copy per
// GPU, held until the process ends.  Host code never uses the array's name as
// an address: the device address of each GPU's copy is looked up once, with
// that device current, and kept in g_scratch.
constexpr size_t kStaticScratchBytes = HWPM_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (which is `device`), or
// null if the runtime cannot give it.
void* static_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch[device] = ptr;
    }
    return g_scratch[device];
}

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

#define HIP_TRY(expr)                                  \
    do {                                               \
        if ((expr) != hipSuccess) return HWPM_EDEVICE; \
    } while (0)

int check_csc_args(const hwpm_csc* A) {
    if (!A) return HWPM_EINVAL;
    if (A->n < 0 || A->nnz < 0) return HWPM_EINVAL;
    if (A->n == INT32_MAX || A->nnz >= kMaxNnz) return HWPM_ETOOBIG;
    if (!A->col_ptr) return HWPM_EINVAL;
    if (A->nnz > 0 && (!A->row_idx || !A->weight)) return HWPM_EINVAL;
    return HWPM_OK;
}

Csc to_csc(const hwpm_csc* A) {
    Csc c;
    c.n = A->n;
    c.nnz = A->nnz;
    c.col_ptr = A->col_ptr;
    c.row_idx = A->row_idx;
    c.w = A->weight;
    return c;
}

// Run the CSC validation; returns HWPM_OK / HWPM_EBADCSC / HWPM_EDEVICE.
int run_check(hwpm_handle h, const Csc& A, const Work& W) {
    HIP_TRY(hipMemsetAsync(W.counters, 0, kCounterWords * sizeof(int32_t), h->stream));
    HIP_TRY(hipMemsetAsync(W.bitmap, 0, ((size_t)A.nnz + 1) / 32 * 4 + 8, h->stream));
    HIP_TRY(launch_check_csc(A, W, h->stream, h->cus));
    HIP_TRY(hipMemcpyAsync(h->host, W.counters, 4 * sizeof(int32_t), hipMemcpyDeviceToHost,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return h->host[kErrCsc] ? HWPM_EBADCSC : HWPM_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
    return ms;
}

// A batch of launches captured into a HIP graph, replayed as one launch.
struct CapturedBatch {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    CapturedBatch() = default;
    CapturedBatch(const CapturedBatch&) = delete;
    CapturedBatch& operator=(const CapturedBatch&) = delete;
    ~CapturedBatch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// Queue a batch of launches on stream s as one graph launch.  queue(stream)
// issues the launches on the stream it is given; the first call captures them
// on the handle's capture stream, later calls replay the same graph (the
// caller only replays batches whose launch arguments are all the same).  The
// batches contain kernels only: no memset or copy nodes.
template <class F>
int replay(hwpm_handle h, hipStream_t s, CapturedBatch& C, hwpm_stats* S, F queue) {
    if (!C.exec) {
        HIP_TRY(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
        const int st = queue(h->cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(h->cap, &g);
        if (st != HWPM_OK || e != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            return st != HWPM_OK ? st : HWPM_EDEVICE;
        }
        C.graph = g;
        HIP_TRY(hipGraphInstantiate(&C.exec, g, nullptr, nullptr, 0));
    }
    HIP_TRY(hipGraphLaunch(C.exec, s));
    ++S->graph_launches;
    return HWPM_OK;
}

// The rounds of Section 5.3 from the perfect matching mate_in (CSC already
// validated or trusted).  Fills the round statistics of *Sp.
int run_improve(hwpm_handle h, const Csc& A, const Work& W, const int32_t* mate_in,
                int32_t* perm_out, double* total_out, const hwpm_options& opt, hwpm_stats* Sp,
                const BatchPlan* BP = nullptr) {
    hwpm_stats& S = *Sp;
    const int32_t n = A.n;
    hipStream_t s = h->stream;
    const bool timing = opt.timing == 1;   // every stage
    const bool tsearch = opt.timing != 0;  // the search stage (both levels)
    hipEvent_t* ev = h->ev;
    // a perfect matching takes n distinct entries: with fewer, none lies in
    // the pattern (and the set-up's search assumes at least one entry)
    if (A.nnz < (int64_t)n) return HWPM_EBADMATCH;
    int probe = opt.probe ? opt.probe : kDefaultProbe;
    // default tile: 4 lanes per root for short columns, 8 from about 20
    // entries per column on (the chunked kernel then holds 32 per tile either way)
    const int tile = opt.tile_width ? opt.tile_width
                                    : ((probe == 3 || probe == 5) && A.nnz > 20 * (int64_t)A.n ? 8 : kDefaultTile);
    // the row lists keep 32-bit CSC positions
    if (probe >= 2 && A.nnz >= ((int64_t)1 << 31)) probe = 1;
    // probe 5: the chunked kernels over row lists built without CSC positions
    // (a hit or a mate refresh searches its entry's position instead)
    const bool light = probe == 5 && transpose_in_buckets(A.n, A.nnz);
    if (probe == 5) probe = 3;
    S.probe_used = light ? 5 : probe;
    S.tile_used = tile;
    const bool transposed = probe >= 2;
    const bool incremental = probe >= 3 && !opt.full_search;
    Work Wr = W;  // the round kernels' view of the workspace
    if (light) Wr.cscpos = nullptr;
    // 2. set-up: mates, matched weights, matching validation, long columns
    if (timing) HIP_TRY(hipEventRecord(ev[0], s));
    HIP_TRY(hipMemsetAsync(W.counters, 0, kCounterWords * sizeof(int32_t), s));
    HIP_TRY(launch_init_match(A, W, mate_in, kLongThreshold, s));
    HIP_TRY(launch_tree_sum(W.wm, n, W, &W.result[1], s));
    const Report rep = report_of(W);
    if (rep.stats < 4 * sizeof(double) || rep.counters < rep.stats + 3 * kMaxRoundStats * sizeof(int32_t) ||
        rep.bytes > kReportMaxBytes)
        return HWPM_EINTERNAL;
    char* const rhost = (char*)(h->host + kHostReport);
    const int32_t* const rcount = (const int32_t*)(rhost + rep.counters);
    HIP_TRY(hipMemcpyAsync(rhost, W.result, rep.bytes, hipMemcpyDeviceToHost, s));
    if (timing) HIP_TRY(hipEventRecord(ev[1], s));
    // The bucket transpose's first pass needs nothing the host reads back
    // here: it is queued before the wait, so the device goes on while the
    // host checks the matching (its kernels return at once if the check
    // failed).  The rest follows, with the split of oversized buckets over
    // the grid on matrices with long columns (skewed ones); the slots of
    // long row lists' hash tables are noted whatever the columns, and the
    // tables are filled only if the rounds use them.
    const bool early = transposed && transpose_in_buckets(n, A.nnz);
    if (early) {
        HIP_TRY(hipEventRecord(h->ready, s));
        if (timing) HIP_TRY(hipEventRecord(ev[2], s));
        if (incremental) HIP_TRY(hipMemsetAsync(W.dirty, 0, (size_t)n * sizeof(int32_t), s));
        HIP_TRY(launch_transpose_buckets(A, W, !light, s, h->cus));
        HIP_TRY(hipEventSynchronize(h->ready));
    } else {
        HIP_TRY(hipStreamSynchronize(s));
    }
    if (rcount[kErrMatch]) return HWPM_EBADMATCH;
    if (BP) HIP_TRY(launch_seg_tree(*BP, W.wm, BP->item_init, s, h->cus));
    const int32_t n_long = rcount[kNumLong];
    // hash tables of the long row lists only for matrices with long columns
    // (where long row lists occur on real patterns); elsewhere the rounds see
    // no tables and the pass that fills them is not launched
    if (n_long == 0) Wr.rtab = nullptr;
    if (n_long > 0) HIP_TRY(launch_long_chunks(W, A, s));
    S.long_columns = n_long;
    memcpy(&S.init_weight, rhost + sizeof(double), sizeof(double));
    if (early) {
        HIP_TRY(launch_transpose_rest(A, W, !light, n_long > 0, s, h->cus));
        HIP_TRY(launch_rowsets(A, Wr, s, h->cus));
        if (timing) HIP_TRY(hipEventRecord(ev[3], s));  // read at the end
    } else if (transposed) {
        if (timing) HIP_TRY(hipEventRecord(ev[2], s));
        if (incremental) HIP_TRY(hipMemsetAsync(W.dirty, 0, (size_t)n * sizeof(int32_t), s));
        Work Wt = W;
        Wt.rtab = Wr.rtab;
        HIP_TRY(launch_transpose(A, Wt, kLongThreshold, n_long > 0, !light, s, h->cus));
        if (timing) HIP_TRY(hipEventRecord(ev[3], s));  // read at the end
    }

    // 3. rounds.  In incremental mode the first round searches every root and
    // later rounds only the roots the previous flips touched (the others keep
    // their Step-C records, which cannot have changed).  Rounds are queued in
    // batches of 2, 4, 8, 8, ... with no host round trip inside a
    // batch: the round that flips nothing raises a device flag and every
    // round kernel queued after it returns at once.
    // With timing, a batch's events are read while the next batch (or the
    // output stage) runs: the batches alternate between two event sets.
    int32_t round = 0;  // rounds queued
    int32_t batch = 2;
    int32_t done = 0, rounds_run = 0;
    int32_t batches = 0;
    int32_t pend_first = 0, pend_nb = 0, pend_ran = 0, pend_set = 0;  // a batch whose events are unread
    auto read_round_events = [&]() {
        for (int32_t b = 0; b < pend_nb; ++b) {
            const int32_t r = pend_first + b;
            if (r >= pend_ran) break;  // queued after the loop ended: did nothing
            hipEvent_t* e = ev + 8 + 4 * (kSlots * pend_set + b);
            const float ms = elapsed(e[0], e[1]);
            S.ms_search += ms;
            if (r == 0) S.ms_search_first = ms;
            if (r < HWPM_MAX_ROUND_STATS) S.round_ms_search[r] = ms;
            if (!timing) continue;
            S.ms_resolve += elapsed(e[1], e[2]);
            S.ms_apply += elapsed(e[2], e[3]);
        }
        pend_nb = 0;
    };
    // 4. outputs: the total weight, the permutation, the per-round
    // statistics and the cycle count, read back into the pinned buffer
    auto queue_outputs = [&](const int32_t* gate) -> int {
        if (timing) HIP_TRY(hipEventRecord(ev[6], s));
        HIP_TRY(launch_tree_sum(W.wm, n, W, &W.result[0], s, gate));
        if (gate)
            HIP_TRY(launch_copy_gated(W.mc, perm_out, n, gate, s, h->cus));
        else
            HIP_TRY(hipMemcpyAsync(perm_out, W.mc, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        if (BP) {
            HIP_TRY(launch_seg_tree(*BP, W.wm, BP->item_total, s, h->cus));
            HIP_TRY(launch_unpack(*BP, W.mc, s, h->cus));
        }
        HIP_TRY(hipMemcpyAsync(rhost, W.result, rep.bytes, hipMemcpyDeviceToHost, s));
        if (timing) HIP_TRY(hipEventRecord(ev[7], s));
        return HWPM_OK;
    };
    // the kernels of rounds r0 .. r0 + nb - 1, on stream st
    auto queue_rounds = [&](hipStream_t st, int32_t r0, int32_t nb, int32_t set) -> int {
        for (int32_t b = 0; b < nb; ++b) {
            const int32_t r = r0 + b;
            const int slot = r % kSlots;
            const bool listed = incremental && r > 0;
            hipEvent_t* e = ev + 8 + 4 * (kSlots * set + b);
            if (tsearch) HIP_TRY(hipEventRecord(e[0], st));
            HIP_TRY(launch_search(A, Wr, tile, kLongThreshold, slot, n_long > 0, probe, listed, incremental, st,
                                  h->cus));
            if (tsearch) HIP_TRY(hipEventRecord(e[1], st));
            HIP_TRY(launch_collect(A, W, slot, st, h->cus));
            HIP_TRY(launch_resolve(W, slot, st, h->cus));
            if (timing) HIP_TRY(hipEventRecord(e[2], st));
            HIP_TRY(launch_apply(A, Wr, slot, transposed, st, h->cus));
            if (transposed) HIP_TRY(launch_mrk_update(A, Wr, slot, incremental, st, h->cus));
            if (BP) HIP_TRY(launch_item_rounds(*BP, W.counters + kDone, st));
            if (timing) HIP_TRY(hipEventRecord(e[3], st));
            HIP_TRY(launch_round_end(W, slot, listed, n, st));
        }
        return HWPM_OK;
    };
    // Batches from the third on hold kSlots rounds that start at the same ring
    // slot (rounds 6, 14, 22, ...), so their launches are all the same: with
    // opt.graph they replay one graph captured at the first of them.
    CapturedBatch rounds_graph;
    for (;;) {
        int32_t nb = batch;
        if (opt.max_rounds > 0 && opt.max_rounds - round < nb) nb = opt.max_rounds - round;
        if (nb <= 0) break;  // the round cap
        const int32_t set = batches & 1;
        const bool replayable = opt.graph && !tsearch && nb == kSlots && round % kSlots == kSlots - 2;
        const int qs = replayable
                           ? replay(h, s, rounds_graph, &S, [&](hipStream_t c) { return queue_rounds(c, round, nb, set); })
                           : queue_rounds(s, round, nb, set);
        if (qs != HWPM_OK) return qs;
        round += nb;
        ++batches;
        // single solves queue the output stage behind every batch, gated on
        // the device's done flag: the batch that ends the rounds then needs
        // no further host round trip (for the others it does nothing)
        if (!BP) {
            const int st = queue_outputs(W.counters + kDone);
            if (st != HWPM_OK) return st;
        }
        HIP_TRY(hipMemcpyAsync(h->host, W.counters + kDone, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        if (tsearch) read_round_events();  // the previous batch's, while this one runs
        HIP_TRY(hipStreamSynchronize(s));
        done = h->host[0];
        rounds_run = h->host[1];
        pend_first = round - nb;
        pend_nb = nb;
        pend_ran = rounds_run;
        pend_set = set;
        // A round with candidates always flips at least one cycle (the
        // candidate whose other column has the largest matched row).
        if (done == 2) return HWPM_EINTERNAL;
        if (done) break;
        batch = 2 * batch < kSlots ? 2 * batch : kSlots;
    }
    if (!done) S.hit_round_cap = 1;
    S.rounds = done ? rounds_run : round;
    static_assert(kMaxRoundStats == HWPM_MAX_ROUND_STATS, "round statistics sizes");
    const int32_t n_stats = S.rounds < kMaxRoundStats ? S.rounds : kMaxRoundStats;
    if (BP || !done) {  // the output stage has not run yet (batches, or the round cap)
        const int st = queue_outputs(nullptr);
        if (st != HWPM_OK) return st;
        if (tsearch) read_round_events();  // while the output stage runs
        HIP_TRY(hipStreamSynchronize(s));
    } else if (tsearch) {
        read_round_events();
    }
    if (timing) {
        S.ms_setup = elapsed(ev[0], ev[1]);
        if (transposed) S.ms_transpose = elapsed(ev[2], ev[3]);
        S.ms_final = elapsed(ev[6], ev[7]);
    }
    unsigned long long cycles = 0;
    memcpy(&cycles, rcount + kCycles, sizeof(cycles));
    S.cycles_applied = (int64_t)cycles;
    if (n_stats > 0) {
        const int32_t* st = (const int32_t*)(rhost + rep.stats);
        memcpy(S.round_candidates, st, (size_t)n_stats * sizeof(int32_t));
        memcpy(S.round_applied, st + kMaxRoundStats, (size_t)n_stats * sizeof(int32_t));
        memcpy(S.round_roots, st + 2 * kMaxRoundStats, (size_t)n_stats * sizeof(int32_t));
    }
    double total;
    memcpy(&total, rhost, sizeof(double));
    S.final_weight = total;
    *total_out = total;
    return HWPM_OK;
}

int timed_check(hwpm_handle h, const Csc& A, const Work& W, bool timing, hwpm_stats* S) {
    hipEvent_t* ev = h->ev;
    if (timing) HIP_TRY(hipEventRecord(ev[0], h->stream));
    const int st = run_check(h, A, W);
    if (st != HWPM_OK) return st;
    if (timing) {
        HIP_TRY(hipEventRecord(ev[1], h->stream));
        HIP_TRY(hipEventSynchronize(ev[1]));
        S->ms_check = elapsed(ev[0], ev[1]);
    }
    return HWPM_OK;
}

int check_options(const hwpm_options& opt) {
    if (opt.max_rounds < 0) return HWPM_EINVAL;
    const int tile = opt.tile_width ? opt.tile_width : kDefaultTile;
    if (tile != 4 && tile != 8 && tile != 16 && tile != 32 && tile != 64) return HWPM_EINVAL;
    const int probe = opt.probe ? opt.probe : kDefaultProbe;
    if (probe < 1 || probe > 5) return HWPM_EINVAL;
    if (probe >= 3 && tile == 64) return HWPM_EINVAL;
    if (opt.mcm_plain != 0 && opt.mcm_plain != 1) return HWPM_EINVAL;
    if (opt.full_search != 0 && opt.full_search != 1) return HWPM_EINVAL;
    if (opt.timing < 0 || opt.timing > 2) return HWPM_EINVAL;
    if (opt.graph != 0 && opt.graph != 1) return HWPM_EINVAL;
    return HWPM_OK;
}

// Phase I (Sections 5.1-5.2): greedy proposal rounds, then BFS phases until
// no augmenting path is found.  Leaves a perfect matching in M.mc, or returns
// HWPM_ESINGULAR.
int run_initial_matching(hwpm_handle h, const Csc& A, const Work& W, const Mcm& M, int heavy,
                         bool timing, bool graph, hwpm_stats* S) {
    hipStream_t s = h->stream;
    hipEvent_t* ev = h->ev;
    int32_t* host = h->host;
    if (timing) HIP_TRY(hipEventRecord(ev[0], s));
    HIP_TRY(hipMemsetAsync(W.counters, 0, kCounterWords * sizeof(int32_t), s));
    HIP_TRY(launch_mcm_init(A, M, W, kLongThreshold, s, h->cus));
    HIP_TRY(hipMemcpyAsync(host, W.counters + kNumLong, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const bool has_long = host[0] > 0;
    // greedy rounds, queued in batches of 1, 2, 4, 8, 8, ... (the round that
    // finds no proposal ends the loop on the device)
    HIP_TRY(hipMemsetAsync(M.counters, 0, kMcmWords * sizeof(int32_t), s));
    // batches of 8 rounds (and of 8 BFS levels, which start at an odd level)
    // are all the same: with graph they replay one captured graph
    CapturedBatch greedy_graph, level_graph;
    for (int32_t batch = 1;; batch = batch < 8 ? 2 * batch : 8) {
        auto queue = [&](hipStream_t st) -> int {
            for (int32_t b = 0; b < batch; ++b)
                HIP_TRY(launch_greedy_round(A, M, W, heavy, kLongThreshold, has_long, st, h->cus));
            return HWPM_OK;
        };
        const int qs = (graph && batch == 8) ? replay(h, s, greedy_graph, S, queue) : queue(s);
        if (qs != HWPM_OK) return qs;
        HIP_TRY(hipMemcpyAsync(host, M.counters + kMcmDone, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (host[0]) break;
    }
    S->greedy_rounds = host[1];
    if (timing) {
        HIP_TRY(hipEventRecord(ev[1], s));
        HIP_TRY(hipEventSynchronize(ev[1]));
        S->ms_greedy = elapsed(ev[0], ev[1]);
        HIP_TRY(hipEventRecord(ev[0], s));
    }
    int32_t phases = 0, levels = 0, unmatched = 0;
    bool first = true;
    for (;;) {
        HIP_TRY(hipMemsetAsync(M.counters, 0, kMcmWords * sizeof(int32_t), s));
        HIP_TRY(launch_bfs_roots(A, M, s, h->cus));
        HIP_TRY(hipMemcpyAsync(host, M.counters, kMcmWords * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        unmatched = host[kMcmFrontier];
        if (first) {
            S->greedy_cardinality = A.n - unmatched;
            first = false;
        }
        if (unmatched == 0) break;
        ++phases;
        // levels, queued in batches of 1, 2, 4, 8, 8, ...: a level with an
        // empty frontier does nothing, so the phase's levels end on the device
        for (int32_t level = 0, batch = 1;; batch = batch < 8 ? 2 * batch : 8) {
            auto queue = [&](hipStream_t st) -> int {
                for (int32_t b = 0; b < batch; ++b)
                    HIP_TRY(launch_bfs_level(A, M, level + b, heavy, st, h->cus));
                return HWPM_OK;
            };
            const int qs = (graph && batch == 8 && (level & 1)) ? replay(h, s, level_graph, S, queue) : queue(s);
            if (qs != HWPM_OK) return qs;
            level += batch;
            const int nw = (level & 1) ? kMcmNext : kMcmFrontier;  // next level's frontier
            HIP_TRY(hipMemcpyAsync(host, M.counters + nw, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (host[0] == 0) break;
        }
        HIP_TRY(launch_bfs_augment(A, M, s, h->cus));
        HIP_TRY(hipMemcpyAsync(host, M.counters, kMcmWords * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        levels += host[kMcmLevels];
        if (host[kMcmAugmented] == 0) break;  // no augmenting path: maximum reached
    }
    S->mcm_phases = phases;
    S->mcm_levels = levels;
    S->mcm_cardinality = A.n - unmatched;
    if (timing) {
        HIP_TRY(hipEventRecord(ev[1], s));
        HIP_TRY(hipEventSynchronize(ev[1]));
        S->ms_mcm = elapsed(ev[0], ev[1]);
    }
    return unmatched == 0 ? HWPM_OK : HWPM_ESINGULAR;
}


// Host-side description of a batch: offsets and the chunk / tree-run tables.
struct HostPlan {
    std::vector<BatchItem> items;
    std::vector<int32_t> col_chunk_item, ent_chunk_item, run_item;
    std::vector<int64_t> col_chunk_first, ent_chunk_first, run_first, item_run0;
    int64_t n_tot = 0, nnz_tot = 0;
};

constexpr int64_t kPackChunkHost = 4096;

// sizes_only: plan from n and nnz alone (the pointers are neither read nor checked).
int build_plan(int32_t count, const hwpm_csc* mats, const int32_t* const* mate_in,
               int32_t* const* perm_out, HostPlan* HP, bool sizes_only = false) {
    HP->items.resize(count);
    for (int32_t b = 0; b < count; ++b) {
        const hwpm_csc& A = mats[b];
        if (A.n < 0 || A.nnz < 0) return HWPM_EINVAL;
        if (!sizes_only && (!A.col_ptr || (A.nnz > 0 && (!A.row_idx || !A.weight)))) return HWPM_EINVAL;
        if (A.n > 0 && perm_out && !perm_out[b]) return HWPM_EINVAL;
        if (A.n > 0 && mate_in && !mate_in[b]) return HWPM_EINVAL;
        BatchItem& it = HP->items[b];
        it.col_ptr = A.col_ptr;
        it.row_idx = A.row_idx;
        it.w = A.weight;
        it.mate_in = mate_in ? mate_in[b] : nullptr;
        it.perm_out = perm_out ? perm_out[b] : nullptr;
        it.n = A.n;
        it.nnz = A.nnz;
        it.col_off = HP->n_tot;
        it.nnz_off = HP->nnz_tot;
        for (int64_t j = 0; j < A.n; j += kPackChunkHost) {
            HP->col_chunk_item.push_back(b);
            HP->col_chunk_first.push_back(j);
        }
        for (int64_t k = 0; k < A.nnz; k += kPackChunkHost) {
            HP->ent_chunk_item.push_back(b);
            HP->ent_chunk_first.push_back(k);
        }
        HP->item_run0.push_back((int64_t)HP->run_item.size());
        if (A.n > kTreeBlock) {
            if (A.n > (int64_t)kTreeBlock * kTreeBlock) return HWPM_ETOOBIG;
            for (int64_t r = 0; r < A.n; r += kTreeBlock) {
                HP->run_item.push_back(b);
                HP->run_first.push_back(r);
            }
        }
        HP->n_tot += A.n;
        HP->nnz_tot += A.nnz;
    }
    if (HP->n_tot >= INT32_MAX || HP->nnz_tot >= kMaxNnz) return HWPM_ETOOBIG;
    return HWPM_OK;
}

size_t batch_layout(const HostPlan& HP, int32_t count, char* base, BatchPlan* out) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    BatchPlan P{};
    P.count = count;
    P.n_tot = HP.n_tot;
    P.nnz_tot = HP.nnz_tot;
    P.items = (BatchItem*)take(HP.items.size() * sizeof(BatchItem));
    P.ncol_chunks = (int32_t)HP.col_chunk_item.size();
    P.col_chunk_item = (int32_t*)take(HP.col_chunk_item.size() * 4);
    P.col_chunk_first = (int64_t*)take(HP.col_chunk_first.size() * 8);
    P.nent_chunks = (int32_t)HP.ent_chunk_item.size();
    P.ent_chunk_item = (int32_t*)take(HP.ent_chunk_item.size() * 4);
    P.ent_chunk_first = (int64_t*)take(HP.ent_chunk_first.size() * 8);
    P.nruns = (int32_t)HP.run_item.size();
    P.run_item = (int32_t*)take(HP.run_item.size() * 4);
    P.run_first = (int64_t*)take(HP.run_first.size() * 8);
    P.item_run0 = (int64_t*)take(HP.item_run0.size() * 8);
    P.partial = (double*)take(HP.run_item.size() * 8 + 8);
    P.col_ptr = (int64_t*)take((size_t)(HP.n_tot + 1) * 8);
    P.row_idx = (int32_t*)take((size_t)HP.nnz_tot * 4);
    P.w = (double*)take((size_t)HP.nnz_tot * 8);
    P.mate = (int32_t*)take((size_t)HP.n_tot * 4);
    P.mat_of_col = (int32_t*)take((size_t)HP.n_tot * 4);
    P.item_flag = (int32_t*)take((size_t)count * 4);
    P.item_rounds = (int32_t*)take((size_t)count * 4);
    P.item_cycles = (unsigned long long*)take((size_t)count * 8);
    P.item_unmatched = (int32_t*)take((size_t)count * 4);
    P.item_err = (int32_t*)take(64);
    P.item_total = (double*)take((size_t)count * 8);
    P.item_init = (double*)take((size_t)count * 8);
    if (out) *out = P;
    return off;
}

// Copy the host tables into the batch region and clear the per-item counters.
int upload_plan(hwpm_handle h, const HostPlan& HP, const BatchPlan& P) {
    hipStream_t s = h->stream;
    auto up = [&](void* dst, const void* src, size_t bytes) {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    HIP_TRY(up(P.items, HP.items.data(), HP.items.size() * sizeof(BatchItem)));
    HIP_TRY(up(P.col_chunk_item, HP.col_chunk_item.data(), HP.col_chunk_item.size() * 4));
    HIP_TRY(up(P.col_chunk_first, HP.col_chunk_first.data(), HP.col_chunk_first.size() * 8));
    HIP_TRY(up(P.ent_chunk_item, HP.ent_chunk_item.data(), HP.ent_chunk_item.size() * 4));
    HIP_TRY(up(P.ent_chunk_first, HP.ent_chunk_first.data(), HP.ent_chunk_first.size() * 8));
    HIP_TRY(up(P.run_item, HP.run_item.data(), HP.run_item.size() * 4));
    HIP_TRY(up(P.run_first, HP.run_first.data(), HP.run_first.size() * 8));
    HIP_TRY(up(P.item_run0, HP.item_run0.data(), HP.item_run0.size() * 8));
    const size_t c = (size_t)P.count;
    HIP_TRY(hipMemsetAsync(P.item_flag, 0, c * 4, s));
    HIP_TRY(hipMemsetAsync(P.item_rounds, 0, c * 4, s));
    HIP_TRY(hipMemsetAsync(P.item_cycles, 0, c * 8, s));
    HIP_TRY(hipMemsetAsync(P.item_unmatched, 0, c * 4, s));
    HIP_TRY(hipMemsetAsync(P.item_err, 0, 64, s));
    HIP_TRY(hipStreamSynchronize(s));  // the host tables may be released now
    return HWPM_OK;
}

size_t batch_bytes(const HostPlan& HP, int32_t count) {
    return batch_layout(HP, count, nullptr, nullptr) +
           workspace_layout((int32_t)HP.n_tot, HP.nnz_tot, nullptr, nullptr);
}

// Per-item statistics after a packed solve (rounds reconstructed from the
// rounds in which each block flipped cycles; a block alone stops after its
// first round without flips, or at the cap).
int fill_item_stats(hwpm_handle h, const HostPlan& HP, const BatchPlan& P, const hwpm_options& opt,
                    double* totals, hwpm_item_stats* items) {
    const size_t c = (size_t)P.count;
    std::vector<int32_t> rounds(c);
    std::vector<unsigned long long> cycles(c);
    std::vector<double> tot(c), init(c);
    HIP_TRY(hipMemcpyAsync(rounds.data(), P.item_rounds, c * 4, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(cycles.data(), P.item_cycles, c * 8, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(tot.data(), P.item_total, c * 8, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(init.data(), P.item_init, c * 8, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (size_t b = 0; b < c; ++b) {
        const int32_t a = rounds[b];
        // alone, an empty matrix runs no search pass at all; any other runs
        // one pass per round that flipped cycles, plus the pass that finds none
        int32_t r = HP.items[b].n > 0 ? a + 1 : 0, cap = 0;
        if (opt.max_rounds > 0 && a >= opt.max_rounds) {
            r = opt.max_rounds;
            cap = 1;
        }
        if (totals) totals[b] = tot[b];
        if (items) {
            items[b].status = HWPM_OK;
            items[b].rounds = r;
            items[b].hit_round_cap = cap;
            items[b].reserved = 0;
            items[b].cycles_applied = (int64_t)cycles[b];
            items[b].init_weight = init[b];
            items[b].final_weight = tot[b];
        }
    }
    return HWPM_OK;
}

}  // namespace

extern "C" {

void hwpm_default_options(hwpm_options* opt) {
    if (!opt) return;
    opt->max_rounds = 0;
    opt->check_csc = 1;
    opt->timing = 0;
    opt->tile_width = 0;
    opt->probe = 0;
    opt->mcm_plain = 0;
    opt->full_search = 0;
    opt->graph = 1;
}

const char* hwpm_strerror(int status) {
    switch (status) {
        case HWPM_OK: return "ok";
        case HWPM_EINVAL: return "invalid argument";
        case HWPM_ESINGULAR: return "the matrix has no perfect matching";
        case HWPM_EBADCSC: return "malformed CSC matrix";
        case HWPM_EBADMATCH: return "initial matching is not a perfect matching inside the pattern";
        case HWPM_ENOMEM: return "workspace too small";
        case HWPM_ETOOBIG: return "matrix too large";
        case HWPM_EDEVICE: return "HIP runtime error";
        case HWPM_EINTERNAL: return "internal consistency check failed";
        case HWPM_PENDING: return "request pending";
        default: return "unknown status";
    }
}

int hwpm_create(hwpm_handle* out, int device, void* stream) {
    if (!out) return HWPM_EINVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return HWPM_EDEVICE;
    DeviceGuard g(device);
    if (!g.ok) return HWPM_EDEVICE;
    hwpm_handle h = new (std::nothrow) hwpm_handle_s();
    if (!h) return HWPM_EDEVICE;
    h->device = device;
    h->stream = (hipStream_t)stream;
    h->host = nullptr;
    h->scratch = static_scratch(device);  // once per device (the device is current here)
    h->cap = nullptr;
    h->has_tune = false;
    hwpm_default_tune_table(&h->tune);
    if (hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        h->cus <= 0)
        h->cus = 256;
    constexpr int kEvents = (int)(sizeof(h->ev) / sizeof(h->ev[0]));
    int ne = 0;
    bool ok = hipHostMalloc((void**)&h->host, kHostBytes, hipHostMallocDefault) == hipSuccess &&
              hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) == hipSuccess;
    while (ok && ne < kEvents) {
        // timing only (host data is always read after a stream synchronize):
        // no system-scope cache flush at each record
        ok = hipEventCreateWithFlags(&h->ev[ne], hipEventDisableSystemFence) == hipSuccess;
        if (ok) ++ne;
    }
    h->ready = nullptr;
    ok = ok && hipEventCreateWithFlags(&h->ready, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        for (int e = 0; e < ne; ++e) (void)hipEventDestroy(h->ev[e]);
        if (h->ready) (void)hipEventDestroy(h->ready);
        if (h->host) (void)hipHostFree(h->host);
        if (h->cap) (void)hipStreamDestroy(h->cap);
        delete h;
        return HWPM_EDEVICE;
    }
    *out = h;
    return HWPM_OK;
}

int hwpm_destroy(hwpm_handle h) {
    if (!h) return HWPM_OK;
    DeviceGuard g(h->device);
    (void)hipStreamSynchronize(h->stream);
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    (void)hipEventDestroy(h->ready);
    (void)hipHostFree(h->host);
    (void)hipStreamDestroy(h->cap);
    delete h;
    return HWPM_OK;
}

int hwpm_workspace_bytes(int32_t n, int64_t nnz, size_t* bytes) {
    if (!bytes || n < 0 || nnz < 0) return HWPM_EINVAL;
    if (n == INT32_MAX || nnz >= kMaxNnz) return HWPM_ETOOBIG;
    *bytes = workspace_layout(n, nnz, nullptr, nullptr);
    return HWPM_OK;
}

int hwpm_check_csc(hwpm_handle h, const hwpm_csc* A, void* workspace, size_t workspace_bytes) {
    if (!h) return HWPM_EINVAL;
    int st = check_csc_args(A);
    if (st != HWPM_OK) return st;
    const size_t need = workspace_layout(A->n, A->nnz, nullptr, nullptr);
    if (!workspace) return HWPM_EINVAL;
    if (workspace_bytes < need) return HWPM_ENOMEM;
    DeviceGuard g(h->device);
    if (!g.ok) return HWPM_EDEVICE;
    Work W;
    workspace_layout(A->n, A->nnz, (char*)workspace, &W);
    return run_check(h, to_csc(A), W);
}

int hwpm_improve(hwpm_handle h, const hwpm_csc* Ain, const int32_t* mate_in, int32_t* perm_out,
                 double* total_out, const hwpm_options* opt_in, hwpm_stats* stats,
                 void* workspace, size_t workspace_bytes) {
    const auto t_begin = std::chrono::steady_clock::now();
    if (!h) return HWPM_EINVAL;
    int st = check_csc_args(Ain);
    if (st != HWPM_OK) return st;
    hwpm_options opt;
    hwpm_default_options(&opt);
    if (opt_in) opt = *opt_in;
    st = check_options(opt);
    if (st != HWPM_OK) return st;
    const int32_t n = Ain->n;
    if (n > 0 && (!mate_in || !perm_out)) return HWPM_EINVAL;
    const size_t need = workspace_layout(n, Ain->nnz, nullptr, nullptr);
    if (n > 0 && !workspace) return HWPM_EINVAL;
    if (n > 0 && workspace_bytes < need) return HWPM_ENOMEM;

    hwpm_stats S;
    memset(&S, 0, sizeof(S));
    if (n == 0) {
        if (total_out) *total_out = 0.0;
        if (stats) *stats = S;
        return HWPM_OK;
    }
    DeviceGuard g(h->device);
    if (!g.ok) return HWPM_EDEVICE;
    const Csc A = to_csc(Ain);
    Work W;
    workspace_layout(n, A.nnz, (char*)workspace, &W);
    if (opt.check_csc) {
        st = timed_check(h, A, W, opt.timing == 1, &S);
        if (st != HWPM_OK) return st;
    }
    double total = 0.0;
    st = run_improve(h, A, W, mate_in, perm_out, &total, opt, &S);
    if (st != HWPM_OK) return st;
    if (total_out) *total_out = total;
    S.ms_total = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t_begin).count();
    if (stats) *stats = S;
    return HWPM_OK;
}

int hwpm_improve_static(hwpm_handle h, const hwpm_csc* A, const int32_t* mate_in, int32_t* perm_out,
                        double* total_out, const hwpm_options* opt, hwpm_stats* stats) {
    if (!h) return HWPM_EINVAL;
    const int st = check_csc_args(A);
    if (st != HWPM_OK) return st;
    if (workspace_layout(A->n, A->nnz, nullptr, nullptr) > kStaticScratchBytes) return HWPM_ETOOBIG;
    if (!h->scratch) return HWPM_EDEVICE;
    // the same solve as hwpm_improve, with the static array as its workspace
    // and no graph instantiation; nothing on this path allocates (the
    // library's kernels, stream-ordered copies and fills, the handle's pinned
    // buffer and events)
    hwpm_options o;
    hwpm_default_options(&o);
    if (opt) o = *opt;
    o.graph = 0;
    return hwpm_improve(h, A, mate_in, perm_out, total_out, &o, stats, h->scratch, kStaticScratchBytes);
}

int hwpm_match(hwpm_handle h, const hwpm_csc* Ain, int32_t* perm_out, double* total_out,
               const hwpm_options* opt_in, hwpm_stats* stats, void* workspace,
               size_t workspace_bytes) {
    const auto t_begin = std::chrono::steady_clock::now();
    if (!h) return HWPM_EINVAL;
    int st = check_csc_args(Ain);
    if (st != HWPM_OK) return st;
    hwpm_options opt;
    hwpm_default_options(&opt);
    if (opt_in) opt = *opt_in;
    st = check_options(opt);
    if (st != HWPM_OK) return st;
    const int32_t n = Ain->n;
    if (n > 0 && !perm_out) return HWPM_EINVAL;
    const size_t need = workspace_layout(n, Ain->nnz, nullptr, nullptr);
    if (n > 0 && !workspace) return HWPM_EINVAL;
    if (n > 0 && workspace_bytes < need) return HWPM_ENOMEM;
    hwpm_stats S;
    memset(&S, 0, sizeof(S));
    if (n == 0) {
        if (total_out) *total_out = 0.0;
        if (stats) *stats = S;
        return HWPM_OK;
    }
    DeviceGuard g(h->device);
    if (!g.ok) return HWPM_EDEVICE;
    const Csc A = to_csc(Ain);
    Work W;
    Mcm M;
    workspace_layout(n, A.nnz, (char*)workspace, &W, &M);
    const bool timing = opt.timing == 1;
    if (opt.check_csc) {
        st = timed_check(h, A, W, timing, &S);
        if (st != HWPM_OK) return st;
    }
    // a perfect matching takes n distinct entries
    if (A.nnz < (int64_t)n) return HWPM_ESINGULAR;
    st = run_initial_matching(h, A, W, M, opt.mcm_plain ? 0 : 1, timing, opt.graph != 0, &S);
    if (st != HWPM_OK) return st;
    double total = 0.0;
    st = run_improve(h, A, W, M.mc, perm_out, &total, opt, &S);
    if (st != HWPM_OK) return st;
    if (total_out) *total_out = total;
    S.ms_total = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t_begin).count();
    if (stats) *stats = S;
    return HWPM_OK;
}

int hwpm_batch_workspace_bytes(int32_t count, const hwpm_csc* mats, size_t* bytes) {
    if (!bytes || count < 0 || (count > 0 && !mats)) return HWPM_EINVAL;
    HostPlan HP;
    const int st = build_plan(count, mats, nullptr, nullptr, &HP, true);
    if (st != HWPM_OK) return st;
    *bytes = batch_bytes(HP, count);
    return HWPM_OK;
}

// match: find the perfect matchings first (hwpm_match_batch); phase1_only:
// stop there, with every block's matching in its perm_out (blocks without
// one: status HWPM_ESINGULAR, perm_out untouched).
static int run_batch(hwpm_handle h, int32_t count, const hwpm_csc* mats, const int32_t* const* mate_in,
                     int32_t* const* perm_out, double* totals, const hwpm_options* opt_in,
                     hwpm_item_stats* items, hwpm_stats* stats, void* workspace, size_t workspace_bytes,
                     bool match, bool phase1_only) {
    const auto t_begin = std::chrono::steady_clock::now();
    if (!h || count < 0 || (count > 0 && (!mats || !perm_out))) return HWPM_EINVAL;
    if (!match && count > 0 && !mate_in) return HWPM_EINVAL;
    hwpm_options opt;
    hwpm_default_options(&opt);
    if (opt_in) opt = *opt_in;
    int st = check_options(opt);
    if (st != HWPM_OK) return st;
    HostPlan HP;
    st = build_plan(count, mats, match ? nullptr : mate_in, perm_out, &HP);
    if (st != HWPM_OK) return st;
    // default launch configuration: the handle's tuning table, by the packed
    // batch's degree bin
    if (h->has_tune && opt.probe == 0 && opt.tile_width == 0) {
        const int b = hwpm_tune_bin(&h->tune, (int32_t)(HP.n_tot < INT32_MAX ? HP.n_tot : INT32_MAX - 1), HP.nnz_tot);
        if (b >= 0 && h->tune.probe[b] != 0) {
            opt.probe = h->tune.probe[b];
            opt.tile_width = h->tune.tile_width[b];
        }
    }
    hwpm_stats S;
    memset(&S, 0, sizeof(S));
    if (HP.n_tot == 0) {
        for (int32_t b = 0; b < count; ++b) {
            if (totals) totals[b] = 0.0;
            if (items) memset(&items[b], 0, sizeof(hwpm_item_stats));
        }
        if (stats) *stats = S;
        return HWPM_OK;
    }
    if (!workspace) return HWPM_EINVAL;
    if (workspace_bytes < batch_bytes(HP, count)) return HWPM_ENOMEM;
    DeviceGuard g(h->device);
    if (!g.ok) return HWPM_EDEVICE;
    BatchPlan P;
    const size_t head = batch_layout(HP, count, (char*)workspace, &P);
    char* rest = (char*)workspace + head;
    Work W;
    Mcm M;
    workspace_layout((int32_t)HP.n_tot, HP.nnz_tot, rest, &W, &M);
    W.mat_of_col = P.mat_of_col;
    W.item_flag = P.item_flag;
    W.item_cycles = P.item_cycles;
    st = upload_plan(h, HP, P);
    if (st != HWPM_OK) return st;
    HIP_TRY(launch_pack(P, !match, h->stream, h->cus));
    HIP_TRY(hipMemcpyAsync(h->host, P.item_err, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    Csc A;
    A.n = (int32_t)HP.n_tot;
    A.nnz = HP.nnz_tot;
    A.col_ptr = P.col_ptr;
    A.row_idx = P.row_idx;
    A.w = P.w;
    if (h->host[0] & 3) return HWPM_EBADCSC;
    if (opt.check_csc) {
        st = timed_check(h, A, W, opt.timing == 1, &S);
        if (st != HWPM_OK) return st;
    }
    if (h->host[0] & 4) return HWPM_EBADMATCH;
    const int32_t* start = P.mate;
    if (match) {
        st = run_initial_matching(h, A, W, M, opt.mcm_plain ? 0 : 1, opt.timing == 1, opt.graph != 0, &S);
        if (st != HWPM_OK && st != HWPM_ESINGULAR) return st;
        if (st == HWPM_ESINGULAR || phase1_only) {
            // Blocks without a perfect matching are masked out: the others'
            // matchings are unpacked and improved as a smaller packed batch
            // (no block joins another, so each still gets its result alone).
            const bool singular = st == HWPM_ESINGULAR;
            std::vector<int32_t> unm(count, 0);
            if (singular) {
                HIP_TRY(launch_item_unmatched(P, M.mc, h->stream, h->cus));
                HIP_TRY(hipMemcpyAsync(unm.data(), P.item_unmatched, (size_t)count * 4, hipMemcpyDeviceToHost,
                                       h->stream));
            }
            HIP_TRY(launch_unpack(P, M.mc, h->stream, h->cus, singular ? P.item_unmatched : nullptr));
            HIP_TRY(hipStreamSynchronize(h->stream));
            std::vector<int32_t> keep;
            for (int32_t b = 0; b < count; ++b) {
                if (items) {
                    memset(&items[b], 0, sizeof(hwpm_item_stats));
                    items[b].status = unm[b] > 0 ? HWPM_ESINGULAR : HWPM_OK;
                }
                if (totals) totals[b] = 0.0;
                if (unm[b] == 0) keep.push_back(b);
            }
            if (!phase1_only && !keep.empty()) {
                const size_t k = keep.size();
                std::vector<hwpm_csc> km(k);
                std::vector<const int32_t*> kin(k);
                std::vector<int32_t*> kout(k);
                std::vector<double> kt(k);
                std::vector<hwpm_item_stats> ki(k);
                for (size_t q = 0; q < k; ++q) {
                    km[q] = mats[keep[q]];
                    kin[q] = perm_out[keep[q]];
                    kout[q] = perm_out[keep[q]];
                }
                hwpm_options ok = opt;
                ok.check_csc = 0;  // validated above
                hwpm_stats Sk;
                st = run_batch(h, (int32_t)k, km.data(), kin.data(), kout.data(), kt.data(), &ok, ki.data(), &Sk,
                               workspace, workspace_bytes, false, false);
                if (st != HWPM_OK) return st;
                for (size_t q = 0; q < k; ++q) {
                    if (totals) totals[keep[q]] = kt[q];
                    if (items) items[keep[q]] = ki[q];
                }
                // the rounds' statistics are the smaller batch's; the initial
                // matching's stay this call's
                hwpm_stats P1 = S;
                S = Sk;
                S.greedy_rounds = P1.greedy_rounds;
                S.greedy_cardinality = P1.greedy_cardinality;
                S.mcm_cardinality = P1.mcm_cardinality;
                S.mcm_phases = P1.mcm_phases;
                S.mcm_levels = P1.mcm_levels;
                S.ms_check = P1.ms_check;
                S.ms_greedy = P1.ms_greedy;
                S.ms_mcm = P1.ms_mcm;
                S.graph_launches += P1.graph_launches;
            }
            S.ms_total = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t_begin).count();
            if (stats) *stats = S;
            return HWPM_OK;
        }
        start = M.mc;
    }
    double total = 0.0;
    st = run_improve(h, A, W, start, P.mate, &total, opt, &S, &P);
    if (st != HWPM_OK) return st;
    st = fill_item_stats(h, HP, P, opt, totals, items);
    if (st != HWPM_OK) return st;
    S.ms_total = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t_begin).count();
    if (stats) *stats = S;
    return HWPM_OK;
}

int hwpm_autotune(hwpm_handle h, const hwpm_csc* A, const int32_t* mate_in, int32_t* perm_out,
                  hwpm_options* opt, float* ms_out, void* workspace, size_t workspace_bytes) {
    static const int32_t kCand[HWPM_TUNE_CANDIDATES][2] = {
        {1, 4}, {1, 8}, {1, 16}, {1, 32}, {1, 64}, {3, 4}, {3, 8}, {3, 16}, {3, 32}, {4, 4}, {5, 4}, {5, 8}};
    if (!h || !opt) return HWPM_EINVAL;
    int st = check_options(*opt);
    if (st != HWPM_OK) return st;
    float best_ms[HWPM_TUNE_CANDIDATES];
    for (int c = 0; c < HWPM_TUNE_CANDIDATES; ++c) best_ms[c] = 3.0e38f;
    hwpm_options o = *opt;
    for (int rep = 0; rep < 2; ++rep) {
        for (int c = 0; c < HWPM_TUNE_CANDIDATES; ++c) {
            o.probe = kCand[c][0];
            o.tile_width = kCand[c][1];
            o.check_csc = (rep == 0 && c == 0) ? opt->check_csc : 0;  // validate once
            o.timing = 0;
            const auto t0 = std::chrono::steady_clock::now();
            st = hwpm_improve(h, A, mate_in, perm_out, nullptr, &o, nullptr, workspace, workspace_bytes);
            const float ms =
                std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (st != HWPM_OK) return st;
            if (ms < best_ms[c]) best_ms[c] = ms;
        }
    }
    int win = 0;
    for (int c = 1; c < HWPM_TUNE_CANDIDATES; ++c)
        if (best_ms[c] < best_ms[win]) win = c;
    if (ms_out)
        for (int c = 0; c < HWPM_TUNE_CANDIDATES; ++c) ms_out[c] = best_ms[c];
    opt->probe = kCand[win][0];
    opt->tile_width = kCand[win][1];
    return HWPM_OK;
}

void hwpm_default_tune_table(hwpm_tune_table* t) {
    if (!t) return;
    memset(t, 0, sizeof(*t));
    static const float kBounds[HWPM_TUNE_BINS] = {4.f, 8.f, 16.f, 32.f, 64.f, 3.0e38f};
    for (int b = 0; b < HWPM_TUNE_BINS; ++b) t->max_degree[b] = kBounds[b];
}

int hwpm_tune_bin(const hwpm_tune_table* t, int32_t n, int64_t nnz) {
    if (!t) return -1;
    if (n <= 0) return 0;
    const double d = (double)nnz / (double)n;
    for (int b = 0; b + 1 < HWPM_TUNE_BINS; ++b)
        if (d <= (double)t->max_degree[b]) return b;
    return HWPM_TUNE_BINS - 1;
}

int hwpm_set_tune_table(hwpm_handle h, const hwpm_tune_table* t) {
    if (!h) return HWPM_EINVAL;
    if (!t) {
        h->has_tune = false;
        return HWPM_OK;
    }
    for (int b = 0; b < HWPM_TUNE_BINS; ++b) {
        if (b > 0 && !(t->max_degree[b] > t->max_degree[b - 1])) return HWPM_EINVAL;
        hwpm_options o;
        hwpm_default_options(&o);
        o.probe = t->probe[b];
        o.tile_width = t->tile_width[b];
        if (t->probe[b] != 0 && check_options(o) != HWPM_OK) return HWPM_EINVAL;
    }
    h->tune = *t;
    h->has_tune = true;
    return HWPM_OK;
}

int hwpm_autotune_table(hwpm_handle h, const hwpm_csc* A, const int32_t* mate_in, int32_t* perm_out,
                        hwpm_tune_table* t, void* workspace, size_t workspace_bytes) {
    if (!h || !A || !t) return HWPM_EINVAL;
    hwpm_options o;
    hwpm_default_options(&o);
    float ms[HWPM_TUNE_CANDIDATES];
    const int st = hwpm_autotune(h, A, mate_in, perm_out, &o, ms, workspace, workspace_bytes);
    if (st != HWPM_OK) return st;
    const int b = hwpm_tune_bin(t, A->n, A->nnz);
    float best = ms[0];
    for (int c = 1; c < HWPM_TUNE_CANDIDATES; ++c) best = ms[c] < best ? ms[c] : best;
    t->probe[b] = o.probe;
    t->tile_width[b] = o.tile_width;
    t->ms_per_mentry[b] = best / (float)(((double)A->n + (double)A->nnz) * 1e-6 + 1e-12);
    return HWPM_OK;
}

int hwpm_improve_batch(hwpm_handle h, int32_t count, const hwpm_csc* mats, const int32_t* const* mate_in,
                       int32_t* const* perm_out, double* totals, const hwpm_options* opt,
                       hwpm_item_stats* items, hwpm_stats* stats, void* workspace,
                       size_t workspace_bytes) {
    return run_batch(h, count, mats, mate_in, perm_out, totals, opt, items, stats, workspace,
                     workspace_bytes, false, false);
}

int hwpm_match_batch(hwpm_handle h, int32_t count, const hwpm_csc* mats, int32_t* const* perm_out,
                     double* totals, const hwpm_options* opt, hwpm_item_stats* items,
                     hwpm_stats* stats, void* workspace, size_t workspace_bytes) {
    return run_batch(h, count, mats, nullptr, perm_out, totals, opt, items, stats, workspace,
                     workspace_bytes, true, false);
}


}  // extern "C"

namespace hwpm {

int match_batch_initial(hwpm_handle h, int32_t count, const hwpm_csc* mats, int32_t* const* perm_out,
                        const hwpm_options* opt, hwpm_item_stats* items, void* workspace,
                        size_t workspace_bytes) {
    return run_batch(h, count, mats, nullptr, perm_out, nullptr, opt, items, nullptr, workspace,
                     workspace_bytes, true, true);
}

}  // namespace hwpm
