/*
 * hwpm.h -- heavy-weight perfect matching on one MI355X (gfx950).
 *
 * C ABI of libhwpm.so.  The library implements the weight-improvement phase
 * of the heavy-weight perfect matching (HWPM) method of Azad, Buluc, Li,
 * Wang and Langguth, "A distributed-memory algorithm for computing a
 * heavy-weight perfect matching on bipartite graphs" (arXiv 1801.09809):
 * bulk-synchronous rounds that find weight-increasing alternating 4-cycles,
 * keep one per matched edge and flip a vertex-disjoint set of them
 * (Section 5.3, Algorithms 2-6), repeated until no positive-gain 4-cycle is
 * left.  Every step runs in hand-written HIP kernels; the host code only
 * launches them and reads back a few counters per round.
 *
 * Problem (Section 3): an n x n sparse matrix A is the bipartite graph with
 * row vertices R, column vertices C and one edge {i,j} of weight w(i,j) per
 * nonzero a_ij.  A perfect matching pairs every column j with a distinct row
 * m_j.  The caller supplies the weights; for static pivoting the paper uses
 * w(i,j) = log|a_ij| (its "Option B": maximising the sum of logs maximises
 * the product of the matched magnitudes) or |a_ij| ("Option A").
 *
 * Matrix layout (hwpm_csc): compressed sparse column, all DEVICE pointers.
 *   col_ptr  int64[n+1]   col_ptr[0] = 0, nondecreasing, col_ptr[n] = nnz
 *   row_idx  int32[nnz]   rows of column j at [col_ptr[j], col_ptr[j+1]),
 *                         each in [0, n), strictly increasing in a column
 *   weight   float64[nnz] finite
 * Matchings are int32[n] arrays with perm[j] = the row matched to column j.
 *
 * Ownership: every buffer is owned by the caller, including the device
 * workspace (hwpm_workspace_bytes tells its size).  The library allocates
 * only a small pinned host buffer and a few HIP events, in hwpm_create.
 *
 * Streams: a handle is bound to one device and one HIP stream; all work is
 * queued on that stream and every call returns when its results are ready.
 * A handle is not thread-safe; calls on different handles may run
 * concurrently if they use different workspaces.
 *
 * Errors: functions return HWPM_OK (0) or a negative status.  On any error
 * the output arguments are left untouched.
 *
 * Results are deterministic: the same input gives bit-identical perm and
 * total weight for every launch configuration, and equal those of the
 * sequential round-by-round definition of the method (the CPU oracle in
 * this repository).
 */
#ifndef HWPM_H
#define HWPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define HWPM_OK          0
#define HWPM_EINVAL     -1  /* bad argument: null pointer, negative size, bad option */
#define HWPM_ESINGULAR  -2  /* the matrix has no perfect matching (Section 3) */
#define HWPM_EBADCSC    -3  /* malformed CSC: col_ptr, row range, row order, non-finite weight */
#define HWPM_EBADMATCH  -4  /* mate_in is not a perfect matching inside the pattern */
#define HWPM_ENOMEM     -5  /* workspace smaller than hwpm_workspace_bytes() */
#define HWPM_ETOOBIG    -6  /* n or nnz beyond the library limits (n < 2^31 - 1, nnz < 2^40) */
#define HWPM_EDEVICE    -7  /* a HIP runtime call failed (no device, launch failure, ...) */
#define HWPM_EINTERNAL  -8  /* an internal consistency check failed (a bug) */
#define HWPM_PENDING     1  /* hwpm_poll: the request has not finished yet (not an error) */

#define HWPM_MAX_ROUND_STATS 512

typedef struct hwpm_handle_s* hwpm_handle;

typedef struct {
    int32_t n;               /* number of rows = number of columns, >= 0 */
    int64_t nnz;             /* number of stored entries, >= 0 */
    const int64_t* col_ptr;  /* device, n+1 */
    const int32_t* row_idx;  /* device, nnz */
    const double* weight;    /* device, nnz */
} hwpm_csc;

typedef struct {
    /* Round cap (the paper's maxiters, Section 4 and Algorithm 2).
     * 0 = repeat until a round applies no cycle (no positive-gain 4-cycle
     * left).  >= 0. */
    int32_t max_rounds;
    /* 1 = validate the CSC on the device before solving (one pass over the
     * matrix); 0 = the caller guarantees a well-formed CSC (e.g. it already
     * passed hwpm_check_csc).  Kernels index with the given arrays, so a
     * malformed CSC with check_csc = 0 is undefined behaviour. */
    int32_t check_csc;
    /* 0 = no timing; 1 = time every stage with HIP events into hwpm_stats
     * (ms_*); 2 = time the search stage (Steps A-C) only: ms_search,
     * ms_search_first and round_ms_search, two events per round (an event
     * between two kernels also holds the second one back, so fewer events
     * perturb the solve less).  Other values: HWPM_EINVAL. */
    int32_t timing;
    /* Lanes per root column in the cycle-search kernel: 0 = default (4; 8 with
     * probes 3 and 5 when the matrix has more than 20 entries per column on
     * average), else one of 4, 8, 16, 32, 64 (64: probes 1 and 2 only).
     * Results do not depend on it. */
    int32_t tile_width;
    /* How the closing edge {m_j, m_i} is probed (results do not depend on it):
     * 0 = default (3); 1 = binary search of row m_j in column m_i; 2 = build
     * the pattern transpose once per call and test m_i against the row list
     * of m_j (the marking trick of Section 4), with per-entry mate columns
     * kept up to date across flips, one entry per lane; 3 = the same, each
     * root's row list loaded by a tile of lanes and summarised in a two-word
     * filter, and only the probes that pass it compared with the list (the
     * default); 4 = the same with every probe compared against the whole
     * row list through cross-lane exchanges;
     * 5 = probe 3 over row lists built without CSC positions (a lighter
     * transpose; a hit or a mate refresh binary-searches its entry instead:
     * the better choice when hits are rare).  Probes 2-5 read only the
     * entries of column j after its matched one (the rows i > m_j) and keep
     * 32-bit CSC positions: a matrix with nnz >= 2^31 uses probe 1. */
    int32_t probe;
    /* Initial matching of hwpm_match (Section 5.2): 0 = heavy-edge tie-break
     * in the greedy and BFS steps (the paper's heuristic, default);
     * 1 = index order only (the paper's "without heuristic" ablation). */
    int32_t mcm_plain;
    /* 0 = incremental rounds (default with probe 3): after the first round
     * only the columns whose cycles can have changed are searched again -- a
     * flipped column, or a column holding a row whose mate changed; every
     * other column keeps its Step-C winner, which is provably unchanged, so
     * the results are identical.  1 = every round searches every column (the
     * paper's rounds as written; the benchmark's search-throughput setting). */
    int32_t full_search;
    /* 1 (default) = batches of launches that repeat inside one call (8
     * rounds that start at the same ring slot, 8 proposal rounds, 8 BFS
     * levels) are captured once per call into a HIP graph and replayed as
     * one launch each; 0 = every kernel is launched directly.  Results do
     * not depend on it.  Timed solves (timing != 0) launch directly. */
    int32_t graph;
} hwpm_options;

typedef struct {
    int32_t rounds;          /* search passes run (the last one finds no cycle unless capped) */
    int32_t hit_round_cap;   /* 1 if max_rounds stopped the loop */
    int64_t cycles_applied;  /* total 4-cycles flipped */
    int32_t long_columns;    /* columns handled by the split (long-column) search */
    int32_t greedy_rounds;   /* hwpm_match: proposal rounds of the greedy step */
    int32_t greedy_cardinality; /* hwpm_match: size of the greedy maximal matching */
    int32_t mcm_cardinality; /* hwpm_match: size of the maximum matching */
    int32_t mcm_phases;      /* hwpm_match: BFS phases run (each starts with an unmatched column) */
    int32_t mcm_levels;      /* hwpm_match: BFS levels over all phases */
    double init_weight;      /* total weight of the starting perfect matching */
    double final_weight;     /* = *total_out */
    /* milliseconds, filled when options.timing = 1 (else 0; ms_total always;
     * the three search-stage fields also when options.timing = 2) */
    float ms_check;          /* CSC validation */
    float ms_greedy;         /* hwpm_match: greedy maximal matching */
    float ms_mcm;            /* hwpm_match: BFS phases */
    float ms_setup;          /* matching validation, mate/weight arrays, long-column table */
    float ms_transpose;      /* pattern transpose + per-entry mate columns (probe >= 2) */
    float ms_search;         /* Steps A-C (cycle search + per-root argmax), all rounds */
    float ms_resolve;        /* Step D conflict resolution (both passes), all rounds */
    float ms_apply;          /* flips (and mate-column updates), all rounds */
    float ms_final;          /* total weight + output copy */
    float ms_total;          /* whole call, host wall clock */
    float ms_search_first;   /* Steps A-C of the first round alone */
    int32_t graph_launches;  /* batches of launches replayed from a captured graph (options.graph) */
    int32_t probe_used;      /* the probe and tile width the rounds ran with (defaults, options */
    int32_t tile_used;       /* or the handle's tuning table resolved) */
    /* per round (first HWPM_MAX_ROUND_STATS rounds) */
    int32_t round_candidates[HWPM_MAX_ROUND_STATS]; /* roots that kept a cycle (Step C) */
    int32_t round_applied[HWPM_MAX_ROUND_STATS];    /* cycles flipped (Step D) */
    float round_ms_search[HWPM_MAX_ROUND_STATS];    /* Steps A-C time, when timing = 1 or 2 */
    int32_t round_roots[HWPM_MAX_ROUND_STATS];      /* columns searched */
} hwpm_stats;

/* Fill *opt with the defaults: max_rounds 0, check_csc 1, timing 0,
 * tile_width 0, probe 0, mcm_plain 0, full_search 0, graph 1. */
void hwpm_default_options(hwpm_options* opt);

/* Text for a status code (static storage). */
const char* hwpm_strerror(int status);

/* Create a handle bound to HIP device `device` and HIP stream `stream`
 * (a hipStream_t; NULL = the device's null stream).  Allocates a small
 * pinned host buffer and HIP events.  Returns HWPM_EDEVICE if the device
 * does not exist or HIP fails, HWPM_EINVAL if out is NULL. */
int hwpm_create(hwpm_handle* out, int device, void* stream);

/* Release a handle (waits for its stream).  NULL is accepted. */
int hwpm_destroy(hwpm_handle h);

/* Bytes of device workspace hwpm_improve / hwpm_check_csc need for an
 * n x n matrix with nnz entries (a pure host computation).  The workspace
 * must be 256-byte aligned (any hipMalloc / PyTorch allocation is). */
int hwpm_workspace_bytes(int32_t n, int64_t nnz, size_t* bytes);

/* Validate a CSC on the device: col_ptr[0] = 0, nondecreasing,
 * col_ptr[n] = nnz, rows in [0, n) and strictly increasing within each
 * column, weights finite.  Returns HWPM_OK or HWPM_EBADCSC. */
int hwpm_check_csc(hwpm_handle h, const hwpm_csc* A, void* workspace, size_t workspace_bytes);

/* Improve a perfect matching with weight-increasing alternating 4-cycles
 * (Section 5.3).  One round:
 *   Steps A+B  for every column j and every row i > m_j of column j, the
 *              cycle (i, j, m_j, m_i) exists if the edge {m_j, m_i} does;
 *              its gain (Section 3) is evaluated in binary64 as
 *              (w(i,j) + w(m_j,m_i)) - (w(i,m_i) + w(m_j,j)); g > 0 makes it
 *              a candidate;
 *   Step C     each column j keeps its candidate of largest gain (equal
 *              gains: smallest row i);
 *   Step D     each column c = m_i accepts, unless c kept a cycle of its own,
 *              the kept cycle of largest gain that uses its matched edge
 *              (equal gains: smallest root column j); accepted cycles are
 *              vertex-disjoint and all are flipped at once.
 * Rounds repeat until one flips nothing, or max_rounds rounds ran.
 *
 *   mate_in    device int32[n]: a perfect matching contained in the pattern
 *              (mate_in[j] = row of column j).  May alias perm_out.
 *   perm_out   device int32[n]: the improved matching.
 *   total_out  host, nullable: sum of the matched weights, added as a perfect
 *              binary tree over columns 0..n-1 padded with +0.0 to a power
 *              of two (pairs (2t, 2t+1) at each level).
 *   opt        nullable (defaults).
 *   stats      host, nullable.
 *   workspace  device, >= hwpm_workspace_bytes(n, nnz) bytes; its contents
 *              are scratch between calls.
 * Errors: HWPM_EINVAL, HWPM_ENOMEM, HWPM_ETOOBIG, HWPM_EBADCSC (when
 * opt->check_csc), HWPM_EBADMATCH (a mate out of range, a row claimed twice,
 * a mate row that is not an entry of its column, or nnz < n; checked before
 * the first round, perm_out untouched), HWPM_EDEVICE, HWPM_EINTERNAL.
 * n = 0 returns HWPM_OK with total 0.0. */
int hwpm_improve(hwpm_handle h, const hwpm_csc* A, const int32_t* mate_in, int32_t* perm_out,
                 double* total_out, const hwpm_options* opt, hwpm_stats* stats,
                 void* workspace, size_t workspace_bytes);

/* ---- allocation-free form ---------------------------------------------
 * hwpm_improve for callers that cannot allocate device memory and cannot
 * bring a workspace of their own (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Its workspace is a fixed
 * device array of HWPM_STATIC_SCRATCH_BYTES that the library holds on every
 * GPU it runs on until the process ends (its address is taken in
 * hwpm_create).  The call allocates nothing: no hipMalloc, hipFree or
 * allocating library routine.  Inputs and outputs are the caller's, as in
 * hwpm_improve.
 *
 * Every call on one GPU uses that GPU's one array, whose contents are
 * scratch between calls: calls that overlap on one GPU (from several
 * handles, threads or streams) race and must be serialised by the caller.
 * Errors as hwpm_improve, plus HWPM_ETOOBIG when
 * hwpm_workspace_bytes(n, nnz) exceeds HWPM_STATIC_SCRATCH_BYTES (outputs
 * untouched), and HWPM_EDEVICE if the array's device address was not
 * available when the handle was created. */
#define HWPM_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
int hwpm_improve_static(hwpm_handle h, const hwpm_csc* A, const int32_t* mate_in, int32_t* perm_out,
                        double* total_out, const hwpm_options* opt, hwpm_stats* stats);

/* The whole HWPM pipeline (Section 5.1): a greedy maximal matching, then a
 * maximum-cardinality matching by multi-source BFS phases (both with the
 * heavy-edge tie-break of Section 5.2 unless opt->mcm_plain), then the rounds
 * of hwpm_improve.
 *   Greedy    rounds of proposals: every unmatched column proposes to its
 *             unmatched row of largest weight (ties: smallest row); a row with
 *             proposals accepts the heaviest (ties: smallest column); until no
 *             unmatched column has an unmatched neighbour.
 *   BFS phase every unmatched column roots a tree; each level, every row not
 *             yet visited that is adjacent to a frontier column joins the tree
 *             of its heaviest such column (ties: smallest column); a tree that
 *             reaches unmatched rows keeps the smallest one and stops; the
 *             mates of the level's matched rows of growing trees form the next
 *             frontier; at the end every recorded path is augmented.  Phases
 *             repeat until one augments nothing.
 *   perm_out  device int32[n]; total_out as in hwpm_improve.
 * Returns HWPM_ESINGULAR when the maximum matching is not perfect (outputs
 * untouched), else as hwpm_improve. */
int hwpm_match(hwpm_handle h, const hwpm_csc* A, int32_t* perm_out, double* total_out,
               const hwpm_options* opt, hwpm_stats* stats, void* workspace, size_t workspace_bytes);

/* ---- tuning ---------------------------------------------------------------
 * Launch-configuration tuner.  Runs hwpm_improve from mate_in once per
 * candidate (probe, tile_width) -- probe 1 with tiles 4, 8, 16, 32, 64,
 * probe 3 with tiles 4, 8, 16, 32, probe 4, and probe 5 with tiles 4 and
 * 8 -- twice over, timing each
 * whole call on the host clock, and writes the fastest candidate's probe and
 * tile_width into *opt (its other fields are used as given: max_rounds,
 * full_search, ...).  Outputs never depend on these two fields, so a tuned
 * solve returns exactly what an untuned one does; perm_out holds that result
 * (device int32[n]).  ms_out (host, nullable) receives the best time of each
 * candidate, in the order above.  Errors as hwpm_improve. */
#define HWPM_TUNE_CANDIDATES 12
int hwpm_autotune(hwpm_handle h, const hwpm_csc* A, const int32_t* mate_in, int32_t* perm_out,
                  hwpm_options* opt, float* ms_out, void* workspace, size_t workspace_bytes);

/* ---- tuning table by degree bin -------------------------------------------
 * Launch configurations chosen per bin of average entries per column,
 * nnz / n: bin b holds the matrices (or packed batches) with
 * max_degree[b-1] < nnz / n <= max_degree[b]; the last bin has no upper
 * bound.  An entry with probe 0 is untuned (the library's defaults).
 * Batches (hwpm_improve_batch, hwpm_match_batch) whose options leave probe
 * and tile_width at 0 take the entry of the packed batch's bin from the
 * handle's table (hwpm_set_tune_table); the server tunes a table of its own
 * online (hwpm_server_options.tune).  Outputs never depend on the table. */
#define HWPM_TUNE_BINS 6
typedef struct {
    float max_degree[HWPM_TUNE_BINS];     /* bin bounds, increasing */
    int32_t probe[HWPM_TUNE_BINS];        /* 0 = untuned */
    int32_t tile_width[HWPM_TUNE_BINS];
    float ms_per_mentry[HWPM_TUNE_BINS];  /* tuned solve time per million columns + entries */
} hwpm_tune_table;

/* Bins of at most 4, 8, 16, 32 and 64 entries per column and one above;
 * every entry untuned. */
void hwpm_default_tune_table(hwpm_tune_table* t);

/* Bin of a matrix (or batch) with n columns and nnz entries (0 for n = 0);
 * -1 for a NULL table. */
int hwpm_tune_bin(const hwpm_tune_table* t, int32_t n, int64_t nnz);

/* Copy *t into the handle (NULL: no table, library defaults). */
int hwpm_set_tune_table(hwpm_handle h, const hwpm_tune_table* t);

/* Tune the bin of one representative matrix: hwpm_autotune on it (from
 * mate_in, with the handle's other defaults) and its winner written into
 * the entry of the matrix's bin in *t.  perm_out as in hwpm_autotune.
 * Errors as hwpm_improve. */
int hwpm_autotune_table(hwpm_handle h, const hwpm_csc* A, const int32_t* mate_in, int32_t* perm_out,
                        hwpm_tune_table* t, void* workspace, size_t workspace_bytes);

/* ---- batches -------------------------------------------------------------
 * Many matrices solved in one call.  The batch is packed into one
 * block-diagonal matrix in the workspace and solved by the same kernels: no
 * entry joins two blocks, so every cycle, Step-C choice and Step-D conflict
 * stays inside its block and every matrix gets exactly the result it gets
 * alone (a block whose rounds have ended has no candidates any more).  The
 * number of kernel launches does not grow with the number of matrices. */
typedef struct {
    int32_t status;          /* HWPM_OK, or HWPM_ESINGULAR (hwpm_match_batch) */
    int32_t rounds;          /* rounds this matrix would run alone */
    int32_t hit_round_cap;
    int32_t reserved;
    int64_t cycles_applied;
    double init_weight;      /* total weight of the starting matching */
    double final_weight;     /* = totals[b] */
} hwpm_item_stats;

/* Workspace bytes for a batch: only n and nnz of each descriptor are used
 * (its pointers are neither read nor checked).  HWPM_EINVAL for count < 0 or
 * a negative size, HWPM_ETOOBIG beyond the limits. */
int hwpm_batch_workspace_bytes(int32_t count, const hwpm_csc* mats, size_t* bytes);

/* hwpm_improve on every matrix of a batch.
 *   mats      host array of count CSC descriptors (their arrays on the device)
 *   mate_in   host array of count device pointers (starting matchings)
 *   perm_out  host array of count device pointers (results; may alias mate_in)
 *   totals    host, nullable: count totals, each summed in its own tree
 *   items     host, nullable: count per-matrix statistics
 *   stats     host, nullable: statistics of the packed solve
 * Errors as hwpm_improve, for the batch as a whole (a malformed matrix or
 * matching fails the call; outputs untouched). */
int hwpm_improve_batch(hwpm_handle h, int32_t count, const hwpm_csc* mats,
                       const int32_t* const* mate_in, int32_t* const* perm_out, double* totals,
                       const hwpm_options* opt, hwpm_item_stats* items, hwpm_stats* stats,
                       void* workspace, size_t workspace_bytes);

/* hwpm_match on every matrix of a batch.  A structurally singular matrix does
 * not fail the call: its item status is HWPM_ESINGULAR and its perm_out is
 * left untouched. */
int hwpm_match_batch(hwpm_handle h, int32_t count, const hwpm_csc* mats, int32_t* const* perm_out,
                     double* totals, const hwpm_options* opt, hwpm_item_stats* items,
                     hwpm_stats* stats, void* workspace, size_t workspace_bytes);

/* ---- serving --------------------------------------------------------------
 * A request loop for callers that produce a stream of independent matrices
 * (e.g. a sparse direct solver that pivots every matrix it factorises), with
 * continuous batching at round granularity.  Each worker owns a handle on its
 * own HIP stream and the requests it holds in flight; it works in steps.  In
 * each step it admits, in arrival order, as many queued requests as fit the
 * server's device arena (each request's inputs and matching stay in a region
 * of the arena while it is in flight; the batch workspace is sized to all of
 * the worker's requests -- admission by HBM footprint), finds their perfect
 * matchings, and then runs up to rounds_per_step weight-improvement rounds
 * (Section 5.3) on every request it holds, old and new, as one block-diagonal
 * batch.  Requests whose rounds have ended leave with their results; the
 * others stay resident and continue in the next step, together with the
 * requests that arrived meanwhile.  The workers' steps overlap on the
 * device.  Every result (permutation, total, round count, cycles) equals
 * that of hwpm_match on the matrix alone: a round depends on the matching
 * alone, whichever call runs it.
 *
 * Ownership: with copy_inputs = 1 (default) hwpm_submit copies the host
 * arrays and the caller may reuse them at once; with copy_inputs = 0 they are
 * kept by reference and must stay valid and unchanged until hwpm_poll has
 * returned the result (or until hwpm_server_destroy has returned) -- the
 * cheaper form when the arrays already sit in page-locked memory.  The
 * server allocates its arena (arena_bytes of device memory) and one stream
 * and handle per worker; hwpm_server_destroy finishes the queued requests and
 * frees everything.
 *
 * Threads: hwpm_submit, hwpm_poll and hwpm_server_get_stats are
 * thread-safe.  A ticket belongs to the first hwpm_poll that waits for it or
 * takes its result: any other call with that ticket returns HWPM_EINVAL.
 * Once hwpm_server_destroy has begun, hwpm_poll returns HWPM_EINVAL; polls
 * already waiting receive their results and return before destroy frees the
 * server.  No call may start after hwpm_server_destroy has returned, and
 * hwpm_submit and hwpm_server_get_stats may not overlap it. */
typedef struct hwpm_server_s* hwpm_server;

typedef struct {
    int32_t device;          /* HIP device ordinal */
    int32_t workers;         /* worker streams, 1..16 */
    int32_t max_batch;       /* most requests one batch admits, >= 1 */
    /* 1 (default) = tune (probe, tile_width) per degree bin online: the
     * first batches of each bin are solved under each candidate
     * configuration in turn (results never depend on it), and the fastest
     * per column and entry is kept for the bin's later batches; 0 = use
     * solve.probe / solve.tile_width as given. */
    int32_t tune;
    size_t arena_bytes;      /* device memory the server owns, >= 1 MiB */
    hwpm_options solve;      /* solve options of every request (solve.max_rounds caps each
                              * request's own rounds, over all its steps) */
    int32_t rounds_per_step; /* rounds a worker runs between admissions, >= 0 (default 8;
                              * 0 = a request's rounds all run in its first step) */
    int32_t copy_inputs;     /* 1 (default): hwpm_submit copies the host arrays; 0: by reference */
} hwpm_server_options;

typedef struct {
    hwpm_item_stats item;    /* the request's statistics (item.status = its status) */
    double queue_ms;         /* host clock: submit -> admitted into a batch */
    double latency_ms;       /* host clock: submit -> result ready */
    int32_t batch_size;      /* requests in the step that admitted it */
    int32_t worker;          /* worker that solved it */
    int32_t steps;           /* round steps it took part in */
    int32_t reserved;
} hwpm_request_info;

typedef struct {
    int64_t submitted;       /* requests accepted by hwpm_submit */
    int64_t completed;       /* requests with a result (any status) */
    int64_t batches;         /* steps run (each: admissions, matchings, one packed round batch) */
    int64_t max_batch_seen;  /* most requests in one step */
    int64_t max_running;     /* most steps in flight at once */
    int64_t pending;         /* requests waiting now */
    int64_t running;         /* steps in flight now */
    int64_t arena_in_use;    /* arena bytes held now */
    int64_t arena_peak;      /* most arena bytes held at once */
    int64_t joined;          /* requests admitted into a step next to requests already in flight */
} hwpm_server_stats;

/* Defaults: device 0, 2 workers, max_batch 64, 8 GiB arena, 8 rounds per
 * step, inputs copied at submission, solve options from hwpm_default_options
 * (check_csc = 1: every request is validated on the device when admitted; a
 * step whose fresh requests include a malformed one matches them one by one,
 * so only that one reports HWPM_EBADCSC). */
void hwpm_server_default_options(hwpm_server_options* opt);

/* Start a server (opt may be NULL for the defaults).  Errors: HWPM_EINVAL
 * (bad option), HWPM_EDEVICE, HWPM_ENOMEM (arena allocation failed). */
int hwpm_server_create(hwpm_server* out, const hwpm_server_options* opt);

/* Finish every queued request, stop the workers and free the server.  Results
 * not yet polled are discarded. */
int hwpm_server_destroy(hwpm_server s);

/* Queue one matrix; A holds HOST pointers, copied or kept by reference as
 * copy_inputs says (see ownership above).  *ticket identifies the request in hwpm_poll.  Errors:
 * HWPM_EINVAL (null pointer, negative size), HWPM_ETOOBIG, HWPM_EBADCSC
 * (col_ptr[0] != 0 or col_ptr[n] != nnz); a rejected matrix is not queued.
 * Every other check of hwpm_check_csc runs on the device and its failure is
 * the request's status in hwpm_poll. */
int hwpm_submit(hwpm_server s, const hwpm_csc* A, uint64_t* ticket);

/* Result of a request.  wait = 0 returns HWPM_PENDING at once if it has not
 * finished; wait = 1 blocks until it has (and claims the ticket: a second
 * caller of the same ticket gets HWPM_EINVAL).  On completion returns the
 * request's status (HWPM_OK, HWPM_ESINGULAR, HWPM_EBADCSC, HWPM_ETOOBIG when
 * it cannot fit the arena even alone, or the batch's error), writes perm_host (host
 * int32[n], nullable) and *total (nullable) when HWPM_OK, fills *info
 * (nullable) and forgets the ticket.  An unknown ticket gives HWPM_EINVAL. */
int hwpm_poll(hwpm_server s, uint64_t ticket, int32_t wait, int32_t* perm_host, double* total,
              hwpm_request_info* info);

int hwpm_server_get_stats(hwpm_server s, hwpm_server_stats* st);

/* The server's online tuning table (untuned bins have probe 0). */
int hwpm_server_get_tune_table(hwpm_server s, hwpm_tune_table* t);

#ifdef __cplusplus
}
#endif

#endif /* HWPM_H */
