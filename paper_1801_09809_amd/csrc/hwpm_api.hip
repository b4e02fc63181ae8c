// C ABI of libhwpm.so (declared in include/hwpm.h): argument checks, the
// workspace carve-up, and the host round loop that launches the kernels of
// hwpm_kernels.hip and reads back two counters per round.
#include <chrono>
#include <new>
#include <string.h>

#include "hwpm.h"
#include "hwpm_internal.h"

using namespace hwpm;

struct hwpm_handle_s {
    int device;
    hipStream_t stream;
    int cus;
    int32_t* host;        // pinned host buffer for counter / result readback
    hipEvent_t ev[8];
};

namespace {

constexpr int kDefaultTile = 16;
constexpr int32_t kLongThreshold = 256;   // longer columns use the split search
constexpr int64_t kMaxNnz = (int64_t)1 << 40;

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

}  // namespace

extern "C" {

void hwpm_default_options(hwpm_options* opt) {
    if (!opt) return;
    opt->max_rounds = 0;
    opt->check_csc = 1;
    opt->timing = 0;
    opt->tile_width = 0;
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
    if (hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        h->cus <= 0)
        h->cus = 256;
    int ne = 0;
    bool ok = hipHostMalloc((void**)&h->host, 4096, hipHostMallocDefault) == hipSuccess;
    for (; ok && ne < 8; ++ne) ok = hipEventCreate(&h->ev[ne]) == hipSuccess;
    if (!ok) {
        for (int e = 0; e < ne; ++e) (void)hipEventDestroy(h->ev[e]);
        if (h->host) (void)hipHostFree(h->host);
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
    for (int e = 0; e < 8; ++e) (void)hipEventDestroy(h->ev[e]);
    (void)hipHostFree(h->host);
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
    if (opt.max_rounds < 0) return HWPM_EINVAL;
    int tile = opt.tile_width ? opt.tile_width : kDefaultTile;
    if (tile != 4 && tile != 8 && tile != 16 && tile != 32 && tile != 64) return HWPM_EINVAL;
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
    hipStream_t s = h->stream;
    const bool timing = opt.timing != 0;
    hipEvent_t* ev = h->ev;

    // 1. optional CSC validation
    if (opt.check_csc) {
        if (timing) HIP_TRY(hipEventRecord(ev[0], s));
        st = run_check(h, A, W);
        if (st != HWPM_OK) return st;
        if (timing) {
            HIP_TRY(hipEventRecord(ev[1], s));
            HIP_TRY(hipEventSynchronize(ev[1]));
            S.ms_check = elapsed(ev[0], ev[1]);
        }
    }

    // 2. set-up: mates, matched weights, matching validation, long columns
    if (timing) HIP_TRY(hipEventRecord(ev[0], s));
    HIP_TRY(hipMemsetAsync(W.counters, 0, kCounterWords * sizeof(int32_t), s));
    HIP_TRY(hipMemsetAsync(W.mr, 0xff, (size_t)n * sizeof(int32_t), s));
    HIP_TRY(launch_init_match(A, W, mate_in, kLongThreshold, s));
    HIP_TRY(launch_long_chunks(W, A, s));
    HIP_TRY(launch_tree_sum(W.wm, n, W, &W.result[1], s));
    HIP_TRY(hipMemcpyAsync(h->host, W.counters, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h->host + 8, &W.result[1], sizeof(double), hipMemcpyDeviceToHost, s));
    if (timing) HIP_TRY(hipEventRecord(ev[1], s));
    HIP_TRY(hipStreamSynchronize(s));
    if (timing) S.ms_setup = elapsed(ev[0], ev[1]);
    if (h->host[kErrMatch]) return HWPM_EBADMATCH;
    const int32_t n_long = h->host[kNumLong];
    S.long_columns = n_long;
    memcpy(&S.init_weight, h->host + 8, sizeof(double));

    // 3. rounds
    int32_t round = 0;
    for (;;) {
        if (opt.max_rounds > 0 && round >= opt.max_rounds) {
            S.hit_round_cap = 1;
            break;
        }
        const int slot = round % kSlots;
        if (timing) HIP_TRY(hipEventRecord(ev[2], s));
        HIP_TRY(launch_search(A, W, tile, kLongThreshold, slot, n_long > 0, s, h->cus));
        if (timing) HIP_TRY(hipEventRecord(ev[3], s));
        HIP_TRY(launch_resolve(W, slot, s, h->cus));
        if (timing) HIP_TRY(hipEventRecord(ev[4], s));
        HIP_TRY(launch_apply(A, W, slot, s, h->cus));
        if (timing) HIP_TRY(hipEventRecord(ev[5], s));
        HIP_TRY(hipMemcpyAsync(h->host, W.counters + kRoundBase + 2 * slot, 2 * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const int32_t n_cand = h->host[0], n_applied = h->host[1];
        if (round < HWPM_MAX_ROUND_STATS) {
            S.round_candidates[round] = n_cand;
            S.round_applied[round] = n_applied;
        }
        if (timing) {
            const float ms = elapsed(ev[2], ev[3]);
            S.ms_search += ms;
            if (round == 0) S.ms_search_first = ms;
            if (round < HWPM_MAX_ROUND_STATS) S.round_ms_search[round] = ms;
            S.ms_resolve += elapsed(ev[3], ev[4]);
            S.ms_apply += elapsed(ev[4], ev[5]);
        }
        S.cycles_applied += n_applied;
        ++round;
        // A round with candidates always flips at least one cycle (the
        // candidate whose other column has the largest matched row).
        if (n_cand > 0 && n_applied == 0) return HWPM_EINTERNAL;
        if (n_applied == 0) break;
    }
    S.rounds = round;

    // 4. outputs
    if (timing) HIP_TRY(hipEventRecord(ev[6], s));
    HIP_TRY(launch_tree_sum(W.wm, n, W, &W.result[0], s));
    HIP_TRY(hipMemcpyAsync(perm_out, W.mc, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(h->host + 8, &W.result[0], sizeof(double), hipMemcpyDeviceToHost, s));
    if (timing) HIP_TRY(hipEventRecord(ev[7], s));
    HIP_TRY(hipStreamSynchronize(s));
    if (timing) S.ms_final = elapsed(ev[6], ev[7]);
    double total;
    memcpy(&total, h->host + 8, sizeof(double));
    S.final_weight = total;
    if (total_out) *total_out = total;
    S.ms_total = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t_begin).count();
    if (stats) *stats = S;
    return HWPM_OK;
}

}  // extern "C"
