// Serving form: a request loop with continuous batching over hwpm_match_batch.
//
// hwpm_submit queues a host CSC (by reference: the caller keeps the arrays
// until the result is polled).  Each worker thread owns a handle on its own
// HIP stream; whenever it is idle it takes, in arrival order, as many queued
// requests as fit into the largest free extent of the device arena (their
// inputs and results plus the batch workspace: admission by HBM footprint),
// copies them in, validates and solves them as one block-diagonal batch and
// hands the results back.  Requests that arrive while batches run are
// admitted by the next idle worker as soon as there is room, and the batches
// of different workers overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hwpm.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Request {
    uint64_t ticket = 0;
    int32_t n = 0;
    int64_t nnz = 0;
    const int64_t* col_ptr = nullptr;  // the caller's host arrays
    const int32_t* row_idx = nullptr;
    const double* w = nullptr;
    size_t input_bytes = 0;  // arena bytes for its arrays and its result
    Clock::time_point t_submit, t_admit, t_done;
    bool done = false;
    bool claimed = false;  // a waiting hwpm_poll owns the ticket
    int status = HWPM_PENDING;
    std::vector<int32_t> perm;
    double total = 0.0;
    hwpm_item_stats item{};
    int32_t batch_size = 0;
    int32_t worker = -1;
};

// First-fit allocator of arena offsets (the memory itself is one hipMalloc).
class Arena {
  public:
    explicit Arena(size_t bytes) { free_[0] = bytes; }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto& f : free_) m = std::max(m, f.second);
        return m;
    }
    bool alloc(size_t bytes, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, start = it->first + bytes;
            free_.erase(it);
            if (rest) free_[start] = rest;
            in_use_ += bytes;
            peak_ = std::max(peak_, in_use_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        in_use_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t in_use() const { return in_use_; }
    size_t peak() const { return peak_; }

  private:
    std::map<size_t, size_t> free_;  // offset -> length, no two adjacent
    size_t in_use_ = 0, peak_ = 0;
};

// Online tuning: the (probe, tile width) candidates each degree bin tries,
// and how many batches each candidate solves before the bin is decided.
constexpr int kTuneCand = 6;
constexpr int32_t kTuneConfigs[kTuneCand][2] = {{5, 4}, {5, 8}, {3, 4}, {3, 8}, {4, 4}, {4, 8}};
constexpr int kTuneTrials = 2;

}  // namespace

struct hwpm_server_s {
    hwpm_server_options opt{};
    char* arena_base = nullptr;
    std::unique_ptr<Arena> arena;
    std::vector<hipStream_t> streams;
    std::vector<hwpm_handle> handles;
    std::mutex mu;
    std::condition_variable cv_work;  // a new request, freed arena space or stop
    std::condition_variable cv_done;  // a result is ready
    std::condition_variable cv_idle;  // the last waiting hwpm_poll left (during destroy)
    std::deque<Request*> pending;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> requests;
    uint64_t next_ticket = 1;
    bool stop = false;
    bool closing = false;     // hwpm_server_destroy has begun: no new polls
    int32_t active_polls = 0; // hwpm_poll calls waiting for a result
    int32_t running = 0;
    hwpm_server_stats stats{};
    std::vector<std::thread> threads;
    // online tuning table and its trials (under mu)
    hwpm_tune_table table{};
    int32_t trials_started[HWPM_TUNE_BINS] = {};
    int32_t trials_done[HWPM_TUNE_BINS] = {};
    float trial_ms[HWPM_TUNE_BINS][kTuneCand] = {};
};

namespace {

size_t batch_footprint(const std::vector<Request*>& b) {
    std::vector<hwpm_csc> d(b.size());
    size_t in = 0;
    for (size_t i = 0; i < b.size(); ++i) {
        d[i].n = b[i]->n;
        d[i].nnz = b[i]->nnz;
        d[i].col_ptr = nullptr;
        d[i].row_idx = nullptr;
        d[i].weight = nullptr;
        in += b[i]->input_bytes;
    }
    size_t ws = 0;
    if (hwpm_batch_workspace_bytes((int32_t)d.size(), d.data(), &ws) != HWPM_OK) return SIZE_MAX;
    return in + align_up(ws);
}

// Under the lock: the next batch in arrival order that fits the largest free
// extent, or an empty batch.  Requests that cannot fit the whole arena even
// alone are completed with HWPM_ETOOBIG.
std::vector<Request*> take_batch(hwpm_server_s* S, size_t* off, size_t* bytes) {
    std::vector<Request*> batch;
    while (!S->pending.empty() && batch_footprint({S->pending.front()}) > S->opt.arena_bytes) {
        Request* r = S->pending.front();
        S->pending.pop_front();
        r->status = HWPM_ETOOBIG;
        r->t_admit = r->t_done = Clock::now();
        r->done = true;
        ++S->stats.completed;
        S->cv_done.notify_all();
    }
    const size_t room = S->arena->largest_free();
    size_t need = 0;
    for (Request* r : S->pending) {
        if ((int32_t)batch.size() >= S->opt.max_batch) break;
        batch.push_back(r);
        const size_t f = batch_footprint(batch);
        if (f > room) {
            batch.pop_back();
            break;
        }
        need = f;
    }
    if (batch.empty() || !S->arena->alloc(need, off)) return {};
    *bytes = need;
    S->pending.erase(S->pending.begin(), S->pending.begin() + (ptrdiff_t)batch.size());
    return batch;
}

// Copy the batch into its arena region, solve it and copy the results back.
// solve_ms (out): host time of the batch solve itself (after the copies in).
int solve_batch(hwpm_server_s* S, int index, std::vector<Request*>& batch, char* base, size_t bytes,
                const hwpm_options& solve, double* solve_ms) {
    hipStream_t stream = S->streams[index];
    size_t at = 0;
    std::vector<hwpm_csc> mats(batch.size());
    std::vector<int32_t*> perms(batch.size());
    for (size_t i = 0; i < batch.size(); ++i) {
        Request* r = batch[i];
        int64_t* cp = (int64_t*)(base + at);
        at += align_up((size_t)(r->n + 1) * 8);
        int32_t* ri = (int32_t*)(base + at);
        at += align_up((size_t)r->nnz * 4);
        double* w = (double*)(base + at);
        at += align_up((size_t)r->nnz * 8);
        perms[i] = (int32_t*)(base + at);
        at += align_up((size_t)r->n * 4);
        if (hipMemcpyAsync(cp, r->col_ptr, (size_t)(r->n + 1) * 8, hipMemcpyHostToDevice, stream) != hipSuccess)
            return HWPM_EDEVICE;
        if (r->nnz > 0 &&
            (hipMemcpyAsync(ri, r->row_idx, (size_t)r->nnz * 4, hipMemcpyHostToDevice, stream) != hipSuccess ||
             hipMemcpyAsync(w, r->w, (size_t)r->nnz * 8, hipMemcpyHostToDevice, stream) != hipSuccess))
            return HWPM_EDEVICE;
        mats[i].n = r->n;
        mats[i].nnz = r->nnz;
        mats[i].col_ptr = cp;
        mats[i].row_idx = ri;
        mats[i].weight = w;
    }
    std::vector<double> totals(batch.size());
    std::vector<hwpm_item_stats> items(batch.size());
    hwpm_handle h = S->handles[index];
    if (hipStreamSynchronize(stream) != hipSuccess) return HWPM_EDEVICE;  // inputs in place
    const auto t0 = Clock::now();
    int st = hwpm_match_batch(h, (int32_t)batch.size(), mats.data(), perms.data(), totals.data(), &solve,
                              items.data(), nullptr, base + at, bytes - at);
    *solve_ms = ms_between(t0, Clock::now());
    if (st == HWPM_EBADCSC && batch.size() > 1) {
        // a malformed member fails the whole batch: solve the members alone so
        // that only the malformed ones report it
        for (size_t i = 0; i < batch.size(); ++i) {
            hwpm_stats one;
            const int si = hwpm_match(h, &mats[i], perms[i], &totals[i], &solve, &one, base + at, bytes - at);
            memset(&items[i], 0, sizeof(items[i]));
            items[i].status = si;
            if (si == HWPM_OK) {
                items[i].rounds = one.rounds;
                items[i].hit_round_cap = one.hit_round_cap;
                items[i].cycles_applied = one.cycles_applied;
                items[i].init_weight = one.init_weight;
                items[i].final_weight = one.final_weight;
            } else if (si != HWPM_ESINGULAR && si != HWPM_EBADCSC) {
                return si;
            }
        }
        st = HWPM_OK;
    } else if (st == HWPM_EBADCSC) {
        items[0].status = HWPM_EBADCSC;
        st = HWPM_OK;
    }
    if (st != HWPM_OK) return st;
    for (size_t i = 0; i < batch.size(); ++i) {
        Request* r = batch[i];
        r->item = items[i];
        r->total = totals[i];
        r->status = items[i].status;
        if (r->status == HWPM_OK && r->n > 0) {
            r->perm.resize((size_t)r->n);
            if (hipMemcpyAsync(r->perm.data(), perms[i], (size_t)r->n * 4, hipMemcpyDeviceToHost, stream) !=
                hipSuccess)
                return HWPM_EDEVICE;
        }
    }
    return hipStreamSynchronize(stream) == hipSuccess ? HWPM_OK : HWPM_EDEVICE;
}

void worker(hwpm_server_s* S, int index) {
    (void)hipSetDevice(S->opt.device);
    for (;;) {
        std::vector<Request*> batch;
        size_t off = 0, bytes = 0;
        hwpm_options solve;
        int cand = -1, bin = -1;
        double work = 0.0;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                batch = take_batch(S, &off, &bytes);
                if (!batch.empty() || (S->stop && S->pending.empty())) break;
                S->cv_work.wait(lk);
            }
            if (batch.empty()) return;
            const auto now = Clock::now();
            for (Request* r : batch) r->t_admit = now;
            // launch configuration: the bin's tuned entry, or the bin's next
            // candidate while the bin is still being tuned
            solve = S->opt.solve;
            cand = -1;
            int64_t n_tot = 0, nnz_tot = 0;
            for (Request* r : batch) {
                n_tot += r->n;
                nnz_tot += r->nnz;
            }
            work = (double)n_tot + (double)nnz_tot;
            bin = hwpm_tune_bin(&S->table, (int32_t)std::min<int64_t>(n_tot, INT32_MAX - 1), nnz_tot);
            if (S->opt.tune && bin >= 0) {
                if (S->table.probe[bin] != 0) {
                    solve.probe = S->table.probe[bin];
                    solve.tile_width = S->table.tile_width[bin];
                } else {
                    cand = S->trials_started[bin]++ % kTuneCand;
                    solve.probe = kTuneConfigs[cand][0];
                    solve.tile_width = kTuneConfigs[cand][1];
                }
            }
            ++S->running;
            ++S->stats.batches;
            S->stats.max_batch_seen = std::max<int64_t>(S->stats.max_batch_seen, (int64_t)batch.size());
            S->stats.max_running = std::max<int64_t>(S->stats.max_running, S->running);
        }
        double solve_ms = 0.0;
        const int st = solve_batch(S, index, batch, S->arena_base + off, bytes, solve, &solve_ms);
        if (st != HWPM_OK) (void)hipStreamSynchronize(S->streams[index]);  // nothing may still use the region
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->arena->release(off, bytes);
            --S->running;
            if (cand >= 0 && st == HWPM_OK && S->table.probe[bin] == 0) {
                // a trial: keep the candidate's best time per million columns
                // and entries; once every candidate has had its trials the bin
                // takes the fastest
                const float ms = (float)(solve_ms / (work * 1e-6 + 1e-12));
                float& best = S->trial_ms[bin][cand];
                if (best == 0.f || ms < best) best = ms;
                if (++S->trials_done[bin] >= kTuneCand * kTuneTrials) {
                    int win = 0;
                    for (int c = 1; c < kTuneCand; ++c)
                        if (S->trial_ms[bin][c] > 0.f &&
                            (S->trial_ms[bin][win] == 0.f || S->trial_ms[bin][c] < S->trial_ms[bin][win]))
                            win = c;
                    S->table.probe[bin] = kTuneConfigs[win][0];
                    S->table.tile_width[bin] = kTuneConfigs[win][1];
                    S->table.ms_per_mentry[bin] = S->trial_ms[bin][win];
                }
            }
            const auto now = Clock::now();
            for (Request* r : batch) {
                if (st != HWPM_OK) r->status = st;
                r->batch_size = (int32_t)batch.size();
                r->worker = index;
                r->t_done = now;
                r->done = true;
                ++S->stats.completed;
            }
        }
        S->cv_work.notify_all();
        S->cv_done.notify_all();
    }
}

void free_server(hwpm_server_s* S) {
    for (hwpm_handle h : S->handles)
        if (h) hwpm_destroy(h);
    for (hipStream_t s : S->streams)
        if (s) (void)hipStreamDestroy(s);
    if (S->arena_base) (void)hipFree(S->arena_base);
    delete S;
}

}  // namespace

extern "C" {

void hwpm_server_default_options(hwpm_server_options* opt) {
    if (!opt) return;
    memset(opt, 0, sizeof(*opt));
    opt->device = 0;
    opt->workers = 2;
    opt->max_batch = 64;
    opt->tune = 1;
    opt->arena_bytes = (size_t)8 << 30;
    hwpm_default_options(&opt->solve);  // check_csc = 1: requests are validated on the device
}

int hwpm_server_create(hwpm_server* out, const hwpm_server_options* opt_in) {
    if (!out) return HWPM_EINVAL;
    hwpm_server_options opt;
    hwpm_server_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (opt.workers < 1 || opt.workers > 16 || opt.max_batch < 1 || opt.arena_bytes < ((size_t)1 << 20) ||
        (opt.tune != 0 && opt.tune != 1))
        return HWPM_EINVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || opt.device < 0 || opt.device >= count) return HWPM_EDEVICE;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (hipSetDevice(opt.device) != hipSuccess) return HWPM_EDEVICE;
    auto* S = new hwpm_server_s();
    S->opt = opt;
    hwpm_default_tune_table(&S->table);
    int st = HWPM_OK;
    void* p = nullptr;
    if (hipMalloc(&p, opt.arena_bytes) != hipSuccess) {
        (void)hipGetLastError();
        st = HWPM_ENOMEM;
    } else {
        S->arena_base = (char*)p;
        S->arena = std::make_unique<Arena>(opt.arena_bytes);
    }
    for (int i = 0; i < opt.workers && st == HWPM_OK; ++i) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            st = HWPM_EDEVICE;
            break;
        }
        S->streams.push_back(s);
        hwpm_handle h = nullptr;
        st = hwpm_create(&h, opt.device, s);
        if (st == HWPM_OK) S->handles.push_back(h);
    }
    if (prev >= 0) (void)hipSetDevice(prev);
    if (st != HWPM_OK) {
        free_server(S);
        return st;
    }
    for (int i = 0; i < opt.workers; ++i) S->threads.emplace_back(worker, S, i);
    *out = S;
    return HWPM_OK;
}

int hwpm_server_destroy(hwpm_server s) {
    if (!s) return HWPM_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->closing = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->threads) t.join();  // every queued request completes
    {
        // polls already waiting get their results and leave before the
        // server's memory goes
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_idle.wait(lk, [s] { return s->active_polls == 0; });
    }
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(s->opt.device);
    free_server(s);
    if (prev >= 0) (void)hipSetDevice(prev);
    return HWPM_OK;
}

int hwpm_submit(hwpm_server s, const hwpm_csc* A, uint64_t* ticket) {
    if (!s || !A || !ticket) return HWPM_EINVAL;
    if (A->n < 0 || A->nnz < 0 || !A->col_ptr || (A->nnz > 0 && (!A->row_idx || !A->weight)))
        return HWPM_EINVAL;
    if (A->n >= INT32_MAX || A->nnz >= ((int64_t)1 << 40)) return HWPM_ETOOBIG;
    if (A->col_ptr[0] != 0 || A->col_ptr[A->n] != A->nnz) return HWPM_EBADCSC;  // the rest on the device
    auto r = std::make_unique<Request>();
    r->t_submit = Clock::now();
    r->n = A->n;
    r->nnz = A->nnz;
    r->col_ptr = A->col_ptr;
    r->row_idx = A->row_idx;
    r->w = A->weight;
    r->input_bytes = align_up((size_t)(A->n + 1) * 8) + align_up((size_t)A->nnz * 4) +
                     align_up((size_t)A->nnz * 8) + align_up((size_t)A->n * 4);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return HWPM_EINVAL;
        r->ticket = s->next_ticket++;
        *ticket = r->ticket;
        s->pending.push_back(r.get());
        s->requests.emplace(r->ticket, std::move(r));
        ++s->stats.submitted;
    }
    s->cv_work.notify_one();
    return HWPM_OK;
}

int hwpm_poll(hwpm_server s, uint64_t ticket, int32_t wait, int32_t* perm_host, double* total,
              hwpm_request_info* info) {
    if (!s) return HWPM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->closing) return HWPM_EINVAL;
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return HWPM_EINVAL;
    Request* r = it->second.get();
    if (r->claimed) return HWPM_EINVAL;  // another caller is waiting for this ticket
    if (!r->done) {
        if (!wait) return HWPM_PENDING;
        // claim the ticket, so that no other caller reads or frees the
        // request while this one waits (workers complete every request)
        r->claimed = true;
        ++s->active_polls;
        s->cv_done.wait(lk, [r] { return r->done; });
        if (--s->active_polls == 0 && s->closing) s->cv_idle.notify_all();
    }
    const int status = r->status;
    if (status == HWPM_OK) {
        if (perm_host && r->n > 0) memcpy(perm_host, r->perm.data(), (size_t)r->n * 4);
        if (total) *total = r->total;
    }
    if (info) {
        info->item = r->item;
        info->item.status = status;
        info->queue_ms = ms_between(r->t_submit, r->t_admit);
        info->latency_ms = ms_between(r->t_submit, r->t_done);
        info->batch_size = r->batch_size;
        info->worker = r->worker;
    }
    s->requests.erase(it);
    return status;
}

int hwpm_server_get_tune_table(hwpm_server s, hwpm_tune_table* t) {
    if (!s || !t) return HWPM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *t = s->table;
    return HWPM_OK;
}

int hwpm_server_get_stats(hwpm_server s, hwpm_server_stats* st) {
    if (!s || !st) return HWPM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *st = s->stats;
    st->pending = (int64_t)s->pending.size();
    st->running = s->running;
    st->arena_in_use = (int64_t)s->arena->in_use();
    st->arena_peak = (int64_t)s->arena->peak();
    return HWPM_OK;
}

}  // extern "C"
