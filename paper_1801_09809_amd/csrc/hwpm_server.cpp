// Serving form: a request loop with continuous batching at round granularity.
//
// hwpm_submit queues a host CSC (copied at once, or kept by reference when
// the server is so configured).  Each worker thread owns a handle on its own
// HIP stream and a set of requests in flight.  A request admitted by a worker
// gets its own region of the device arena (its inputs and its matching) for
// as long as it is in flight.  The worker runs in steps: it admits, in
// arrival order, as many queued requests as fit (admission by HBM
// footprint), finds their perfect matchings (one packed call), and then
// improves the matchings of every request it holds -- those just admitted
// and those from earlier steps -- by up to rounds_per_step rounds in one
// block-diagonal batch (Section 5.3 rounds; a round on the packed matrix is
// that round on every block at once).  Requests whose rounds have ended leave
// with their results; the others stay resident and continue in the next
// step, joined by whatever arrived meanwhile.  Each round is a function of
// the matching alone, so a request's rounds are the same whether they run in
// one call or across steps, alone or packed with others.
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
#include "hwpm_serving.h"

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
    const int64_t* col_ptr = nullptr;  // the caller's host arrays, or the copies below
    const int32_t* row_idx = nullptr;
    const double* w = nullptr;
    std::vector<int64_t> cp_copy;      // copies made by hwpm_submit (copy_inputs = 1)
    std::vector<int32_t> ri_copy;
    std::vector<double> w_copy;
    size_t input_bytes = 0;  // arena bytes for its arrays and its matching
    size_t off = 0;          // its arena region while in flight
    int64_t* d_col_ptr = nullptr;  // device copies in that region
    int32_t* d_row_idx = nullptr;
    double* d_w = nullptr;
    int32_t* d_perm = nullptr;     // its current matching, then its result
    Clock::time_point t_submit, t_admit, t_done;
    bool done = false;
    bool claimed = false;  // a waiting hwpm_poll owns the ticket
    int status = HWPM_PENDING;
    std::vector<int32_t> perm;
    double total = 0.0;
    hwpm_item_stats item{};
    int32_t rounds = 0;        // rounds run so far (over its steps)
    int64_t cycles = 0;        // cycles flipped so far
    double init_weight = 0.0;  // weight of its initial perfect matching
    int32_t steps = 0;         // round steps it took part in
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

// Batch workspace bytes for a set of requests (SIZE_MAX when too big).
size_t workspace_for(const std::vector<Request*>& a, const std::vector<Request*>& b) {
    std::vector<hwpm_csc> d;
    d.reserve(a.size() + b.size());
    for (const auto* v : {&a, &b})
        for (const Request* r : *v) {
            hwpm_csc c{};
            c.n = r->n;
            c.nnz = r->nnz;
            d.push_back(c);
        }
    size_t ws = 0;
    if (hwpm_batch_workspace_bytes((int32_t)d.size(), d.data(), &ws) != HWPM_OK) return SIZE_MAX;
    return align_up(ws);
}

void complete(hwpm_server_s* S, Request* r, int status) {
    r->status = status;
    r->t_done = Clock::now();
    r->done = true;
    ++S->stats.completed;
}

// Under the lock: admit queued requests in arrival order next to the
// worker's requests in flight (`held`), as long as each one's region and the
// batch workspace of them all fit the arena; the workspace (*ws_off,
// *ws_bytes, held by the worker between steps) grows as needed.  Requests
// that cannot fit the whole arena even alone are completed with
// HWPM_ETOOBIG.
std::vector<Request*> admit(hwpm_server_s* S, const std::vector<Request*>& held, size_t* ws_off,
                            size_t* ws_bytes) {
    std::vector<Request*> fresh;
    while (!S->pending.empty()) {
        Request* r = S->pending.front();
        if ((int32_t)(held.size() + fresh.size()) >= S->opt.max_batch) break;
        const size_t alone = workspace_for({r}, {});
        if (alone == SIZE_MAX || r->input_bytes + alone > S->opt.arena_bytes) {
            S->pending.pop_front();
            r->t_admit = Clock::now();
            complete(S, r, HWPM_ETOOBIG);
            S->cv_done.notify_all();
            continue;
        }
        size_t off = 0;
        if (!S->arena->alloc(r->input_bytes, &off)) break;
        fresh.push_back(r);
        const size_t need = workspace_for(held, fresh);
        if (need > *ws_bytes) {
            // grow the workspace: give the old one back, take a larger one
            // (or the old size again, which then always fits)
            if (*ws_bytes) S->arena->release(*ws_off, *ws_bytes);
            size_t w = 0;
            if (need != SIZE_MAX && S->arena->alloc(need, &w)) {
                *ws_off = w;
                *ws_bytes = need;
            } else {
                if (*ws_bytes) (void)S->arena->alloc(*ws_bytes, ws_off);
                fresh.pop_back();
                S->arena->release(off, r->input_bytes);
                break;
            }
        }
        r->off = off;
        S->pending.pop_front();
    }
    return fresh;
}

// Place a request's arrays in its region and copy them in.
int upload(Request* r, char* base, hipStream_t stream) {
    size_t at = r->off;
    r->d_col_ptr = (int64_t*)(base + at);
    at += align_up((size_t)(r->n + 1) * 8);
    r->d_row_idx = (int32_t*)(base + at);
    at += align_up((size_t)r->nnz * 4);
    r->d_w = (double*)(base + at);
    at += align_up((size_t)r->nnz * 8);
    r->d_perm = (int32_t*)(base + at);
    if (hipMemcpyAsync(r->d_col_ptr, r->col_ptr, (size_t)(r->n + 1) * 8, hipMemcpyHostToDevice, stream) !=
        hipSuccess)
        return HWPM_EDEVICE;
    if (r->nnz > 0 &&
        (hipMemcpyAsync(r->d_row_idx, r->row_idx, (size_t)r->nnz * 4, hipMemcpyHostToDevice, stream) != hipSuccess ||
         hipMemcpyAsync(r->d_w, r->w, (size_t)r->nnz * 8, hipMemcpyHostToDevice, stream) != hipSuccess))
        return HWPM_EDEVICE;
    return HWPM_OK;
}

hwpm_csc descriptor(const Request* r) {
    hwpm_csc c;
    c.n = r->n;
    c.nnz = r->nnz;
    c.col_ptr = r->d_col_ptr;
    c.row_idx = r->d_row_idx;
    c.weight = r->d_w;
    return c;
}

// One step of a worker: copy the fresh requests in, find their perfect
// matchings, then run up to `rounds` rounds on every request in flight (held
// and fresh) as one packed batch.  Requests that finish (their rounds ended,
// or a failure of their own) are moved to *finished with their status and
// results; the others stay in *held.  step_ms (out): host time of the
// matching and round calls.
int run_step(hwpm_server_s* S, int index, std::vector<Request*>* held, const std::vector<Request*>& fresh,
             char* ws, size_t ws_bytes, const hwpm_options& solve, int32_t rounds,
             std::vector<Request*>* finished, double* step_ms) {
    hipStream_t stream = S->streams[index];
    hwpm_handle h = S->handles[index];
    for (Request* r : fresh) {
        const int st = upload(r, S->arena_base, stream);
        if (st != HWPM_OK) return st;
    }
    if (hipStreamSynchronize(stream) != hipSuccess) return HWPM_EDEVICE;  // inputs in place
    const auto t0 = Clock::now();
    std::vector<Request*> members = *held;
    if (!fresh.empty()) {
        // initial perfect matchings of the fresh requests (validated first
        // when the solve options ask for it)
        const size_t f = fresh.size();
        std::vector<hwpm_csc> mats(f);
        std::vector<int32_t*> perms(f);
        std::vector<hwpm_item_stats> items(f);
        for (size_t i = 0; i < f; ++i) {
            mats[i] = descriptor(fresh[i]);
            perms[i] = fresh[i]->d_perm;
        }
        int st = hwpm::match_batch_initial(h, (int32_t)f, mats.data(), perms.data(), &solve, items.data(), ws,
                                           ws_bytes);
        if (st == HWPM_EBADCSC) {
            // a malformed request fails the packed call: match each alone, so
            // that only the malformed ones report it
            for (size_t i = 0; i < f; ++i) {
                hwpm_item_stats one{};
                const int si = hwpm::match_batch_initial(h, 1, &mats[i], &perms[i], &solve, &one, ws, ws_bytes);
                items[i] = one;
                items[i].status = si == HWPM_OK ? one.status : si;
                if (si != HWPM_OK && si != HWPM_EBADCSC) return si;
            }
            st = HWPM_OK;
        }
        if (st != HWPM_OK) return st;
        for (size_t i = 0; i < f; ++i) {
            if (items[i].status == HWPM_OK) {
                members.push_back(fresh[i]);
            } else {
                fresh[i]->status = items[i].status;
                finished->push_back(fresh[i]);
            }
        }
    }
    held->clear();
    if (!members.empty()) {
        const size_t m = members.size();
        std::vector<hwpm_csc> mats(m);
        std::vector<const int32_t*> in(m);
        std::vector<int32_t*> out(m);
        std::vector<double> totals(m);
        std::vector<hwpm_item_stats> items(m);
        for (size_t i = 0; i < m; ++i) {
            mats[i] = descriptor(members[i]);
            in[i] = members[i]->d_perm;
            out[i] = members[i]->d_perm;
        }
        hwpm_options opt = solve;
        opt.check_csc = 0;  // validated when admitted
        opt.max_rounds = rounds;
        const int st = hwpm_improve_batch(h, (int32_t)m, mats.data(), in.data(), out.data(), totals.data(), &opt,
                                          items.data(), nullptr, ws, ws_bytes);
        if (st != HWPM_OK) {
            for (Request* r : members) held->push_back(r);
            return st;
        }
        for (size_t i = 0; i < m; ++i) {
            Request* r = members[i];
            const hwpm_item_stats& it = items[i];
            if (r->steps == 0) r->init_weight = it.init_weight;
            ++r->steps;
            r->rounds += it.rounds;
            r->cycles += it.cycles_applied;
            const bool ended = !it.hit_round_cap;                                         // a round found nothing
            const bool capped = solve.max_rounds > 0 && r->rounds >= solve.max_rounds;  // the caller's cap
            if (!ended && !capped) {
                held->push_back(r);
                continue;
            }
            r->status = HWPM_OK;
            r->total = totals[i];
            r->item.status = HWPM_OK;
            r->item.rounds = r->rounds;
            r->item.hit_round_cap = ended ? 0 : 1;
            r->item.reserved = 0;
            r->item.cycles_applied = r->cycles;
            r->item.init_weight = r->init_weight;
            r->item.final_weight = it.final_weight;
            if (r->n > 0) {
                r->perm.resize((size_t)r->n);
                if (hipMemcpyAsync(r->perm.data(), r->d_perm, (size_t)r->n * 4, hipMemcpyDeviceToHost, stream) !=
                    hipSuccess)
                    return HWPM_EDEVICE;
            }
            finished->push_back(r);
        }
    }
    const bool ok = hipStreamSynchronize(stream) == hipSuccess;
    *step_ms = ms_between(t0, Clock::now());
    return ok ? HWPM_OK : HWPM_EDEVICE;
}

void worker(hwpm_server_s* S, int index) {
    (void)hipSetDevice(S->opt.device);
    std::vector<Request*> held;       // requests in flight on this worker
    size_t ws_off = 0, ws_bytes = 0;  // their batch workspace, held between steps
    for (;;) {
        std::vector<Request*> fresh;
        hwpm_options solve;
        int cand = -1, bin = -1;
        double work = 0.0;
        int32_t rounds = 0;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                fresh = admit(S, held, &ws_off, &ws_bytes);
                if (!fresh.empty() || !held.empty()) break;
                if (ws_bytes) {  // idle: the workspace goes back to the arena
                    S->arena->release(ws_off, ws_bytes);
                    ws_bytes = 0;
                    S->cv_work.notify_all();
                }
                if (S->stop && S->pending.empty()) return;
                S->cv_work.wait(lk);
            }
            const auto now = Clock::now();
            for (Request* r : fresh) {
                r->t_admit = now;
                r->batch_size = (int32_t)(held.size() + fresh.size());
                r->worker = index;
            }
            if (!held.empty()) S->stats.joined += (int64_t)fresh.size();
            // launch configuration: the bin's tuned entry, or the bin's next
            // candidate while the bin is still being tuned
            solve = S->opt.solve;
            int64_t n_tot = 0, nnz_tot = 0;
            for (const auto* v : {&held, &fresh})
                for (Request* r : *v) {
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
            // rounds of this step: rounds_per_step, within every request's
            // share of the caller's cap
            rounds = S->opt.rounds_per_step;
            if (solve.max_rounds > 0)
                for (const auto* v : {&held, &fresh})
                    for (Request* r : *v) {
                        const int32_t left = solve.max_rounds - r->rounds;
                        if (rounds == 0 || left < rounds) rounds = left;
                    }
            ++S->running;
            ++S->stats.batches;
            S->stats.max_batch_seen =
                std::max<int64_t>(S->stats.max_batch_seen, (int64_t)(held.size() + fresh.size()));
            S->stats.max_running = std::max<int64_t>(S->stats.max_running, S->running);
        }
        std::vector<Request*> finished;
        double step_ms = 0.0;
        const int st = run_step(S, index, &held, fresh, S->arena_base + ws_off, ws_bytes, solve, rounds, &finished,
                                &step_ms);
        if (st != HWPM_OK) {
            // nothing may still use the regions; every request of the step fails
            (void)hipStreamSynchronize(S->streams[index]);
            for (Request* r : fresh)
                if (std::find(finished.begin(), finished.end(), r) == finished.end() &&
                    std::find(held.begin(), held.end(), r) == held.end())
                    held.push_back(r);
            for (Request* r : held) {
                r->status = st;
                finished.push_back(r);
            }
            held.clear();
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            --S->running;
            if (cand >= 0 && st == HWPM_OK && S->table.probe[bin] == 0) {
                // a trial: keep the candidate's best time per million columns
                // and entries; once every candidate has had its trials the bin
                // takes the fastest
                const float ms = (float)(step_ms / (work * 1e-6 + 1e-12));
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
            for (Request* r : finished) {
                S->arena->release(r->off, r->input_bytes);
                if (r->status != HWPM_OK) {
                    r->item = hwpm_item_stats{};
                    r->item.status = r->status;
                }
                complete(S, r, r->status);
            }
            if (held.empty() && ws_bytes) {
                S->arena->release(ws_off, ws_bytes);
                ws_bytes = 0;
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
    opt->rounds_per_step = 8;
    opt->copy_inputs = 1;
}

int hwpm_server_create(hwpm_server* out, const hwpm_server_options* opt_in) {
    if (!out) return HWPM_EINVAL;
    hwpm_server_options opt;
    hwpm_server_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (opt.workers < 1 || opt.workers > 16 || opt.max_batch < 1 || opt.arena_bytes < ((size_t)1 << 20) ||
        (opt.tune != 0 && opt.tune != 1) || opt.rounds_per_step < 0 || (opt.copy_inputs != 0 && opt.copy_inputs != 1))
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
    if (s->opt.copy_inputs) {
        // the server's own copies: the caller may reuse its arrays at once
        r->cp_copy.assign(A->col_ptr, A->col_ptr + A->n + 1);
        r->ri_copy.assign(A->row_idx, A->row_idx + A->nnz);
        r->w_copy.assign(A->weight, A->weight + A->nnz);
        r->col_ptr = r->cp_copy.data();
        r->row_idx = r->ri_copy.data();
        r->w = r->w_copy.data();
    } else {
        r->col_ptr = A->col_ptr;
        r->row_idx = A->row_idx;
        r->w = A->weight;
    }
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
        info->steps = r->steps;
        info->reserved = 0;
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
