// Served form: a request loop with memory-budget admission and several
// queries in flight, each on its own slot's stream (queries are not merged
// into shared launches).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "slg.h"
#include "slg_arena.h"
#include "slg_host.h"

namespace {

using Clock = std::chrono::steady_clock;
constexpr int32_t kMaxWorkers = 16;

struct Request {
    uint64_t ticket = 0;
    slg_graph *g = nullptr;
    int32_t s[SLG_MAX_S] = {};
    int32_t k = 0;
    Clock::time_point t_submit, t_start, t_done;
    bool started = false, done = false, cancelled = false;
    slg_status status = SLG_OK;
    slg_result *result = nullptr;
    std::string message;
    int64_t two_paths = 0;
    uint64_t held = 0;  // budget bytes this query holds while it runs
    int32_t attempts = 0;
};

struct Worker {
    std::thread th;
    hipStream_t st = nullptr;
    slg_context *ctx = nullptr;
};

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

struct slg_server {
    int device = 0;
    std::shared_ptr<slg::ServeCore> core;  // its mutex and condition guard everything below
    std::deque<Request *> queue;           // not started (or yielded), arrival order
    std::unordered_map<uint64_t, Request *> live;  // not yet retired
    std::deque<Request *> finished;        // completion order, may hold retired entries' tickets
    uint64_t next_ticket = 1;
    Request *waiter = nullptr;  // the one query waiting for memory
    bool stop = false;
    std::vector<Worker> workers;
    int64_t submitted = 0, completed = 0, failed = 0, yields = 0, running = 0;
};

namespace {

// Budget request of query q (runs on q's worker thread, inside a planning
// phase). Returns false to refuse; *yield tells whether q should go back to
// the queue (another query already waits) rather than fail.
bool grant(slg_server *sv, Request *q, uint64_t bytes, bool *yield) {
    slg::ServeCore &c = *sv->core;
    std::unique_lock<std::mutex> lk(c.mu);
    if (c.budget && q->held + bytes > c.budget) return false;  // can never fit
    while (c.budget && c.used + bytes > c.budget) {
        if (sv->stop) {
            q->cancelled = true;
            if (sv->waiter == q) sv->waiter = nullptr;
            c.cv.notify_all();
            return false;
        }
        if (sv->waiter && sv->waiter != q) {
            *yield = true;
            return false;
        }
        sv->waiter = q;  // everyone else finishes, yields, or is a result the caller holds
        c.cv.wait(lk);
    }
    if (sv->waiter == q) sv->waiter = nullptr;
    c.used += bytes;
    c.peak = std::max(c.peak, c.used);
    q->held += bytes;
    c.cv.notify_all();  // the admission gate may be open again
    return true;
}

void finish(slg_server *sv, Request *q, slg_status st) {
    q->status = st;
    q->done = true;
    q->t_done = Clock::now();
    sv->finished.push_back(q);
    if (st == SLG_OK)
        ++sv->completed;
    else
        ++sv->failed;
}

void worker_main(slg_server *sv, int wi) {
    Worker &w = sv->workers[wi];
    (void)hipSetDevice(sv->device);
    slg::ServeCore &c = *sv->core;
    std::unique_lock<std::mutex> lk(c.mu);
    for (;;) {
        c.cv.wait(lk, [&] { return sv->stop || (!sv->queue.empty() && !sv->waiter); });
        if (sv->stop) return;
        Request *q = sv->queue.front();
        sv->queue.pop_front();
        if (!q->started) {
            q->started = true;
            q->t_start = Clock::now();
        }
        ++q->attempts;
        ++sv->running;
        lk.unlock();

        bool yield = false;
        const slg::ReserveFn reserve = [&](uint64_t bytes) { return grant(sv, q, bytes, &yield); };
        slg_result *r = nullptr;
        uint64_t scratch = 0, output = 0;
        const slg_status rc = slg::serve_query(w.ctx, q->g, q->s, q->k, w.st, reserve, sv->core, &r, &scratch,
                                               &output);
        lk.lock();
        --sv->running;
        // the query's stream has drained: its scratch is free again
        c.used -= scratch;
        q->held -= scratch;
        if (rc == SLG_OK) {
            c.held_by_results += output;  // the result now owns these bytes
            q->held -= output;
            q->result = r;
            int64_t e = 0;
            (void)slg_result_info(r, 0, &e, &q->two_paths);
            finish(sv, q, SLG_OK);
        } else {
            c.used -= output;
            q->held -= output;
            if (yield && !sv->stop) {
                ++sv->yields;
                sv->queue.push_front(q);
            } else {
                q->message = q->cancelled ? "server shut down" : slg_last_error(w.ctx);
                finish(sv, q, q->cancelled ? SLG_ERR_CANCELLED : rc);
            }
        }
        if (sv->waiter == q) sv->waiter = nullptr;
        c.cv.notify_all();
    }
}

void fill_info(const Request *q, slg_request_info *info) {
    if (!info) return;
    info->ticket = q->ticket;
    info->status = q->status;
    info->attempts = q->attempts;
    info->queue_ms = q->started ? ms_between(q->t_submit, q->t_start) : ms_between(q->t_submit, q->t_done);
    info->latency_ms = ms_between(q->t_submit, q->t_done);
    info->two_paths = q->two_paths;
    const size_t n = std::min(q->message.size(), sizeof(info->message) - 1);
    std::copy(q->message.begin(), q->message.begin() + n, info->message);
    info->message[n] = '\0';
}

// Hands a finished query to the caller and retires its ticket (lock held;
// the caller frees *res after unlocking when it does not want it).
slg_status retire(slg_server *sv, Request *q, slg_result **res, slg_request_info *info) {
    fill_info(q, info);
    *res = q->result;
    const slg_status st = q->status;
    sv->live.erase(q->ticket);
    auto it = std::find(sv->finished.begin(), sv->finished.end(), q);
    if (it != sv->finished.end()) sv->finished.erase(it);
    delete q;
    return st;
}

void hand_over(slg_result *r, slg_result **out) {
    if (out)
        *out = r;
    else if (r)
        (void)slg_result_free(r);
}

template <class Pred>
bool wait_for(slg_server *sv, std::unique_lock<std::mutex> &lk, int32_t timeout_ms, Pred pred) {
    if (timeout_ms < 0) {
        sv->core->cv.wait(lk, pred);
        return true;
    }
    return sv->core->cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred);
}

}  // namespace

extern "C" {

slg_status slg_server_create(slg_context *ctx, int32_t workers, uint64_t mem_budget_bytes, slg_server **out) {
    if (!ctx || !out || workers < 1 || workers > kMaxWorkers) return SLG_ERR_INVALID_ARG;
    *out = nullptr;
    slg_server *sv = new (std::nothrow) slg_server();
    if (!sv) return slg::set_error(ctx, SLG_ERR_OUT_OF_MEMORY, "host allocation failed");
    sv->device = slg::context_device(ctx);
    sv->core = std::make_shared<slg::ServeCore>();
    sv->core->budget = mem_budget_bytes;
    // one block cache for every slot: freed blocks keep at most the budget
    // (16 GiB without one) beyond what the queries hold. A smaller cache
    // thrashes on large queries: every one that ends pushes the cache over,
    // the largest blocks go back to the device's pool and the next large
    // query takes them from there again.
    const uint64_t cache = mem_budget_bytes ? mem_budget_bytes : (uint64_t(16) << 30);
    std::shared_ptr<slg::Arena> arena;
    auto undo = [&](slg_status code, const char *msg) {
        for (Worker &w : sv->workers) {
            if (w.st) (void)hipStreamDestroy(w.st);
            if (w.ctx) (void)slg_context_destroy(w.ctx);
        }
        delete sv;
        return slg::set_error(ctx, code, msg);
    };
    if (hipSetDevice(sv->device) != hipSuccess) return undo(SLG_ERR_DEVICE, "hipSetDevice failed");
    arena = std::make_shared<slg::Arena>(sv->device, cache);
    sv->workers.resize(workers);
    for (Worker &w : sv->workers) {
        if (slg::create_context(sv->device, 0, nullptr, false, &w.ctx) != SLG_OK)
            return undo(SLG_ERR_DEVICE, "worker context creation failed");
        slg::copy_tuning(w.ctx, ctx);
        slg::share_arena(w.ctx, arena);
        if (hipStreamCreateWithFlags(&w.st, hipStreamNonBlocking) != hipSuccess)
            return undo(SLG_ERR_DEVICE, "worker stream creation failed");
    }
    for (int i = 0; i < workers; ++i) sv->workers[i].th = std::thread(worker_main, sv, i);
    *out = sv;
    return SLG_OK;
}

slg_status slg_server_submit(slg_server *sv, slg_graph *g, const int32_t *s, int32_t num_s, uint64_t *ticket) {
    if (!sv || !g || !s || !ticket || num_s < 1 || num_s > SLG_MAX_S) return SLG_ERR_INVALID_ARG;
    if (s[0] < 1) return SLG_ERR_INVALID_ARG;
    for (int32_t t = 1; t < num_s; ++t)
        if (s[t] <= s[t - 1]) return SLG_ERR_INVALID_ARG;
    if (slg::context_device(slg::graph_context(g)) != sv->device) return SLG_ERR_INVALID_ARG;
    Request *q = new (std::nothrow) Request();
    if (!q) return SLG_ERR_OUT_OF_MEMORY;
    q->g = g;
    q->k = num_s;
    std::copy(s, s + num_s, q->s);
    std::lock_guard<std::mutex> lk(sv->core->mu);
    if (sv->stop) {
        delete q;
        return SLG_ERR_CANCELLED;
    }
    q->ticket = sv->next_ticket++;
    q->t_submit = Clock::now();
    sv->live[q->ticket] = q;
    sv->queue.push_back(q);
    ++sv->submitted;
    *ticket = q->ticket;
    sv->core->cv.notify_all();
    return SLG_OK;
}

slg_status slg_server_wait(slg_server *sv, uint64_t ticket, int32_t timeout_ms, slg_result **out,
                           slg_request_info *info) {
    if (!sv) return SLG_ERR_INVALID_ARG;
    if (out) *out = nullptr;
    std::unique_lock<std::mutex> lk(sv->core->mu);
    if (!sv->live.count(ticket)) return SLG_ERR_INVALID_ARG;
    // look the ticket up on every wake-up: another thread may retire it
    auto ended = [&] {
        auto it = sv->live.find(ticket);
        return it == sv->live.end() || it->second->done;
    };
    if (!wait_for(sv, lk, timeout_ms, ended)) return SLG_ERR_TIMEOUT;
    auto it = sv->live.find(ticket);
    if (it == sv->live.end()) return SLG_ERR_INVALID_ARG;
    slg_result *r = nullptr;
    const slg_status st = retire(sv, it->second, &r, info);
    lk.unlock();
    hand_over(r, out);
    return st;
}

slg_status slg_server_next(slg_server *sv, int32_t timeout_ms, slg_result **out, slg_request_info *info) {
    if (!sv) return SLG_ERR_INVALID_ARG;
    if (out) *out = nullptr;
    std::unique_lock<std::mutex> lk(sv->core->mu);
    if (!wait_for(sv, lk, timeout_ms, [&] { return !sv->finished.empty(); })) return SLG_ERR_TIMEOUT;
    slg_result *r = nullptr;
    const slg_status st = retire(sv, sv->finished.front(), &r, info);
    lk.unlock();
    hand_over(r, out);
    return st;
}

slg_status slg_server_stats(slg_server *sv, int64_t *out, int32_t cap, int32_t *count) {
    if (!sv || !out || cap < 0) return SLG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(sv->core->mu);
    const slg::ServeCore &c = *sv->core;
    const int64_t v[9] = {sv->submitted, sv->completed, sv->failed, sv->yields, (int64_t)sv->queue.size(),
                          sv->running, (int64_t)c.used, (int64_t)c.peak, (int64_t)c.held_by_results};
    const int32_t n = std::min<int32_t>(cap, 9);
    std::copy(v, v + n, out);
    if (count) *count = n;
    return SLG_OK;
}

slg_status slg_server_destroy(slg_server *sv) {
    if (!sv) return SLG_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(sv->core->mu);
        sv->stop = true;
        for (Request *q : sv->queue) {
            q->cancelled = true;
            q->message = "server shut down";
            finish(sv, q, SLG_ERR_CANCELLED);
        }
        sv->queue.clear();
        sv->core->cv.notify_all();
    }
    for (Worker &w : sv->workers)
        if (w.th.joinable()) w.th.join();
    for (auto &kv : sv->live) {
        if (kv.second->result) (void)slg_result_free(kv.second->result);
        delete kv.second;
    }
    sv->live.clear();
    (void)hipSetDevice(sv->device);
    for (Worker &w : sv->workers) {
        (void)hipStreamSynchronize(w.st);
        (void)hipStreamDestroy(w.st);
        (void)slg_context_destroy(w.ctx);
    }
    (void)hipGetLastError();
    delete sv;  // the ledger lives on while served results remain
    return SLG_OK;
}

}  // extern "C"
