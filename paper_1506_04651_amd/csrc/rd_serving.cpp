/*
 * rd_serving.cpp -- request sessions (include/rd.h, "Serving").
 *
 * A session owns an arena of device memory of a fixed byte budget.  Requests
 * queue in arrival order; a scheduler thread admits a request as soon as its
 * working set (states, stats if asked for, and the claim-order scratch of its
 * persistent launch) fits in the arena, copies the caller's states into the
 * arena once the producer's work on them has completed (an event recorded at
 * submission), launches the reaction-step kernel on one of a pool of streams,
 * copies the results back and records an event.  Requests admitted while
 * others run go to other streams, so their kernels overlap on the device;
 * completion frees arena space, which admits the next requests.  Per-cell
 * arithmetic does not depend on what else runs, so a request gives bitwise
 * the same result alone or in a mix (same kernel variant).
 *
 * A request that is larger than the whole budget is refused (RD_ETOOBIG).
 * The queue head may be bypassed by later requests that fit, until it has
 * waited kHeadWaitNs; from then on admission waits for the head.
 *
 * Locking: one mutex guards the queue, the arena, the slot and event pools
 * and the request table; the scheduler releases it while it enqueues copies
 * and kernels, so rd_submit / rd_poll never wait behind HIP calls.
 */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rd_internal.h"

namespace rd {

static uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

/* First-fit allocator over [0, size) with coalescing. */
class Arena {
public:
    explicit Arena(size_t size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t noff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
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

private:
    std::map<size_t, size_t> free_;
};

enum ReqState { Q_QUEUED = 0, Q_RUNNING = 1, Q_DONE = 2 };

struct Request {
    uint64_t id = 0;
    Prepared pr;
    double* user_states = nullptr;
    int32_t* user_stats = nullptr;
    int32_t m = 0;
    size_t bytes = 0, off = 0;
    int state = Q_QUEUED;
    int status = 0;
    int slot = -1, stream = -1;
    int32_t deferred = 0; /* scheduler passes in which it did not fit */
    int64_t n_failed = 0, batch = -1;
    uint64_t t_submit = 0, t_admit = 0, t_done = 0;
    double k_start_ms = -1.0, k_end_ms = -1.0;
    hipEvent_t ready = nullptr; /* recorded on the producer's stream at submission */
    char err[256] = "";
};

}  // namespace rd

struct rd_session {
    int device = 0;
    size_t budget = 0;
    char* arena_base = nullptr;
    std::unique_ptr<rd::Arena> arena;
    std::vector<hipStream_t> streams;
    unsigned next_stream = 0;
    unsigned long long* counters = nullptr; /* 2 per slot */
    unsigned long long* host_fail = nullptr;/* pinned, 1 per slot */
    std::vector<int> free_slots;
    /* per slot: completion (no timing), kernel start and end (timing) */
    std::vector<hipEvent_t> ev_done, ev_k0, ev_k1;
    std::vector<hipEvent_t> free_ready; /* pool of submission events */
    hipEvent_t origin = nullptr;        /* device time zero of the session */
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<rd::Request*> queue;
    std::vector<rd::Request*> running;
    std::unordered_map<uint64_t, std::shared_ptr<rd::Request>> reqs;
    uint64_t next_id = 1;
    int64_t next_batch = 0;
    bool closing = false;
    std::thread worker;
    rd_options defaults{};
};

namespace rd {

constexpr int kSessionSlots = 1024;
constexpr uint64_t kHeadWaitNs = 50ull * 1000 * 1000;

static void req_error(Request* r, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(r->err, sizeof(r->err), fmt, ap);
    va_end(ap);
}

#define REQ_TRY(r, expr)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            req_error(r, "%s failed: %s", #expr, hipGetErrorString(e_));                   \
            return false;                                                                  \
        }                                                                                  \
    } while (0)

/* Enqueue the copies and the kernel of an admitted request (called without
 * the session lock); false on a HIP error, with the message in r->err. */
static bool launch_request(rd_session* s, Request* r) {
    hipStream_t st = s->streams[r->stream];
    const int64_t n = r->pr.args.n;
    const size_t sbytes = (size_t)n * r->m * sizeof(double);
    const size_t tbytes = r->user_stats ? align256((size_t)n * RD_NSTATS * sizeof(int32_t)) : 0;
    char* base = s->arena_base + r->off;
    double* a_states = (double*)base;
    int32_t* a_stats = r->user_stats ? (int32_t*)(base + align256(sbytes)) : nullptr;
    void* a_order = order_bytes(n) ? (void*)(base + align256(sbytes) + tbytes) : nullptr;
    Prepared pr = r->pr;
    pr.args.states = a_states;
    pr.args.stats = a_stats;
    pr.args.counter = s->counters + 2 * r->slot;
    pr.args.nfail = pr.args.counter + 1;
    /* the caller's states are read only after its producer stream got there */
    REQ_TRY(r, hipStreamWaitEvent(st, r->ready, 0));
    REQ_TRY(r, hipMemcpyAsync(a_states, r->user_states, sbytes, hipMemcpyDeviceToDevice, st));
    DevCtx* ctx = current_ctx();
    if (!ctx) { req_error(r, "no device context"); return false; }
    bool cleared = false;
    if (enqueue_order(*ctx, pr, st, pr.args.counter, &cleared, a_order) != 0) {
        req_error(r, "claim-order launch failed");
        return false;
    }
    const LaunchArgs& a = pr.args;
    if (!cleared) REQ_TRY(r, launch_reset(a.counter, 2, st));
    REQ_TRY(r, hipEventRecord(s->ev_k0[r->slot], st));
    REQ_TRY(r, pr.entry->launch(a, pr.grid, st));
    REQ_TRY(r, hipEventRecord(s->ev_k1[r->slot], st));
    REQ_TRY(r, hipMemcpyAsync(r->user_states, a_states, sbytes, hipMemcpyDeviceToDevice, st));
    if (a_stats)
        REQ_TRY(r, hipMemcpyAsync(r->user_stats, a_stats, (size_t)n * RD_NSTATS * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, st));
    REQ_TRY(r, hipMemcpyAsync(s->host_fail + r->slot, a.nfail, sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, st));
    REQ_TRY(r, hipEventRecord(s->ev_done[r->slot], st));
    return true;
}

/* Under the session lock. */
static void complete(rd_session* s, Request* r, int status) {
    if (status == 0 && r->slot >= 0) {
        r->n_failed = (int64_t)s->host_fail[r->slot];
        float a = 0.f, b = 0.f;
        if (hipEventElapsedTime(&a, s->origin, s->ev_k0[r->slot]) == hipSuccess &&
            hipEventElapsedTime(&b, s->origin, s->ev_k1[r->slot]) == hipSuccess) {
            r->k_start_ms = a;
            r->k_end_ms = b;
        }
    }
    r->status = status;
    r->state = Q_DONE;
    r->t_done = now_ns();
    if (r->slot >= 0) {
        s->arena->release(r->off, r->bytes);
        s->free_slots.push_back(r->slot);
    }
    if (r->ready) s->free_ready.push_back(r->ready);
    r->ready = nullptr;
    r->slot = -1;
}

static void scheduler(rd_session* s) {
    hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    std::vector<Request*> admit;
    for (;;) {
        /* completions */
        for (size_t i = 0; i < s->running.size();) {
            Request* r = s->running[i];
            const hipError_t q = hipEventQuery(s->ev_done[r->slot]);
            if (q == hipErrorNotReady) { ++i; continue; }
            if (q != hipSuccess) req_error(r, "request failed on the device: %s", hipGetErrorString(q));
            complete(s, r, q == hipSuccess ? 0 : RD_EDEVICE);
            s->running[i] = s->running.back();
            s->running.pop_back();
            s->cv_done.notify_all();
        }
        /* admissions, in arrival order; later requests may pass a head that
         * does not fit yet unless the head has waited too long */
        const uint64_t t = now_ns();
        admit.clear();
        const int64_t batch = s->next_batch;
        for (auto it = s->queue.begin(); it != s->queue.end();) {
            Request* r = *it;
            if (s->free_slots.empty()) break;
            size_t off = 0;
            if (!s->arena->alloc(r->bytes, &off)) {
                ++r->deferred;
                if (it == s->queue.begin() && t - r->t_submit > kHeadWaitNs) break;
                ++it;
                continue;
            }
            r->off = off;
            r->slot = s->free_slots.back();
            s->free_slots.pop_back();
            r->stream = (int)(s->next_stream++ % s->streams.size());
            r->t_admit = now_ns();
            r->batch = batch;
            r->state = Q_RUNNING;
            admit.push_back(r);
            it = s->queue.erase(it);
        }
        if (!admit.empty()) {
            ++s->next_batch;
            lk.unlock();
            std::vector<char> ok(admit.size());
            for (size_t i = 0; i < admit.size(); ++i) {
                ok[i] = launch_request(s, admit[i]);
                /* part of a failed request may be queued: let it drain before
                 * its arena range can be handed to another request */
                if (!ok[i]) hipStreamSynchronize(s->streams[admit[i]->stream]);
            }
            lk.lock();
            for (size_t i = 0; i < admit.size(); ++i) {
                if (ok[i]) {
                    s->running.push_back(admit[i]);
                } else {
                    complete(s, admit[i], RD_EDEVICE);
                    s->cv_done.notify_all();
                }
            }
        }
        if (s->closing && s->queue.empty() && s->running.empty()) break;
        if (s->running.empty() && admit.empty()) {
            s->cv_work.wait(lk);
        } else {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        }
    }
}

static void fill_info(const Request& r, rd_request_info* info) {
    if (!info) return;
    std::memset(info, 0, sizeof(*info));
    info->done = r.state == Q_DONE;
    info->status = r.status;
    info->n_failed = r.n_failed;
    info->n_cells = r.pr.args.n;
    info->t_submit_ns = r.t_submit;
    info->t_admit_ns = r.t_admit;
    info->t_done_ns = r.t_done;
    info->batch_id = r.batch;
    info->kernel_start_ms = r.k_start_ms;
    info->kernel_end_ms = r.k_end_ms;
    info->stream = r.stream;
    info->deferred = r.deferred;
}

/* Result of a finished request for the caller: its status, and its error
 * message in the calling thread's last-error buffer. */
static int finished_status(const Request& r) {
    if (r.status < 0) set_error("%s", r.err[0] ? r.err : "request failed");
    return r.status < 0 ? r.status : 0;
}

}  // namespace rd

using namespace rd;

extern "C" {

size_t rd_request_bytes(int64_t n_cells, int32_t m, int32_t with_stats) {
    if (n_cells <= 0 || m <= 0) return 0;
    size_t b = align256((size_t)n_cells * m * sizeof(double));
    if (with_stats) b += align256((size_t)n_cells * RD_NSTATS * sizeof(int32_t));
    return b + order_bytes(n_cells);
}

/* Release what a partly created session holds (no worker thread yet). */
static void free_partial_session(rd_session* s) {
    for (hipStream_t st : s->streams) hipStreamDestroy(st);
    for (auto* v : {&s->ev_done, &s->ev_k0, &s->ev_k1})
        for (hipEvent_t ev : *v) hipEventDestroy(ev);
    if (s->origin) hipEventDestroy(s->origin);
    if (s->counters) hipFree(s->counters);
    if (s->host_fail) hipHostFree(s->host_fail);
    if (s->arena_base) hipFree(s->arena_base);
    delete s;
}

int32_t rd_session_create(rd_session** out, int32_t device, size_t hbm_budget_bytes,
                          const rd_options* defaults) {
    if (!out || hbm_budget_bytes < 256) { set_error("bad session arguments"); return RD_EINVAL; }
    if (defaults && defaults->h_cells) {
        set_error("per-cell warm-start arrays are not accepted by sessions");
        return RD_EINVAL;
    }
    if (defaults && (defaults->session_streams < 0 || defaults->session_streams > 64)) {
        set_error("session_streams must be in [0, 64]");
        return RD_EINVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        set_error("bad device %d", device);
        return RD_EINVAL;
    }
    if (hipSetDevice(device) != hipSuccess) { set_error("hipSetDevice failed"); return RD_EDEVICE; }
    auto* s = new rd_session();
    s->device = device;
    s->budget = hbm_budget_bytes;
    rd_default_options(&s->defaults);
    if (defaults) s->defaults = *defaults;
    if (hipMalloc((void**)&s->arena_base, hbm_budget_bytes) != hipSuccess) {
        set_error("hipMalloc(arena of %zu bytes) failed", hbm_budget_bytes);
        delete s;
        return RD_ENOMEM;
    }
    s->arena.reset(new Arena(hbm_budget_bytes));
    const int ns = s->defaults.session_streams > 0 ? s->defaults.session_streams : 4;
    for (int i = 0; i < ns; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            set_error("hipStreamCreate failed");
            free_partial_session(s);
            return RD_EDEVICE;
        }
        s->streams.push_back(st);
    }
    if (hipMalloc((void**)&s->counters, 2 * kSessionSlots * sizeof(unsigned long long)) != hipSuccess ||
        hipHostMalloc((void**)&s->host_fail, kSessionSlots * sizeof(unsigned long long), 0) != hipSuccess) {
        set_error("session workspace allocation failed");
        free_partial_session(s);
        return RD_ENOMEM;
    }
    for (int i = kSessionSlots - 1; i >= 0; --i) {
        s->free_slots.push_back(i);
        hipEvent_t a, b, c;
        if (hipEventCreateWithFlags(&a, hipEventDisableTiming) != hipSuccess) {
            set_error("hipEventCreate failed");
            free_partial_session(s);
            return RD_EDEVICE;
        }
        s->ev_done.push_back(a);
        if (hipEventCreate(&b) != hipSuccess) {
            set_error("hipEventCreate failed");
            free_partial_session(s);
            return RD_EDEVICE;
        }
        s->ev_k0.push_back(b);
        if (hipEventCreate(&c) != hipSuccess) {
            set_error("hipEventCreate failed");
            free_partial_session(s);
            return RD_EDEVICE;
        }
        s->ev_k1.push_back(c);
    }
    /* slot i uses entry i of the event vectors */
    std::reverse(s->ev_done.begin(), s->ev_done.end());
    std::reverse(s->ev_k0.begin(), s->ev_k0.end());
    std::reverse(s->ev_k1.begin(), s->ev_k1.end());
    if (hipEventCreate(&s->origin) != hipSuccess || hipEventRecord(s->origin, s->streams[0]) != hipSuccess ||
        hipEventSynchronize(s->origin) != hipSuccess) {
        set_error("session clock event failed");
        free_partial_session(s);
        return RD_EDEVICE;
    }
    s->worker = std::thread(scheduler, s);
    *out = s;
    return 0;
}

int32_t rd_submit_ex(rd_session* s, double* states, int64_t n_cells, int32_t m, double dt,
                     double rtol, double atol, const rd_model* model, int32_t* stats,
                     void* producer_stream, uint64_t* req_id) {
    if (!s || !req_id) { set_error("null session or req_id"); return RD_EINVAL; }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->closing) { set_error("session is closing"); return RD_ECLOSED; }
    }
    if (hipSetDevice(s->device) != hipSuccess) { set_error("hipSetDevice failed"); return RD_EDEVICE; }
    auto r = std::make_shared<Request>();
    int rc = prepare(states, n_cells, m, dt, rtol, atol, model, &s->defaults, stats, &r->pr);
    if (rc < 0) return rc;
    r->user_states = states;
    r->user_stats = stats;
    r->m = m;
    r->bytes = rd_request_bytes(n_cells, m, stats != nullptr);
    if (r->bytes > s->budget) {
        set_error("request of %zu bytes exceeds the session budget of %zu", r->bytes, s->budget);
        return RD_ETOOBIG;
    }
    if (n_cells > 0) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (!s->free_ready.empty()) {
                r->ready = s->free_ready.back();
                s->free_ready.pop_back();
            }
        }
        if (!r->ready && hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) != hipSuccess) {
            set_error("hipEventCreate failed");
            return RD_EDEVICE;
        }
        if (hipError_t e = hipEventRecord(r->ready, (hipStream_t)producer_stream); e != hipSuccess) {
            set_error("hipEventRecord on the producer stream: %s", hipGetErrorString(e));
            std::lock_guard<std::mutex> lk(s->mu);
            s->free_ready.push_back(r->ready);
            return RD_EDEVICE;
        }
    }
    r->t_submit = now_ns();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->closing) {
        /* destroyed meanwhile: the scheduler may have stopped */
        if (r->ready) s->free_ready.push_back(r->ready);
        set_error("session is closing");
        return RD_ECLOSED;
    }
    r->id = s->next_id++;
    *req_id = r->id;
    if (n_cells == 0) {
        r->state = Q_DONE;
        r->t_admit = r->t_done = r->t_submit;
        s->reqs.emplace(r->id, std::move(r));
        return 0;
    }
    s->queue.push_back(r.get());
    s->reqs.emplace(r->id, std::move(r));
    s->cv_work.notify_one();
    return 0;
}

int32_t rd_submit(rd_session* s, double* states, int64_t n_cells, int32_t m, double dt, double rtol,
                  double atol, const rd_model* model, int32_t* stats, uint64_t* req_id) {
    return rd_submit_ex(s, states, n_cells, m, dt, rtol, atol, model, stats, nullptr, req_id);
}

int32_t rd_poll(rd_session* s, uint64_t req_id, rd_request_info* info) {
    if (!s) { set_error("null session"); return RD_EINVAL; }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) { set_error("unknown request %llu", (unsigned long long)req_id); return RD_ENOTFOUND; }
    fill_info(*it->second, info);
    if (it->second->state != Q_DONE) return 1;
    const int st = finished_status(*it->second);
    s->reqs.erase(it);
    return st;
}

int32_t rd_wait(rd_session* s, uint64_t req_id, rd_request_info* info) {
    if (!s) { set_error("null session"); return RD_EINVAL; }
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) { set_error("unknown request %llu", (unsigned long long)req_id); return RD_ENOTFOUND; }
    /* shared ownership: a concurrent rd_poll / rd_wait on the same id may
     * remove the table entry while this thread waits */
    std::shared_ptr<Request> r = it->second;
    s->cv_done.wait(lk, [&] { return r->state == Q_DONE; });
    fill_info(*r, info);
    const int st = finished_status(*r);
    s->reqs.erase(req_id);
    return st;
}

int32_t rd_session_destroy(rd_session* s) {
    if (!s) { set_error("null session"); return RD_EINVAL; }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->closing = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (hipStream_t st : s->streams) {
        hipStreamSynchronize(st);
        hipStreamDestroy(st);
    }
    for (auto* v : {&s->ev_done, &s->ev_k0, &s->ev_k1, &s->free_ready})
        for (hipEvent_t ev : *v) hipEventDestroy(ev);
    hipEventDestroy(s->origin);
    hipFree(s->counters);
    hipHostFree(s->host_fail);
    hipFree(s->arena_base);
    delete s;
    return 0;
}

}  // extern "C"
