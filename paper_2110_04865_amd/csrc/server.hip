// Serving loop: continuous batching of minimum-spanning-forest requests
// under a device-memory budget.
//
// submit() copies a request into host memory and queues it; a worker thread
// owns the device work:
//   - admission: waiting requests are admitted in arrival order while their
//     footprint (msf_request_footprint) fits in the budget left by the
//     requests in flight; an admitted request gets a slot: its own stream,
//     counters and stream-ordered device workspace, its inputs copied in,
//     and its adjacency build enqueued;
//   - stepping: every pass over the active slots advances each slot whose
//     previous step has reached the host by one step (a round of Algorithm 2
//     with complete shortcutting, or the build/output stage), so rounds of
//     all requests in flight overlap on the device, and a request that
//     arrives mid-flight joins at the next pass;
//   - retirement: a finished slot's forest is copied out, its latency is
//     stamped (host steady clock, submit to ready), its workspace is freed
//     on its stream, and its budget is returned to waiting requests.
// A failing request completes with its error status and never affects the
// others.  Each request's result is bit-identical to msf_solve on it alone:
// every slot runs the same deterministic solve on its own state.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "msf_internal.hpp"

using namespace msf;

namespace {

using clk = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    int32_t n = 0;
    int64_t m = 0;
    msf_wtype wt = MSF_W_U32;
    std::vector<int32_t> edges;
    std::vector<uint32_t> w;  // raw 32-bit weights
    size_t footprint = 0;
    clk::time_point t_submit, t_done;
    bool done = false;
    msf_status status = MSF_OK;
    std::string err;
    std::vector<int32_t> ids;
    int64_t count = 0;
    msf_total total{0, 0.0};
};

struct ReqSlot {
    Ctx ctx;
    Request *req = nullptr;
    int32_t *d_ids = nullptr;
};

}  // namespace

struct msf_server {
    int device = 0;
    size_t budget = 0;
    size_t used = 0;
    size_t max_slots = 64;
    std::mutex mu;
    std::condition_variable cv_work;  // worker: new request or stop
    std::condition_variable cv_done;  // clients: a request finished
    std::deque<Request *> waiting;
    std::unordered_map<uint64_t, Request *> tickets;
    std::vector<ReqSlot *> active;   // worker-only
    std::vector<ReqSlot *> pool;     // worker-only: idle slots with streams
    std::thread worker;
    std::atomic<bool> stop{false};
    uint64_t next_ticket = 1;
};

namespace {

void finish(msf_server *s, Request *r, msf_status st, const char *msg)
{
    std::lock_guard<std::mutex> lk(s->mu);
    r->status = st;
    if (msg) r->err = msg;
    r->t_done = clk::now();
    r->done = true;
    r->edges.clear();
    r->edges.shrink_to_fit();
    r->w.clear();
    r->w.shrink_to_fit();
    s->used -= r->footprint;
    s->cv_done.notify_all();
}

ReqSlot *take_slot(msf_server *s)
{
    if (!s->pool.empty()) {
        ReqSlot *sl = s->pool.back();
        s->pool.pop_back();
        return sl;
    }
    ReqSlot *sl = new (std::nothrow) ReqSlot();
    if (!sl) return nullptr;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        delete sl;
        return nullptr;
    }
    if (ctx_init(&sl->ctx, s->device, st, true) != MSF_OK) {
        ctx_release(&sl->ctx);
        (void)hipStreamDestroy(st);
        delete sl;
        return nullptr;
    }
    return sl;
}

void retire_slot(msf_server *s, ReqSlot *sl)
{
    ctx_release_workspace(&sl->ctx);  // stream-ordered frees
    sl->req = nullptr;
    sl->d_ids = nullptr;
    s->pool.push_back(sl);
}

// Copy a request in and enqueue its build.  On failure the request
// completes with the error; the slot goes back to the pool.
bool admit(msf_server *s, Request *r)
{
    ReqSlot *sl = take_slot(s);
    if (!sl) {
        finish(s, r, MSF_ENOMEM, "no slot (stream) available");
        return false;
    }
    Ctx *c = &sl->ctx;
    const size_t mm = (size_t)(r->m > 0 ? r->m : 1), nn = (size_t)(r->n > 0 ? r->n : 1);
    void *ve = nullptr, *vw = nullptr, *vi = nullptr;
    msf_status rc = ws_get(c, msf::WS_EDGES, 8 * mm, &ve);
    if (!rc) rc = ws_get(c, msf::WS_W, 4 * mm, &vw);
    if (!rc) rc = ws_get(c, msf::WS_IDS, 4 * nn, &vi);
    if (!rc && r->m > 0) {
        if (hipMemcpyAsync(ve, r->edges.data(), 8 * (size_t)r->m, hipMemcpyHostToDevice,
                           c->stream) != hipSuccess ||
            hipMemcpyAsync(vw, r->w.data(), 4 * (size_t)r->m, hipMemcpyHostToDevice,
                           c->stream) != hipSuccess) {
            (void)hipGetLastError();
            rc = MSF_EDEVICE;
            set_error("request upload failed");
        }
    }
    if (!rc) rc = solve_start(c, r->n, r->m, (const int32_t *)ve, vw, r->wt, (int32_t *)vi);
    if (rc) {
        finish(s, r, rc, msf_last_error());
        retire_slot(s, sl);
        return false;
    }
    sl->req = r;
    sl->d_ids = (int32_t *)vi;
    s->active.push_back(sl);
    return true;
}

// Advance a slot whose step has landed; returns true if it retired.
bool step_slot(msf_server *s, ReqSlot *sl)
{
    Ctx *c = &sl->ctx;
    Request *r = sl->req;
    msf_status rc = solve_advance(c);
    if (rc) {
        finish(s, r, rc, msf_last_error());
        (void)hipStreamSynchronize(c->stream);
        retire_slot(s, sl);
        return true;
    }
    if (!solve_done(c)) return false;
    int64_t cnt = 0;
    msf_total tot{0, 0.0};
    solve_result(c, &cnt, &tot);
    r->ids.resize((size_t)(cnt > 0 ? cnt : 0));
    if (cnt > 0 &&
        (hipMemcpyAsync(r->ids.data(), sl->d_ids, 4 * (size_t)cnt, hipMemcpyDeviceToHost,
                        c->stream) != hipSuccess ||
         hipStreamSynchronize(c->stream) != hipSuccess)) {
        (void)hipGetLastError();
        finish(s, r, MSF_EDEVICE, "result download failed");
        retire_slot(s, sl);
        return true;
    }
    r->count = cnt;
    r->total = tot;
    finish(s, r, MSF_OK, nullptr);
    retire_slot(s, sl);
    return true;
}

void worker_main(msf_server *s)
{
    (void)hipSetDevice(s->device);
    for (;;) {
        // admission, in arrival order, while the budget allows
        for (;;) {
            Request *r = nullptr;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                if (s->waiting.empty() || s->active.size() >= s->max_slots) break;
                Request *f = s->waiting.front();
                if (s->used + f->footprint > s->budget) break;
                s->waiting.pop_front();
                s->used += f->footprint;
                r = f;
            }
            admit(s, r);
        }
        // one pass over the slots in flight
        bool progressed = false;
        for (size_t i = 0; i < s->active.size();) {
            ReqSlot *sl = s->active[i];
            if (solve_ready(&sl->ctx)) {
                progressed = true;
                if (step_slot(s, sl)) {
                    s->active[i] = s->active.back();
                    s->active.pop_back();
                    continue;
                }
            }
            ++i;
        }
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop && s->active.empty() && s->waiting.empty()) break;
        if (!progressed) {
            if (s->active.empty())
                s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
            else
                s->cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
    for (ReqSlot *sl : s->pool) {
        hipStream_t st = sl->ctx.stream;
        ctx_release(&sl->ctx);
        (void)hipStreamDestroy(st);
        delete sl;
    }
    s->pool.clear();
}

}  // namespace

extern "C" {

msf_status msf_server_create(msf_ctx *ctx, size_t mem_budget_bytes, msf_server **out)
{
    if (!ctx || !out || mem_budget_bytes == 0) {
        set_error("bad arguments");
        return MSF_EINVAL;
    }
    msf_server *s = new (std::nothrow) msf_server();
    if (!s) {
        set_error("host allocation failed");
        return MSF_ENOMEM;
    }
    s->device = ctx->c.device;
    s->budget = mem_budget_bytes;
    if (const char *v = getenv("MSF_SERVER_SLOTS")) {
        const long k = atol(v);
        if (k > 0) s->max_slots = (size_t)k;
    }
    // keep freed slot memory in the device pool for the next admissions
    (void)hipSetDevice(s->device);
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, s->device) == hipSuccess) {
        uint64_t keep = ~0ull;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    (void)hipGetLastError();
    try {
        s->worker = std::thread(worker_main, s);
    } catch (...) {
        delete s;
        set_error("cannot start worker thread");
        return MSF_ENOMEM;
    }
    *out = s;
    return MSF_OK;
}

void msf_server_destroy(msf_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        // requests never admitted are dropped
        for (Request *r : s->waiting) {
            r->status = MSF_EINVAL;
            r->err = "server destroyed";
            r->done = true;
        }
        s->waiting.clear();
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (auto &kv : s->tickets) delete kv.second;
    delete s;
}

msf_status msf_server_submit(msf_server *s, int32_t n, int64_t m, const int32_t *edges,
                             const void *weights, msf_wtype wt, uint64_t *ticket)
{
    if (!s || !ticket || n < 0 || m < 0 || m > 0x7FFFFFFFll || (m > 0 && (!edges || !weights)) ||
        (wt != MSF_W_U32 && wt != MSF_W_F32)) {
        set_error("bad arguments");
        return MSF_EINVAL;
    }
    const size_t fp = msf_request_footprint(n, m);
    if (fp > s->budget) {
        set_error("request footprint %zu bytes exceeds the budget of %zu bytes", fp, s->budget);
        return MSF_EBUDGET;
    }
    Request *r = new (std::nothrow) Request();
    if (!r) {
        set_error("host allocation failed");
        return MSF_ENOMEM;
    }
    r->n = n;
    r->m = m;
    r->wt = wt;
    r->footprint = fp;
    try {
        r->edges.assign(edges, edges + 2 * (size_t)m);
        r->w.resize((size_t)m);
    } catch (...) {
        delete r;
        set_error("host allocation failed");
        return MSF_ENOMEM;
    }
    if (m > 0) std::memcpy(r->w.data(), weights, 4 * (size_t)m);
    r->t_submit = clk::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete r;
            set_error("server is stopping");
            return MSF_EINVAL;
        }
        r->ticket = s->next_ticket++;
        s->tickets[r->ticket] = r;
        s->waiting.push_back(r);
        s->cv_work.notify_all();
    }
    *ticket = r->ticket;
    return MSF_OK;
}

msf_status msf_server_poll(msf_server *s, uint64_t ticket, int *done)
{
    if (!s || !done) {
        set_error("bad arguments");
        return MSF_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) {
        set_error("unknown ticket %llu", (unsigned long long)ticket);
        return MSF_ENOTFOUND;
    }
    *done = it->second->done ? 1 : 0;
    return MSF_OK;
}

msf_status msf_server_latency(msf_server *s, uint64_t ticket, double *seconds)
{
    if (!s || !seconds) {
        set_error("bad arguments");
        return MSF_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) {
        set_error("unknown ticket %llu", (unsigned long long)ticket);
        return MSF_ENOTFOUND;
    }
    if (!it->second->done) {
        set_error("ticket %llu not finished", (unsigned long long)ticket);
        return MSF_EINVAL;
    }
    *seconds = std::chrono::duration<double>(it->second->t_done - it->second->t_submit).count();
    return MSF_OK;
}

msf_status msf_server_result(msf_server *s, uint64_t ticket, int32_t *forest_ids,
                             int64_t *forest_count, msf_total *total)
{
    if (!s || !forest_count) {
        set_error("bad arguments");
        return MSF_EINVAL;
    }
    Request *r = nullptr;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->tickets.find(ticket);
        if (it == s->tickets.end()) {
            set_error("unknown ticket %llu", (unsigned long long)ticket);
            return MSF_ENOTFOUND;
        }
        r = it->second;
        s->cv_done.wait(lk, [&] { return r->done; });
        s->tickets.erase(it);
    }
    msf_status st = r->status;
    if (st == MSF_OK) {
        if (r->count > 0 && !forest_ids) {
            st = MSF_EINVAL;
            set_error("NULL forest_ids");
        } else {
            if (r->count > 0) std::memcpy(forest_ids, r->ids.data(), 4 * (size_t)r->count);
            *forest_count = r->count;
            if (total) *total = r->total;
        }
    } else {
        set_error("%s", r->err.c_str());
    }
    delete r;
    return st;
}

}  // extern "C"
