// Serving loop: continuous batching of minimum-spanning-forest requests
// under a device-memory budget.
//
// submit() copies a request into a pinned host staging buffer (reused from a
// pool, so the copy touches no fresh pages and the upload is a true
// asynchronous DMA) and queues it; a worker thread owns the device work:
//   - admission: waiting requests are admitted in arrival order while their
//     footprint (msf_request_footprint) fits in the budget left by the
//     requests in flight and the workspace the slots keep; an admitted
//     request gets a slot: its own stream, counters and stream-ordered
//     device workspace (kept from its previous request, grown if needed),
//     its inputs copied in, and its adjacency build enqueued;
//   - stepping: every pass over the active slots advances each slot whose
//     previous step has reached the host by one step (a round of Algorithm 2
//     with complete shortcutting, or the build/output stage), so rounds of
//     all requests in flight overlap on the device, and a request that
//     arrives mid-flight joins at the next pass;
//   - retirement: a finished slot's forest is copied back into the
//     request's staging buffer (asynchronously, polled like any step), its
//     latency is stamped (host steady clock, submit to ready), and its
//     budget is returned to waiting requests.  The slot keeps its workspace
//     for its next request (freeing and reallocating it per request cost
//     more than the solves: 4x the throughput and a tenth of the p99 at
//     four times the plain rate); idle slots give theirs back, largest
//     first, when a waiting request would not fit otherwise.
// Budget: used = the footprints of the requests in flight + the workspace
// every slot keeps, so the device memory of the slots never exceeds it
// (footprints bound what a request adds to a slot's workspace).
// A failing request completes with its error status and never affects the
// others.  Each request's result is bit-identical to msf_solve on it alone:
// every slot runs the same deterministic solve on its own state.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
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

// Pinned host buffers, reused across requests (pinning is slow, reuse is
// free).  A request's buffer holds its edges then its weights (12 bytes per
// edge) and later its forest ids (at most one per edge).
struct StagePool {
    std::mutex mu;
    std::multimap<size_t, void *> idle;  // capacity -> buffer
    // buffers pinned so far and the host time spent pinning them
    std::atomic<uint64_t> pinned{0}, pin_ns{0};
    void *get(size_t bytes, size_t *cap)
    {
        if (bytes < 4096) bytes = 4096;
        {
            std::lock_guard<std::mutex> lk(mu);
            auto it = idle.lower_bound(bytes);
            if (it != idle.end() && it->first <= 4 * bytes) {
                void *p = it->second;
                *cap = it->first;
                idle.erase(it);
                return p;
            }
        }
        // a power of two (at least 1 MB), so later requests of similar
        // size find it idle instead of pinning again
        size_t c = (size_t)1 << 20;
        while (c < bytes) c <<= 1;
        void *p = nullptr;
        const auto t0 = std::chrono::steady_clock::now();
        if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        pin_ns += (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
                      std::chrono::steady_clock::now() - t0)
                      .count();
        ++pinned;
        *cap = c;
        return p;
    }
    void put(void *p, size_t cap)
    {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu);
        idle.emplace(cap, p);
    }
    ~StagePool()
    {
        for (auto &kv : idle) (void)hipHostFree(kv.second);
    }
};

// memcpy split over a few threads for large requests.
void copy_in(void *dst, const void *src, size_t bytes)
{
    const size_t piece = (size_t)16 << 20;
    if (bytes <= 2 * piece) {
        std::memcpy(dst, src, bytes);
        return;
    }
    size_t nt = bytes / piece;
    if (nt > 8) nt = 8;
    const size_t chunk = (bytes + nt - 1) / nt;
    std::vector<std::thread> th;
    for (size_t t = 1; t < nt; ++t) {
        const size_t lo = t * chunk, hi = lo + chunk < bytes ? lo + chunk : bytes;
        if (lo >= hi) break;
        th.emplace_back([=] { std::memcpy((char *)dst + lo, (const char *)src + lo, hi - lo); });
    }
    std::memcpy(dst, src, chunk < bytes ? chunk : bytes);
    for (auto &x : th) x.join();
}

struct Request {
    uint64_t ticket = 0;
    int32_t n = 0;
    int64_t m = 0;
    msf_wtype wt = MSF_W_U32;
    void *stage = nullptr;  // pinned: edges, weights; then forest ids
    size_t stage_cap = 0;
    size_t footprint = 0;
    clk::time_point t_submit, t_done;
    // set last, with release order, once every other field is final; polls
    // read it without the server's main mutex
    std::atomic<bool> done{false};
    msf_status status = MSF_OK;
    std::string err;
    int64_t count = 0;
    msf_total total{0, 0.0};
};

struct ReqSlot {
    Ctx ctx;
    Request *req = nullptr;
    int32_t *d_ids = nullptr;
    bool downloading = false;
    size_t kept = 0;  // device workspace bytes it holds (counted in used)
};

}  // namespace

struct msf_server {
    int device = 0;
    size_t budget = 0;
    size_t used = 0;
    // requests in flight; 8 measured best on one MI355X for mixed graphs
    // (more slots only interleave large solves; MSF_SERVER_SLOTS overrides)
    size_t max_slots = 8;
    std::mutex mu;
    std::condition_variable cv_work;  // worker: new request or stop
    std::condition_variable cv_done;  // clients: a request finished
    std::deque<Request *> waiting;
    // ticket -> request; its own mutex, so client polls never contend with
    // the worker's admission and stepping
    std::mutex tmu;
    std::unordered_map<uint64_t, Request *> tickets;
    std::vector<ReqSlot *> active;   // worker-only
    std::vector<ReqSlot *> pool;     // worker-only: idle slots with streams
    std::thread worker;
    std::atomic<bool> stop{false};
    uint64_t next_ticket = 1;
    StagePool stage;
};

namespace {

void finish(msf_server *s, Request *r, msf_status st, const char *msg)
{
    std::lock_guard<std::mutex> lk(s->mu);
    r->status = st;
    if (msg) r->err = msg;
    r->t_done = clk::now();
    s->used -= r->footprint;
    r->done.store(true, std::memory_order_release);  // last touch of r here
    s->cv_done.notify_all();
}

// An idle slot for a request of `need` bytes: the one keeping the least
// workspace that is still at least need (it grows least and wastes least),
// else the one keeping the most; a new slot if none is idle.
ReqSlot *take_slot(msf_server *s, size_t need)
{
    if (!s->pool.empty()) {
        size_t best = s->pool.size();
        for (size_t i = 0; i < s->pool.size(); ++i) {
            const size_t k = s->pool[i]->kept;
            if (best == s->pool.size()) {
                best = i;
                continue;
            }
            const size_t b = s->pool[best]->kept;
            const bool fits = k >= need, bfits = b >= need;
            if ((fits && (!bfits || k < b)) || (!fits && !bfits && k > b)) best = i;
        }
        ReqSlot *sl = s->pool[best];
        s->pool[best] = s->pool.back();
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
    // the one-level build needs half the staging memory of the two-level
    // one, so more requests fit the budget at once; an explicit
    // MSF_BUCKETED_BUILD still wins
    if (!getenv("MSF_BUCKETED_BUILD") && sl->ctx.bucketed_build == 1) sl->ctx.bucketed_build = 2;
    // requests are budgeted without the head sweep's run arrays
    if (!getenv("MSF_HEADS")) sl->ctx.heads = 0;
    return sl;
}

size_t workspace_bytes(const Ctx &c)
{
    size_t t = 0;
    for (const auto &b : c.ws) t += b.cap;
    return t;
}

void retire_slot(msf_server *s, ReqSlot *sl)
{
    // the slot keeps its workspace; used follows what it now holds
    const size_t k = workspace_bytes(sl->ctx);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->used = s->used - sl->kept + k;
    }
    sl->kept = k;
    sl->req = nullptr;
    sl->d_ids = nullptr;
    sl->downloading = false;
    s->pool.push_back(sl);
}

// Copy a request in and enqueue its build.  On failure the request
// completes with the error; the slot goes back to the pool.
bool admit(msf_server *s, Request *r)
{
    ReqSlot *sl = take_slot(s, r->footprint);
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
        const char *st = (const char *)r->stage;
        if (hipMemcpyAsync(ve, st, 8 * (size_t)r->m, hipMemcpyHostToDevice, c->stream) !=
                hipSuccess ||
            hipMemcpyAsync(vw, st + 8 * (size_t)r->m, 4 * (size_t)r->m, hipMemcpyHostToDevice,
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
    if (sl->downloading) {  // forest ids are in the staging buffer
        finish(s, r, MSF_OK, nullptr);
        retire_slot(s, sl);
        return true;
    }
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
    r->count = cnt;
    r->total = tot;
    if (cnt > 0 &&
        (hipMemcpyAsync(r->stage, sl->d_ids, 4 * (size_t)cnt, hipMemcpyDeviceToHost,
                        c->stream) != hipSuccess ||
         hipEventRecord(c->ev[3], c->stream) != hipSuccess)) {
        (void)hipGetLastError();
        finish(s, r, MSF_EDEVICE, "result download failed");
        (void)hipStreamSynchronize(c->stream);
        retire_slot(s, sl);
        return true;
    }
    if (cnt == 0) {
        finish(s, r, MSF_OK, nullptr);
        retire_slot(s, sl);
        return true;
    }
    sl->downloading = true;
    return false;
}

void worker_main(msf_server *s)
{
    (void)hipSetDevice(s->device);
    for (;;) {
        // admission, in arrival order, while the budget allows; idle slots
        // give back their workspace (largest first) to make room
        for (;;) {
            Request *r = nullptr;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                if (s->waiting.empty() || s->active.size() >= s->max_slots) break;
                Request *f = s->waiting.front();
                while (s->used + f->footprint > s->budget) {
                    ReqSlot *big = nullptr;
                    for (ReqSlot *sl : s->pool)
                        if (sl->kept && (!big || sl->kept > big->kept)) big = sl;
                    if (!big) break;
                    ctx_release_workspace(&big->ctx);  // stream-ordered frees
                    s->used -= big->kept;
                    big->kept = 0;
                }
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
            r->done.store(true, std::memory_order_release);
        }
        s->waiting.clear();
        s->cv_work.notify_all();
        s->cv_done.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    if (getenv("MSF_SERVER_TRACE"))
        fprintf(stderr, "[msf server] pinned staging buffers: %llu, %.1f ms pinning\n",
                (unsigned long long)s->stage.pinned.load(), 1e-6 * (double)s->stage.pin_ns.load());
    {
        std::lock_guard<std::mutex> tl(s->tmu);
        for (auto &kv : s->tickets) {
            s->stage.put(kv.second->stage, kv.second->stage_cap);
            delete kv.second;
        }
    }
    delete s;
}

msf_status msf_server_submit(msf_server *s, int32_t n, int64_t m, const int32_t *edges,
                             const void *weights, msf_wtype wt, uint64_t *ticket)
{
    if (!s || !ticket || n < 0 || m < 0 || m > MSF_MAX_EDGES || (m > 0 && (!edges || !weights)) ||
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
    r->t_submit = clk::now();
    r->stage = s->stage.get(12 * (size_t)m, &r->stage_cap);
    if (!r->stage) {
        delete r;
        set_error("pinned host allocation failed");
        return MSF_ENOMEM;
    }
    if (m > 0) {
        copy_in(r->stage, edges, 8 * (size_t)m);
        copy_in((char *)r->stage + 8 * (size_t)m, weights, 4 * (size_t)m);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            s->stage.put(r->stage, r->stage_cap);
            delete r;
            set_error("server is stopping");
            return MSF_EINVAL;
        }
        r->ticket = s->next_ticket++;
        {
            std::lock_guard<std::mutex> tl(s->tmu);
            s->tickets[r->ticket] = r;
        }
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
    std::lock_guard<std::mutex> tl(s->tmu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) {
        set_error("unknown ticket %llu", (unsigned long long)ticket);
        return MSF_ENOTFOUND;
    }
    *done = it->second->done.load(std::memory_order_acquire) ? 1 : 0;
    return MSF_OK;
}

msf_status msf_server_latency(msf_server *s, uint64_t ticket, double *seconds)
{
    if (!s || !seconds) {
        set_error("bad arguments");
        return MSF_EINVAL;
    }
    std::lock_guard<std::mutex> tl(s->tmu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) {
        set_error("unknown ticket %llu", (unsigned long long)ticket);
        return MSF_ENOTFOUND;
    }
    if (!it->second->done.load(std::memory_order_acquire)) {
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
        std::lock_guard<std::mutex> tl(s->tmu);
        auto it = s->tickets.find(ticket);
        if (it == s->tickets.end()) {
            set_error("unknown ticket %llu", (unsigned long long)ticket);
            return MSF_ENOTFOUND;
        }
        r = it->second;
        s->tickets.erase(it);  // one result() per ticket: later calls miss
    }
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] { return r->done.load(std::memory_order_acquire); });
    }
    msf_status st = r->status;
    if (st == MSF_OK) {
        if (r->count > 0 && !forest_ids) {
            st = MSF_EINVAL;
            set_error("NULL forest_ids");
        } else {
            if (r->count > 0) copy_in(forest_ids, r->stage, 4 * (size_t)r->count);
            *forest_count = r->count;
            if (total) *total = r->total;
        }
    } else {
        set_error("%s", r->err.c_str());
    }
    s->stage.put(r->stage, r->stage_cap);
    delete r;
    return st;
}

}  // extern "C"
