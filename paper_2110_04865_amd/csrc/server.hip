// Serving loop: continuous batching of minimum-spanning-forest requests
// under a device-memory budget.
//
// submit() copies a request into a pinned host staging buffer (reused from a
// pool, so the copy touches no fresh pages and the upload is a true
// asynchronous DMA) and queues it; a worker thread owns the device work:
//   - shared launches: the waiting requests whose state fits one
//     workgroup's LDS (at most 2^17 edges) are taken together, while the
//     budget allows, into one launch of the persistent kernel (each request
//     one graph of the batch); two such jobs alternate, so requests that
//     arrive while one runs go into the next;
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
#include "persist.hpp"

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

// Small requests (state that fits one workgroup's LDS) admitted together
// are solved by one launch of the persistent kernel: their inputs are
// copied into one concatenated buffer, each becomes one graph of the batch,
// and their forests go back to their staging buffers.  Step 1 waits for the
// solve and the counts, step 2 for the forest ids.
struct BatchJob {
    Ctx ctx;
    std::vector<Request *> reqs;
    int step = 0;          // 0 idle, 1 solving, 2 downloading ids
    size_t kept = 0;       // device workspace bytes it holds (counted in used)
    int64_t *hres = nullptr;  // pinned: offsets (2 (G+1)), then counts, u64 and f64 totals
    uint32_t *hctl = nullptr; // pinned: error word
    size_t hcap = 0;          // graphs hres has room for
};

// Most graphs one shared launch takes.
constexpr size_t BATCH_MAX_GRAPHS = 1024;

bool small_request(int32_t n, int64_t m)
{
    return m > 0 && n > 0 && (uint32_t)n <= PERSIST_MAX_N && m <= ((int64_t)1 << 17) &&
           persist_state_bytes((uint32_t)n, (uint32_t)m) <= SMALL_LDS;
}

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
    BatchJob *jobs[2] = {nullptr, nullptr};  // worker-only: shared launches
    bool batch_small = true;         // MSF_SERVER_BATCH=0 sends every request to a slot
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

BatchJob *job_new(msf_server *s)
{
    BatchJob *j = new (std::nothrow) BatchJob();
    if (!j) return nullptr;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        delete j;
        return nullptr;
    }
    if (ctx_init(&j->ctx, s->device, st, true) != MSF_OK) {
        ctx_release(&j->ctx);
        (void)hipStreamDestroy(st);
        delete j;
        return nullptr;
    }
    return j;
}

void job_free(BatchJob *j)
{
    hipStream_t st = j->ctx.stream;
    ctx_release(&j->ctx);
    (void)hipStreamDestroy(st);
    if (j->hres) (void)hipHostFree(j->hres);
    delete j;
}

void job_fail(msf_server *s, BatchJob *j, msf_status st, const char *msg)
{
    for (Request *r : j->reqs) finish(s, r, st, msg);
    j->reqs.clear();
    (void)hipStreamSynchronize(j->ctx.stream);
    j->step = 0;
}

// Pinned host arrays of a job for G graphs: offsets (2 (G + 1) int64), the
// results (counts, u64 totals, f64 totals: 3 G), the order (G u32) and the
// error word.
bool job_host(BatchJob *j, size_t G)
{
    if (j->hcap >= G) return true;
    if (j->hres) (void)hipHostFree(j->hres);
    j->hres = nullptr;
    j->hcap = 0;
    const size_t bytes = 8 * (2 * (G + 1) + 3 * G) + 4 * G + 64;
    if (hipHostMalloc((void **)&j->hres, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        j->hres = nullptr;
        return false;
    }
    j->hcap = G;
    return true;
}

// Copy the requests in and enqueue one persistent launch over all of them.
void job_start(msf_server *s, BatchJob *j, std::vector<Request *> &&reqs)
{
    Ctx *c = &j->ctx;
    hipStream_t st = c->stream;
    j->reqs = std::move(reqs);
    const size_t G = j->reqs.size();
    const msf_wtype wt = j->reqs[0]->wt;
    if (!job_host(j, G)) {
        job_fail(s, j, MSF_ENOMEM, "pinned host allocation failed");
        return;
    }
    int64_t *vo = j->hres, *eo = vo + (G + 1), *res = eo + (G + 1);
    uint32_t *order = (uint32_t *)(res + 3 * G);
    j->hctl = order + G;
    vo[0] = eo[0] = 0;
    uint32_t nmax = 1, mmax = 1;
    for (size_t g = 0; g < G; ++g) {
        const Request *r = j->reqs[g];
        vo[g + 1] = vo[g] + r->n;
        eo[g + 1] = eo[g] + r->m;
        nmax = std::max(nmax, (uint32_t)r->n);
        mmax = std::max(mmax, (uint32_t)r->m);
        order[g] = (uint32_t)g;
    }
    std::stable_sort(order, order + G, [&](uint32_t x, uint32_t y) {
        return j->reqs[x]->m > j->reqs[y]->m;
    });
    const size_t N = (size_t)vo[G], M = (size_t)eo[G];
    int cus = 1;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device);
    const PersistCfg cfg{1024, 4, SMALL_LDS};
    const int bpc = std::max(1, persist_blocks_per_cu(cfg, (int)wt));
    const size_t slots = std::min<size_t>(G, (size_t)cus * bpc);
    const size_t slot_bytes = persist_slot_bytes(nmax, mmax);
    void *ve, *vw, *voff, *vids, *vres, *vord, *vctl, *vscr;
    msf_status rc = ws_get(c, WS_EDGES, 8 * M, &ve);
    if (!rc) rc = ws_get(c, WS_W, 4 * M, &vw);
    if (!rc) rc = ws_get(c, WS_BATCH0, 16 * (G + 1), &voff);
    if (!rc) rc = ws_get(c, WS_IDS, 4 * std::max<size_t>(N, 1), &vids);
    if (!rc) rc = ws_get(c, WS_BATCH3, 24 * G, &vres);
    if (!rc) rc = ws_get(c, WS_PORDER, 4 * G, &vord);
    if (!rc) rc = ws_get(c, WS_PCTL, 256, &vctl);
    if (!rc) rc = ws_get(c, WS_PSCRATCH, slots * slot_bytes, &vscr);
    if (rc) {
        job_fail(s, j, rc, msf_last_error());
        return;
    }
    bool ok = hipMemcpyAsync(voff, vo, 16 * (G + 1), hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(vord, order, 4 * G, hipMemcpyHostToDevice, st) == hipSuccess;
    for (size_t g = 0; ok && g < G; ++g) {
        const Request *r = j->reqs[g];
        const char *stg = (const char *)r->stage;
        ok = hipMemcpyAsync((int32_t *)ve + 2 * eo[g], stg, 8 * (size_t)r->m,
                            hipMemcpyHostToDevice, st) == hipSuccess &&
             hipMemcpyAsync((uint32_t *)vw + eo[g], stg + 8 * (size_t)r->m, 4 * (size_t)r->m,
                            hipMemcpyHostToDevice, st) == hipSuccess;
    }
    PersistArgs A;
    A.G = (int32_t)G;
    A.order = (const uint32_t *)vord;
    A.queue = (uint32_t *)vctl;
    A.err = (uint32_t *)vctl + 1;
    A.vtx_off = (const int64_t *)voff;
    A.edge_off = (const int64_t *)voff + (G + 1);
    A.edges = (const int32_t *)ve;
    A.w = (const uint32_t *)vw;
    A.out = (int32_t *)vids;
    A.counts = (int64_t *)vres;
    A.tot_u64 = (uint64_t *)vres + G;
    A.tot_f64 = (double *)vres + 2 * G;
    A.scratch = (uint8_t *)vscr;
    A.slot_bytes = slot_bytes;
    A.m_cap = mmax;
    A.lds_bytes = cfg.lds;
    ok = ok && launch_persist(st, A, cfg, (int)wt, (unsigned)slots) == hipSuccess &&
         hipMemcpyAsync(res, vres, 24 * G, hipMemcpyDeviceToHost, st) == hipSuccess &&
         hipEventRecord(c->ev[3], st) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        job_fail(s, j, MSF_EDEVICE, "shared launch failed");
        return;
    }
    j->step = 1;
}

const char *err_text(int64_t flags)
{
    if (flags & ERR_ENDPOINT) return "edge endpoint outside [0, n)";
    if (flags & ERR_NAN) return "NaN edge weight";
    return "internal error in the batched solve";
}

// Advance a job whose step has landed; returns true when it is idle again.
bool job_step(msf_server *s, BatchJob *j)
{
    Ctx *c = &j->ctx;
    hipStream_t st = c->stream;
    const size_t G = j->reqs.size();
    int64_t *vo = j->hres, *res = vo + 2 * (G + 1);
    if (j->step == 1) {
        // counts and totals are here: fetch each forest into its staging
        void *vids = c->ws[WS_IDS].ptr;
        bool ok = true;
        for (size_t g = 0; g < G && ok; ++g) {
            Request *r = j->reqs[g];
            const int64_t cnt = res[g];
            if (cnt > 0)
                ok = hipMemcpyAsync(r->stage, (const int32_t *)vids + vo[g], 4 * (size_t)cnt,
                                    hipMemcpyDeviceToHost, st) == hipSuccess;
        }
        if (!ok || hipEventRecord(c->ev[3], st) != hipSuccess) {
            (void)hipGetLastError();
            job_fail(s, j, MSF_EDEVICE, "result download failed");
            return true;
        }
        j->step = 2;
        return false;
    }
    for (size_t g = 0; g < G; ++g) {
        Request *r = j->reqs[g];
        const int64_t cnt = res[g];
        if (cnt < 0) {
            finish(s, r, MSF_EINVAL, err_text(-cnt));
            continue;
        }
        r->count = cnt;
        r->total.u64 = (uint64_t)res[G + g];
        std::memcpy(&r->total.f64, &res[2 * G + g], sizeof(double));
        finish(s, r, MSF_OK, nullptr);
    }
    j->reqs.clear();
    j->step = 0;
    const size_t k = workspace_bytes(j->ctx);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->used = s->used - j->kept + k;
    }
    j->kept = k;
    return true;
}

// Gives back the workspace of idle slots and jobs, largest first, until
// `need` more bytes fit the budget (called with s->mu held).
bool make_room(msf_server *s, size_t need)
{
    while (s->used + need > s->budget) {
        ReqSlot *big = nullptr;
        for (ReqSlot *sl : s->pool)
            if (sl->kept && (!big || sl->kept > big->kept)) big = sl;
        BatchJob *bj = nullptr;
        for (BatchJob *j : s->jobs)
            if (j && j->step == 0 && j->kept && (!bj || j->kept > bj->kept)) bj = j;
        if (bj && (!big || bj->kept > big->kept)) {
            ctx_release_workspace(&bj->ctx);
            s->used -= bj->kept;
            bj->kept = 0;
            continue;
        }
        if (!big) return false;
        ctx_release_workspace(&big->ctx);  // stream-ordered frees
        s->used -= big->kept;
        big->kept = 0;
    }
    return true;
}

void worker_main(msf_server *s)
{
    (void)hipSetDevice(s->device);
    for (;;) {
        // small requests: one shared launch of the persistent kernel for
        // all waiting ones (same weight type), when a job is idle
        if (s->batch_small) {
            BatchJob *j = nullptr;
            for (BatchJob *&x : s->jobs) {
                if (!x) x = job_new(s);
                if (x && x->step == 0) {
                    j = x;
                    break;
                }
            }
            // no job could be set up: every request goes to a slot
            if (!s->jobs[0] && !s->jobs[1]) s->batch_small = false;
            if (j) {
                std::vector<Request *> take;
                {
                    std::lock_guard<std::mutex> lk(s->mu);
                    for (auto it = s->waiting.begin();
                         it != s->waiting.end() && take.size() < BATCH_MAX_GRAPHS;) {
                        Request *r = *it;
                        if (!small_request(r->n, r->m) || (!take.empty() && r->wt != take[0]->wt)) {
                            ++it;
                            continue;
                        }
                        if (!make_room(s, r->footprint)) break;
                        s->used += r->footprint;
                        take.push_back(r);
                        it = s->waiting.erase(it);
                    }
                }
                if (!take.empty()) job_start(s, j, std::move(take));
            }
        }
        // the others (all of them with batching off): one slot each, in
        // arrival order, while the budget allows
        for (;;) {
            Request *r = nullptr;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                if (s->active.size() >= s->max_slots) break;
                auto it = s->waiting.begin();
                while (it != s->waiting.end() && s->batch_small && small_request((*it)->n, (*it)->m))
                    ++it;
                if (it == s->waiting.end()) break;
                Request *f = *it;
                if (!make_room(s, f->footprint)) break;
                s->waiting.erase(it);
                s->used += f->footprint;
                r = f;
            }
            admit(s, r);
        }
        // one pass over the slots and jobs in flight
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
        bool jobs_busy = false;
        for (BatchJob *j : s->jobs) {
            if (!j || j->step == 0) continue;
            if (hipEventQuery(j->ctx.ev[3]) == hipSuccess) {
                progressed = true;
                job_step(s, j);
            }
            jobs_busy |= j->step != 0;
        }
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop && s->active.empty() && s->waiting.empty() && !jobs_busy) break;
        if (!progressed) {
            if (s->active.empty() && !jobs_busy)
                s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
            else {
                // work in flight: poll again soon (a step is tens of us)
                lk.unlock();
                std::this_thread::yield();
            }
        }
    }
    for (ReqSlot *sl : s->pool) {
        hipStream_t st = sl->ctx.stream;
        ctx_release(&sl->ctx);
        (void)hipStreamDestroy(st);
        delete sl;
    }
    s->pool.clear();
    for (BatchJob *&j : s->jobs) {
        if (j) job_free(j);
        j = nullptr;
    }
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
    if (const char *v = getenv("MSF_SERVER_BATCH")) s->batch_small = atoi(v) != 0;
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
