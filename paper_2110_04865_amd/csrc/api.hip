// C ABI of the library (include/msf.h): contexts, workspace, the solve
// driver (round loop of Algorithm 2 with complete shortcutting), the
// adjacency handle, and the standalone multilinear and shortcut calls.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <new>

#include "msf_internal.hpp"
#include "persist.hpp"

namespace msf {

static thread_local std::string g_err;

void set_error(const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

msf_status hip_fail(hipError_t e, const char *what)
{
    set_error("HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
    return (e == hipErrorOutOfMemory) ? MSF_ENOMEM : MSF_EDEVICE;
}

msf_status ws_get(Ctx *c, Slot s, size_t bytes, void **out)
{
    DevBuf &b = c->ws[s];
    if (bytes == 0) bytes = 256;
    if (b.cap < bytes) {
        if (b.ptr) {
            if (c->async_alloc) {
                MSF_HIP(hipFreeAsync(b.ptr, c->stream));
            } else {
                MSF_HIP(hipStreamSynchronize(c->stream));
                MSF_HIP(hipFree(b.ptr));
            }
            b.ptr = nullptr;
            b.cap = 0;
        }
        const size_t gran = c->async_alloc ? ((size_t)1 << 16) : ((size_t)1 << 20);
        size_t cap = (bytes + gran - 1) & ~(gran - 1);
        if (c->fail_alloc_after == 0) {
            // the test hook: this allocation fails as a real one would
            c->fail_alloc_after = -1;
            set_error("device allocation of %zu bytes refused (MSF_TEST_FAIL_ALLOC_AFTER)", cap);
            return MSF_ENOMEM;
        }
        if (c->fail_alloc_after > 0) --c->fail_alloc_after;
        hipError_t e = c->async_alloc ? hipMallocAsync(&b.ptr, cap, c->stream)
                                      : hipMalloc(&b.ptr, cap);
        if (e != hipSuccess) {
            b.ptr = nullptr;
            (void)hipGetLastError();
            set_error("device allocation of %zu bytes failed", cap);
            return MSF_ENOMEM;
        }
        b.cap = cap;
    }
    *out = b.ptr;
    return MSF_OK;
}

msf_status read_counters(Ctx *c)
{
    MSF_HIP(hipMemcpyAsync(c->hcnt, c->dcnt, sizeof(Counters), hipMemcpyDeviceToHost, c->stream));
    MSF_HIP(hipStreamSynchronize(c->stream));
    return MSF_OK;
}

void zero_counters(Ctx *c)
{
    launch_fill_u32(c->stream, reinterpret_cast<uint32_t *>(c->dcnt), 0u,
                    sizeof(Counters) / sizeof(uint32_t));
}

// The error word and the device-driven rounds' termination flag (which
// the sweep and the chase fold test at entry), before a call that runs
// those kernels outside a solve.
static void clear_err_done(Ctx *c)
{
    launch_fill_u32(c->stream, &c->dcnt->err, 0u, 1);
    launch_fill_u32(c->stream, &c->dcnt->gdone, 0u, 1);
}

msf_status decode_err(uint32_t err)
{
    if (err & ERR_ENDPOINT) {
        set_error("edge endpoint outside [0, n)");
        return MSF_EINVAL;
    }
    if (err & ERR_NAN) {
        set_error("NaN edge weight");
        return MSF_EINVAL;
    }
    if (err & ERR_PARENT) {
        set_error("parent entry outside [0, n)");
        return MSF_EINVAL;
    }
    if (err & ERR_CYCLE) {
        set_error("parent vector is not a rooted forest (cycle)");
        return MSF_EINVAL;
    }
    return MSF_OK;
}

}  // namespace msf

using namespace msf;

// ------------------------------------------------------------------ ABI --

extern "C" {

const char *msf_last_error(void) { return g_err.c_str(); }

const char *msf_version(void) { return "msf-gfx950 0.1"; }

}  // extern "C"

namespace msf {

msf_status ctx_init(Ctx *c, int device, hipStream_t stream, bool async_alloc)
{
    c->device = device;
    c->stream = stream;
    c->async_alloc = async_alloc;
    MSF_TRY(noalloc_init(device));
    if (hipMalloc(&c->dcnt, sizeof(Counters)) != hipSuccess ||
        hipHostMalloc(&c->hcnt, sizeof(Counters), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        set_error("counter allocation failed");
        return MSF_ENOMEM;
    }
    for (auto &ev : c->sev)
        if (hipEventCreate(&ev) != hipSuccess) {
            set_error("event creation failed");
            return MSF_EDEVICE;
        }
    for (auto &ev : c->ev)
        if (hipEventCreate(&ev) != hipSuccess) {
            set_error("event creation failed");
            return MSF_EDEVICE;
        }
    for (auto &ev : c->kev)
        if (hipEventCreate(&ev) != hipSuccess) {
            set_error("event creation failed");
            return MSF_EDEVICE;
        }
    if (const char *f = getenv("MSF_FILTER")) c->filter_mode = atoi(f);
    if (const char *f = getenv("MSF_FILTER_THRESHOLD")) c->filter_threshold = atof(f);
    if (const char *f = getenv("MSF_CHECK_ROUNDS")) c->check_rounds = atoi(f) != 0;
    if (const char *f = getenv("MSF_FIRST_ROUND")) c->first_round = atoi(f);
    if (const char *f = getenv("MSF_BUCKETED_BUILD")) c->bucketed_build = atoi(f);
    if (const char *f = getenv("MSF_SLICES")) c->slices = atoi(f);
    if (const char *f = getenv("MSF_HEADS")) c->heads = atoi(f);
    if (const char *f = getenv("MSF_BATCH_MODE")) c->batch_mode = atoi(f);
    if (const char *f = getenv("MSF_SMALL_M")) c->small_m = atoll(f);
    if (const char *f = getenv("MSF_GRAPH_ORDER")) c->graph_order = atoi(f);
    if (const char *f = getenv("MSF_GRAPH_ROUNDS")) c->graph_rounds = atoi(f);
    if (const char *f = getenv("MSF_GRAPH_ROUNDS_MAX_N")) c->graph_rounds_max_n = atoll(f);
    if (const char *f = getenv("MSF_TL_ROW_IN_COL")) c->tl_row_in_col = atoi(f);
    if (const char *f = getenv("MSF_TEST_FAIL_ALLOC_AFTER")) c->fail_alloc_after = atoll(f);
    return MSF_OK;
}

void ctx_release_workspace(Ctx *c)
{
    for (auto &b : c->ws) {
        if (!b.ptr) continue;
        if (c->async_alloc) (void)hipFreeAsync(b.ptr, c->stream);
        else (void)hipFree(b.ptr);
        b.ptr = nullptr;
        b.cap = 0;
    }
}

void ctx_release(Ctx *c)
{
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec), c->gexec = nullptr;
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream), c->cap_stream = nullptr;
    ctx_release_workspace(c);
    (void)hipStreamSynchronize(c->stream);
    for (auto &ev : c->ev)
        if (ev) (void)hipEventDestroy(ev), ev = nullptr;
    for (auto &ev : c->sev)
        if (ev) (void)hipEventDestroy(ev), ev = nullptr;
    for (auto &ev : c->kev)
        if (ev) (void)hipEventDestroy(ev), ev = nullptr;
    if (c->dcnt) (void)hipFree(c->dcnt), c->dcnt = nullptr;
    if (c->hcnt) (void)hipHostFree(c->hcnt), c->hcnt = nullptr;
}

}  // namespace msf

extern "C" {

msf_status msf_ctx_create(int device, void *hip_stream, msf_ctx **out)
{
    if (!out) {
        set_error("out is NULL");
        return MSF_EINVAL;
    }
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) {
        set_error("no HIP device available");
        return MSF_EDEVICE;
    }
    if (device < 0 || device >= ndev) {
        set_error("device %d out of range (%d devices)", device, ndev);
        return MSF_EINVAL;
    }
    MSF_HIP(hipSetDevice(device));
    msf_ctx *x = new (std::nothrow) msf_ctx();
    if (!x) {
        set_error("host allocation failed");
        return MSF_ENOMEM;
    }
    msf_status rc = ctx_init(&x->c, device, (hipStream_t)hip_stream, false);
    if (rc) {
        msf_ctx_destroy(x);
        return rc;
    }
    *out = x;
    return MSF_OK;
}

void msf_ctx_destroy(msf_ctx *x)
{
    if (!x) return;
    ctx_release(&x->c);
    delete x;
}

static msf_status check_graph_args(msf_ctx *ctx, int32_t n, int64_t m, const int32_t *edges,
                                   const void *weights, msf_wtype wt, msf_mem mem)
{
    if (!ctx) {
        set_error("ctx is NULL");
        return MSF_EINVAL;
    }
    if (n < 0 || m < 0 || m > MSF_MAX_EDGES) {
        set_error("bad sizes n=%d m=%lld", (int)n, (long long)m);
        return MSF_EINVAL;
    }
    if (m > 0 && (!edges || !weights)) {
        set_error("NULL edges/weights with m > 0");
        return MSF_EINVAL;
    }
    if (wt != MSF_W_U32 && wt != MSF_W_F32) {
        set_error("bad weight type");
        return MSF_EINVAL;
    }
    if (mem != MSF_MEM_HOST && mem != MSF_MEM_DEVICE) {
        set_error("bad memory kind");
        return MSF_EINVAL;
    }
    return MSF_OK;
}

msf_status msf_solve(msf_ctx *ctx, int32_t n, int64_t m, const int32_t *edges, const void *weights,
                     msf_wtype wt, msf_mem mem, int32_t *forest_ids, int64_t *forest_count,
                     msf_total *total)
{
    msf_status rc = check_graph_args(ctx, n, m, edges, weights, wt, mem);
    if (rc) return rc;
    if (!forest_count || (n > 1 && m > 0 && !forest_ids)) {
        set_error("NULL output");
        return MSF_EINVAL;
    }
    Ctx *c = &ctx->c;
    MSF_HIP(hipSetDevice(c->device));
    const int32_t *d_edges = edges;
    const void *d_w = weights;
    int32_t *d_ids = forest_ids;
    if (mem == MSF_MEM_HOST) {
        void *ve, *vw, *vi;
        if ((rc = ws_get(c, WS_EDGES, 8 * (size_t)std::max<int64_t>(m, 1), &ve))) return rc;
        if ((rc = ws_get(c, WS_W, 4 * (size_t)std::max<int64_t>(m, 1), &vw))) return rc;
        if ((rc = ws_get(c, WS_IDS, 4 * (size_t)std::max(n, 1), &vi))) return rc;
        if (m > 0) {
            MSF_HIP(hipMemcpyAsync(ve, edges, 8 * (size_t)m, hipMemcpyHostToDevice, c->stream));
            MSF_HIP(hipMemcpyAsync(vw, weights, 4 * (size_t)m, hipMemcpyHostToDevice, c->stream));
        }
        d_edges = (const int32_t *)ve;
        d_w = vw;
        d_ids = (int32_t *)vi;
    }
    int64_t cnt = 0;
    msf_total tot{0, 0.0};
    rc = small_eligible(c, n, m) ? solve_small(c, n, m, d_edges, d_w, wt, d_ids, &cnt, &tot)
                                 : solve_device(c, n, m, d_edges, d_w, wt, d_ids, &cnt, &tot);
    if (rc) return rc;
    if (mem == MSF_MEM_HOST && cnt > 0) {
        MSF_HIP(hipMemcpyAsync(forest_ids, d_ids, 4 * (size_t)cnt, hipMemcpyDeviceToHost,
                               c->stream));
        MSF_HIP(hipStreamSynchronize(c->stream));
    }
    *forest_count = cnt;
    if (total) *total = tot;
    return MSF_OK;
}

msf_status msf_get_stats(const msf_ctx *ctx, msf_stats *out)
{
    if (!ctx || !out) {
        set_error("NULL argument");
        return MSF_EINVAL;
    }
    Ctx *c = const_cast<Ctx *>(&ctx->c);
    if (c->ml_pending) {
        // the sweep of the last msf_multilinear: wait for its end event
        MSF_HIP(hipSetDevice(c->device));
        MSF_HIP(hipEventSynchronize(c->sev[1]));
        float ms = 0.f, gms = 0.f;
        MSF_HIP(hipEventElapsedTime(&ms, c->sev[0], c->sev[1]));
        MSF_HIP(hipEventElapsedTime(&gms, c->kev[0], c->sev[0]));
        c->stats.sweep_ms[0] = ms;
        c->stats.pass_ms[0] = c->stats.pass_bytes[0] > 0 ? gms : 0.0;
        c->ml_pending = false;
    }
    *out = c->stats;
    return MSF_OK;
}

// ---------------------------------------------------------------- graph --

msf_status msf_graph_create(msf_ctx *ctx, int32_t n, int64_t m, const int32_t *edges,
                            const void *weights, msf_wtype wt, msf_mem mem, msf_graph **out)
{
    msf_status rc = check_graph_args(ctx, n, m, edges, weights, wt, mem);
    if (rc) return rc;
    if (!out) {
        set_error("out is NULL");
        return MSF_EINVAL;
    }
    Ctx *c = &ctx->c;
    MSF_HIP(hipSetDevice(c->device));
    msf_graph *g = new (std::nothrow) msf_graph();
    if (!g) {
        set_error("host allocation failed");
        return MSF_ENOMEM;
    }
    g->ctx = ctx;
    const size_t nn = (size_t)std::max(n, 1), mm = (size_t)std::max<int64_t>(m, 1);
    const size_t nch =
        sweep_nchunks((uint32_t)std::min<size_t>(2 * mm, 0xFFFFFFFFull)) + 2 * MAX_SLICES + 2;
    const int slices = choose_slices(n, m, c->slices);
    const size_t sizes[6] = {8 * mm, 4 * mm, 4 * (size_t)slices * (nn + 1),
                             4 * (2 * mm + SWEEP_PAD), 8 * (2 * mm + SWEEP_PAD), 4 * nch};
    for (int i = 0; i < 6; ++i) {
        if (hipMalloc(&g->bufs[i], sizes[i]) != hipSuccess) {
            (void)hipGetLastError();
            msf_graph_destroy(g);
            set_error("device allocation failed");
            return MSF_ENOMEM;
        }
    }
    const hipMemcpyKind kind = mem == MSF_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    if (m > 0) {
        hipError_t e1 = hipMemcpyAsync(g->bufs[0], edges, 8 * (size_t)m, kind, c->stream);
        hipError_t e2 = hipMemcpyAsync(g->bufs[1], weights, 4 * (size_t)m, kind, c->stream);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            msf_graph_destroy(g);
            return hip_fail(e1 != hipSuccess ? e1 : e2, "hipMemcpyAsync");
        }
    }
    // the degree order (one slice): built in the caller's order into the
    // workspace, then renumbered into the graph's buffers
    const bool order = c->graph_order != 0 && n > 0 && m > 0 && slices == 1;
    void *vrp0 = nullptr, *vcol0 = nullptr, *vkey0 = nullptr, *vcrow0 = nullptr;
    if (order && ((rc = ws_get(c, WS_ROWPTR, 4 * (nn + 1), &vrp0)) ||
                  (rc = ws_get(c, WS_COL, sizes[3], &vcol0)) ||
                  (rc = ws_get(c, WS_KEY, sizes[4], &vkey0)) ||
                  (rc = ws_get(c, WS_CHUNKROW, sizes[5], &vcrow0)))) {
        msf_graph_destroy(g);
        return rc;
    }
    zero_counters(c);
    if (order)
        rc = build_adjacency(c, n, m, (const int32_t *)g->bufs[0], g->bufs[1], wt, 1, &g->a,
                             (uint32_t *)vrp0, (uint32_t *)vcol0, (uint64_t *)vkey0,
                             (uint32_t *)vcrow0);
    else
        rc = build_adjacency(c, n, m, (const int32_t *)g->bufs[0], g->bufs[1], wt, slices, &g->a,
                             (uint32_t *)g->bufs[2], (uint32_t *)g->bufs[3],
                             (uint64_t *)g->bufs[4], (uint32_t *)g->bufs[5]);
    if (rc == MSF_OK) rc = read_counters(c);
    if (rc == MSF_OK) rc = decode_err(c->hcnt->err);
    if (rc) {
        msf_graph_destroy(g);
        return rc;
    }
    if (order) {
        void *vdeg, *vtab, *vinv, *vseg, *vsr;
        const int64_t nnz = (int64_t)c->hcnt->sstart[1] - (int64_t)c->hcnt->sstart[0];
        if (hipMalloc(&g->perm, 4 * nn) != hipSuccess) {
            (void)hipGetLastError();
            g->perm = nullptr;
            msf_graph_destroy(g);
            set_error("device allocation failed");
            return MSF_ENOMEM;
        }
        if ((rc = ws_get(c, WS_DEG, 8 * nn, &vdeg)) ||
            (rc = ws_get(c, WS_T2, 4 * relabel_table_words(n), &vtab)) ||
            (rc = ws_get(c, WS_Q2, 4 * nn, &vinv)) ||
            (rc = ws_get(c, WS_RUNROW, 4 * (2 * nn + 1), &vseg)) ||
            (rc = ws_get(c, WS_RUNS, 4 * relabel_segments_cap(n, nnz), &vsr)) ||
            (rc = relabel_csr_by_degree(c, n, (const uint32_t *)vrp0, (const uint32_t *)vcol0,
                                        (const uint64_t *)vkey0, (uint32_t *)vdeg,
                                        (uint32_t *)vtab, g->perm, (uint32_t *)vinv,
                                        (uint32_t *)vseg, (uint32_t *)vsr, (uint32_t *)g->bufs[2],
                                        (uint32_t *)g->bufs[3], (uint64_t *)g->bufs[4]))) {
            msf_graph_destroy(g);
            return rc;
        }
        launch_relabel_edges(c->stream, (int32_t *)g->bufs[0], m, (const uint32_t *)vinv);
        g->a.row_ptr = (uint32_t *)g->bufs[2];
        g->a.col = (uint32_t *)g->bufs[3];
        g->a.key = (uint64_t *)g->bufs[4];
        g->a.chunk_row = (uint32_t *)g->bufs[5];
        g->a.edges = (const int32_t *)g->bufs[0];
    }
    if (g->a.sl.S == 1) {
        launch_long_entries(c->stream, g->a.row_ptr, n, c->dcnt);
        if ((rc = read_counters(c))) {
            msf_graph_destroy(g);
            return rc;
        }
    }
    for (int q = 0; q <= g->a.sl.S; ++q) g->a.sl.sstart[q] = c->hcnt->sstart[q];
    set_chunks(&g->a);
    g->a.segs = c->hcnt->segs;
    g->long_rows = g->a.sl.S == 1 && g->a.nnz > 0 &&
                   4 * c->hcnt->long_entries >= (uint64_t)g->a.nnz;
    if (g->a.nnz) launch_chunk_rows_sliced(c->stream, g->a);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        msf_graph_destroy(g);
        return hip_fail(e, "build");
    }
    *out = g;
    return MSF_OK;
}

void msf_graph_destroy(msf_graph *g)
{
    if (!g) return;
    if (g->ctx) {
        (void)hipSetDevice(g->ctx->c.device);
        (void)hipStreamSynchronize(g->ctx->c.stream);
    }
    for (auto &p : g->bufs)
        if (p) (void)hipFree(p);
    if (g->perm) (void)hipFree(g->perm);
    delete g;
}

msf_status msf_multilinear(msf_ctx *ctx, const msf_graph *g, const uint32_t *p, uint64_t *r)
{
    if (!ctx || !g || g->ctx != ctx) {
        set_error("bad ctx/graph");
        return MSF_EINVAL;
    }
    const int32_t n = g->a.n;
    if (n > 0 && (!p || !r)) {
        set_error("NULL p/r");
        return MSF_EINVAL;
    }
    if (n == 0) return MSF_OK;
    Ctx *c = &ctx->c;
    MSF_HIP(hipSetDevice(c->device));
    clear_err_done(c);
    launch_check_parents(c->stream, p, n, c->dcnt);
    msf_status rc = read_counters(c);
    if (rc) return rc;
    if ((rc = decode_err(c->hcnt->err))) return rc;
    launch_fill_u64(c->stream, r, KEY_INF, (size_t)n);
    // device events around the gather of p into the graph's vertex order
    // and around the sweep kernel (statistics: one round whose sweep_ms /
    // sweep_bytes describe the sweep; pass_ms[0] / pass_bytes[0] the gather)
    const uint32_t *pg = p;
    MSF_HIP(hipEventRecord(c->kev[0], c->stream));
    if (g->perm) {
        void *vq;
        if ((rc = ws_get(c, WS_Q, 4 * (size_t)n, &vq))) return rc;
        launch_relabel_gather(c->stream, p, g->perm, n, (uint32_t *)vq);
        pg = (const uint32_t *)vq;
    }
    MSF_HIP(hipEventRecord(c->sev[0], c->stream));
    launch_sweep(c->stream, g->a, pg, r, c->dcnt, false, nullptr, true, g->long_rows);
    MSF_HIP(hipEventRecord(c->sev[1], c->stream));
    MSF_HIP(hipGetLastError());
    c->stats = msf_stats{};
    c->stats.rounds = 1;
    c->stats.active_nnz[0] = g->a.nnz;
    c->stats.sweep_bytes[0] = 12.0 * g->a.nnz + 8.0 * g->a.segs + 4.0;
    c->stats.pass_bytes[0] = g->perm ? 12.0 * n : 0.0;
    c->ml_pending = true;
    return MSF_OK;
}

msf_status msf_multilinear_rows(msf_ctx *ctx, const msf_graph *g, const uint32_t *p, uint64_t *r,
                                int32_t row_lo, int32_t row_hi)
{
    if (!ctx || !g || g->ctx != ctx) {
        set_error("bad ctx/graph");
        return MSF_EINVAL;
    }
    const int32_t n = g->a.n;
    if (row_lo < 0 || row_hi < row_lo || row_hi > n) {
        set_error("row range [%d, %d) outside [0, %d)", row_lo, row_hi, n);
        return MSF_EINVAL;
    }
    if (g->a.sl.S != 1) {
        set_error("row ranges need a graph stored as one column slice");
        return MSF_EINVAL;
    }
    if (n > 0 && (!p || !r)) {
        set_error("NULL p/r");
        return MSF_EINVAL;
    }
    if (n == 0) return MSF_OK;
    Ctx *c = &ctx->c;
    MSF_HIP(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    // the range's entries [row_ptr[row_lo], row_ptr[row_hi]) and its rows
    // with entries, then the parent check
    Adj rows = g->a;
    rows.row_ptr = g->a.row_ptr + row_lo;
    rows.n = row_hi - row_lo;
    zero_counters(c);
    launch_slice_info(s, rows, c->dcnt);
    launch_check_parents(s, p, n, c->dcnt);
    msf_status rc = read_counters(c);
    if (rc) return rc;
    if ((rc = decode_err(c->hcnt->err))) return rc;
    // the graph's adjacency with its entry range cut to the row range (the
    // sweep takes the entries of a slice from its start and end), and the
    // chunk-row table of that range
    Adj a = g->a;
    a.sl.sstart[0] = c->hcnt->sstart[0];
    a.sl.sstart[1] = c->hcnt->sstart[1];
    set_chunks(&a);
    a.segs = c->hcnt->segs;
    void *vcr;
    if ((rc = ws_get(c, WS_CHUNKROW2, 4 * ((size_t)a.nchunks + 1), &vcr))) return rc;
    a.chunk_row = (uint32_t *)vcr;
    if (a.nnz) launch_chunk_rows_sliced(s, a);
    launch_fill_u64(s, r, KEY_INF, (size_t)n);
    // device events as in msf_multilinear
    const uint32_t *pg = p;
    MSF_HIP(hipEventRecord(c->kev[0], s));
    if (g->perm) {
        void *vq;
        if ((rc = ws_get(c, WS_Q, 4 * (size_t)n, &vq))) return rc;
        launch_relabel_gather(s, p, g->perm, n, (uint32_t *)vq);
        pg = (const uint32_t *)vq;
    }
    MSF_HIP(hipEventRecord(c->sev[0], s));
    launch_sweep(s, a, pg, r, c->dcnt, false, nullptr, true, g->long_rows);
    MSF_HIP(hipEventRecord(c->sev[1], s));
    MSF_HIP(hipGetLastError());
    c->stats = msf_stats{};
    c->stats.rounds = 1;
    c->stats.active_nnz[0] = a.nnz;
    c->stats.sweep_bytes[0] = 12.0 * a.nnz + 8.0 * a.segs + 4.0;
    c->stats.pass_bytes[0] = g->perm ? 12.0 * n : 0.0;
    c->ml_pending = true;
    return MSF_OK;
}

msf_status msf_graph_order(msf_ctx *ctx, const msf_graph *g, uint32_t *order)
{
    if (!ctx || !g || g->ctx != ctx) {
        set_error("bad ctx/graph");
        return MSF_EINVAL;
    }
    const int32_t n = g->a.n;
    if (n > 0 && !order) {
        set_error("NULL order");
        return MSF_EINVAL;
    }
    if (n == 0) return MSF_OK;
    Ctx *c = &ctx->c;
    MSF_HIP(hipSetDevice(c->device));
    if (g->perm)
        MSF_HIP(hipMemcpyAsync(order, g->perm, 4 * (size_t)n, hipMemcpyDeviceToDevice, c->stream));
    else
        launch_iota_u32(c->stream, order, (size_t)n);
    MSF_HIP(hipGetLastError());
    MSF_HIP(hipStreamSynchronize(c->stream));
    return MSF_OK;
}

msf_status msf_multilinear_pairwise(msf_ctx *ctx, const msf_graph *g, const uint32_t *p,
                                    uint64_t *r)
{
    if (!ctx || !g || g->ctx != ctx) {
        set_error("bad ctx/graph");
        return MSF_EINVAL;
    }
    const int32_t n = g->a.n;
    if (n > 0 && (!p || !r)) {
        set_error("NULL p/r");
        return MSF_EINVAL;
    }
    if (n == 0) return MSF_OK;
    Ctx *c = &ctx->c;
    MSF_HIP(hipSetDevice(c->device));
    // the padded length the graph's column array was allocated with
    const size_t extent = 2 * (size_t)std::max<int64_t>(g->a.m, 1) + SWEEP_PAD;
    void *vpj;
    msf_status rc = ws_get(c, WS_PAIR, 4 * extent, &vpj);
    if (rc) return rc;
    clear_err_done(c);
    launch_check_parents(c->stream, p, n, c->dcnt);
    if ((rc = read_counters(c))) return rc;
    if ((rc = decode_err(c->hcnt->err))) return rc;
    launch_fill_u64(c->stream, r, KEY_INF, (size_t)n);
    const uint32_t *pg = p;
    if (g->perm) {
        void *vq;
        if ((rc = ws_get(c, WS_Q, 4 * (size_t)n, &vq))) return rc;
        launch_relabel_gather(c->stream, p, g->perm, n, (uint32_t *)vq);
        pg = (const uint32_t *)vq;
    }
    launch_sweep_pairwise(c->stream, g->a, pg, r, (uint32_t *)vpj, extent, c->dcnt);
    MSF_HIP(hipGetLastError());
    return MSF_OK;
}

msf_status msf_shortcut(msf_ctx *ctx, int32_t n, uint32_t *p, int32_t *sub_iters)
{
    return msf_shortcut_strategy(ctx, n, p, MSF_SHORTCUT_FRONTIER, 0.0, sub_iters);
}

msf_status msf_shortcut_strategy(msf_ctx *ctx, int32_t n, uint32_t *p, int32_t strategy,
                                 double switch_fraction, int32_t *sub_iters)
{
    if (!ctx || n < 0 || (n > 0 && !p)) {
        set_error("bad arguments");
        return MSF_EINVAL;
    }
    if (strategy != MSF_SHORTCUT_FRONTIER && strategy != MSF_SHORTCUT_FULL &&
        strategy != MSF_SHORTCUT_SWITCH) {
        set_error("unknown shortcut strategy");
        return MSF_EINVAL;
    }
    if (!(switch_fraction >= 0.0 && switch_fraction <= 1.0)) {
        set_error("switch_fraction outside [0, 1]");
        return MSF_EINVAL;
    }
    if (n == 0) {
        if (sub_iters) *sub_iters = 0;
        return MSF_OK;
    }
    Ctx *c = &ctx->c;
    MSF_HIP(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    void *vq, *vf, *vf2, *vst;
    msf_status rc;
    if ((rc = ws_get(c, WS_Q, 4 * (size_t)n, &vq)) || (rc = ws_get(c, WS_FL, 4 * (size_t)n, &vf)) ||
        (rc = ws_get(c, WS_RL2, 4 * (size_t)n, &vf2)) ||
        (rc = ws_get(c, WS_STATUS, 8 * ((size_t)compaction_tiles((uint64_t)n) + 1), &vst)))
        return rc;
    uint64_t *status = (uint64_t *)vst;
    uint32_t *q = (uint32_t *)vq, *F[2] = {(uint32_t *)vf, (uint32_t *)vf2};
    zero_counters(c);
    launch_check_parents(s, p, n, c->dcnt);
    if ((rc = read_counters(c))) return rc;
    if ((rc = decode_err(c->hcnt->err))) return rc;
    MSF_HIP(hipMemcpyAsync(q, p, 4 * (size_t)n, hipMemcpyDeviceToDevice, s));
    // every pass at least halves each vertex's distance to its root, whatever
    // the kind of pass, so both kinds share one bound
    int cap = 2;
    while ((1ll << (cap - 1)) < (long long)n) ++cap;  // ceil(log2 n) + 1
    int passes = 0, fi = 0;
    bool done = false;
    if (strategy != MSF_SHORTCUT_FRONTIER) {
        // full passes while more than `limit` vertices are unfinished
        const double limit = strategy == MSF_SHORTCUT_FULL ? 0.0 : switch_fraction * (double)n;
        while (passes < cap) {
            launch_fill_u32(s, &c->dcnt->nR, 0u, 1);
            launch_jump_full(s, q, n, c->dcnt);
            if ((rc = read_counters(c))) return rc;
            ++passes;
            const uint32_t left = c->hcnt->nR;
            done = left == 0;
            if (done || (double)left <= limit) break;
        }
    }
    uint32_t nF = 0;
    if (!done && strategy != MSF_SHORTCUT_FULL) {
        launch_jump_init(s, q, n, F[0], status, c->dcnt);
        if ((rc = read_counters(c))) return rc;
        nF = c->hcnt->nF;
    }
    while (nF > 0 && passes < cap) {
        launch_fill_u32(s, &c->dcnt->nR, 0u, 1);
        launch_jump_pass(s, F[fi], nF, q, F[fi ^ 1], status, c->dcnt);
        if ((rc = read_counters(c))) return rc;
        nF = c->hcnt->nR;
        fi ^= 1;
        ++passes;
    }
    launch_check_roots(s, p, q, n, c->dcnt);
    if ((rc = read_counters(c))) return rc;
    if ((rc = decode_err(c->hcnt->err))) return rc;
    MSF_HIP(hipMemcpyAsync(p, q, 4 * (size_t)n, hipMemcpyDeviceToDevice, s));
    MSF_HIP(hipStreamSynchronize(s));
    if (sub_iters) *sub_iters = passes;
    return MSF_OK;
}

msf_status msf_components(msf_ctx *ctx, const msf_graph *g, uint32_t *labels, int32_t *rounds)
{
    if (!ctx || !g || g->ctx != ctx) {
        set_error("bad ctx/graph");
        return MSF_EINVAL;
    }
    const int32_t n = g->a.n;
    if (n > 0 && !labels) {
        set_error("NULL labels");
        return MSF_EINVAL;
    }
    if (n == 0) {
        if (rounds) *rounds = 0;
        return MSF_OK;
    }
    Ctx *c = &ctx->c;
    MSF_HIP(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    msf_status rc;
    if (kept_heads_eligible(c, g->a) || (int64_t)n > c->graph_rounds_max_n ||
        c->graph_rounds == 0) {
        // the host-stepped rounds over compacted root lists, with the head
        // sweep where msf_solve would take it (the graph is only read)
        if ((rc = solve_start_kept(c, g->a, g->perm, labels))) return rc;
        while (!solve_done(c)) {
            MSF_HIP(hipEventSynchronize(c->ev[3]));
            if ((rc = solve_advance(c))) return rc;
        }
        MSF_HIP(hipStreamSynchronize(s));
        if (rounds) *rounds = c->stats.hook_rounds;
        return MSF_OK;
    }
    const size_t nn = (size_t)n;
    void *vr, *vh, *ve, *vw, *vf, *vpart, *vp = labels;
    if ((rc = ws_get(c, WS_R, 8 * nn, &vr)) || (rc = ws_get(c, WS_H, 4 * nn, &vh)) ||
        (rc = ws_get(c, WS_HEDGE, 4 * nn, &ve)) || (rc = ws_get(c, WS_HWK, 4 * nn, &vw)) ||
        (rc = ws_get(c, WS_FLAGS, (size_t)std::max<int64_t>(g->a.m, 1) + 4, &vf)) ||
        (rc = ws_get(c, WS_PART, chase_part_bytes(), &vpart)) ||
        (g->perm && (rc = ws_get(c, WS_Q2, 4 * nn, &vp))))
        return rc;
    // otherwise the rounds of the forest solve, all on the device (fixed launch sizes,
    // termination by the device flag): the forest flags and weight sums they
    // keep are not read; p ends as the root of every vertex's tree, in the
    // graph's vertex order, translated back at the end
    GraphRound R;
    R.a = g->a;
    R.p = (uint32_t *)vp;
    R.h = (uint32_t *)vh;
    R.hedge = (uint32_t *)ve;
    R.hwk = (uint32_t *)vw;
    R.r = (uint64_t *)vr;
    R.flags = (uint8_t *)vf;
    R.part = (uint32_t *)vpart;
    R.wt = MSF_W_U32;  // the weight sum is not read
    zero_counters(c);
    launch_iota_u32(s, R.p, nn);
    launch_fill_u64(s, R.r, KEY_INF, nn);
    for (;;) {
        for (int k = 0; k < 4; ++k) enqueue_graph_round(s, R, c->dcnt, true);
        if ((rc = read_counters(c))) return rc;
        if ((rc = decode_err(c->hcnt->err))) return rc;
        if (c->hcnt->gdone) break;
    }
    // the flag stays set only while device-driven rounds run
    launch_fill_u32(s, &c->dcnt->gdone, 0u, 1);
    if (g->perm) launch_relabel_labels(s, R.p, g->perm, n, labels);
    MSF_HIP(hipGetLastError());
    MSF_HIP(hipStreamSynchronize(s));
    if (rounds) {
        // rounds that kept a hook (the last round keeps none)
        int32_t k = 0;
        for (uint32_t i = 0; i < c->hcnt->grounds && i < 64; ++i) k += c->hcnt->ghist[i] != 0;
        *rounds = k;
    }
    return MSF_OK;
}

msf_status msf_solve_starcheck(msf_ctx *ctx, const msf_graph *g, uint8_t *in_forest,
                               int32_t *rounds)
{
    if (!ctx || !g || g->ctx != ctx) {
        set_error("bad ctx/graph");
        return MSF_EINVAL;
    }
    const int32_t n = g->a.n;
    const int64_t m = g->a.m;
    if (m > 0 && !in_forest) {
        set_error("NULL in_forest");
        return MSF_EINVAL;
    }
    Ctx *c = &ctx->c;
    MSF_HIP(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    if (m > 0) MSF_HIP(hipMemsetAsync(in_forest, 0, (size_t)m, s));
    if (n == 0 || m == 0) {
        MSF_HIP(hipStreamSynchronize(s));
        if (rounds) *rounds = 0;
        return MSF_OK;
    }
    void *vr, *vh, *vp0, *vp1, *vst;
    msf_status rc;
    if ((rc = ws_get(c, WS_R, 8 * (size_t)n, &vr)) || (rc = ws_get(c, WS_H, 4 * (size_t)n, &vh)) ||
        (rc = ws_get(c, WS_P, 4 * (size_t)n, &vp0)) || (rc = ws_get(c, WS_Q, 4 * (size_t)n, &vp1)) ||
        (rc = ws_get(c, WS_FLAGS, 4 * (size_t)n, &vst)))
        return rc;
    uint64_t *r = (uint64_t *)vr;
    uint32_t *h = (uint32_t *)vh, *star = (uint32_t *)vst;
    uint32_t *P[2] = {(uint32_t *)vp0, (uint32_t *)vp1};
    zero_counters(c);
    launch_iota_u32(s, P[0], (size_t)n);
    // O(log n) rounds for AS; the cap only guards against a defect
    int lg = 1;
    while ((1ll << lg) < (long long)n) ++lg;
    const int cap = 8 * lg + 16;
    int cur = 0, done_rounds = 0;
    for (;;) {
        if (done_rounds >= cap) {
            set_error("starcheck: no convergence");
            return MSF_EDEVICE;
        }
        uint32_t *p = P[cur];
        launch_star_check(s, p, n, star);
        launch_fill_u64(s, r, KEY_INF, (size_t)n);
        launch_sweep(s, g->a, p, r, c->dcnt);
        launch_fill_u32(s, &c->dcnt->nR, 0u, 1);
        launch_cc_hook(s, p, r, g->a.edges, n, h, c->dcnt, star, in_forest);
        if ((rc = read_counters(c))) return rc;
        const uint32_t hooks = c->hcnt->nR;
        if (hooks) launch_cc_apply(s, h, n, p);
        launch_fill_u32(s, &c->dcnt->nR, 0u, 1);
        launch_jump_once(s, p, n, P[cur ^ 1], c->dcnt);
        if ((rc = read_counters(c))) return rc;
        const uint32_t changed = c->hcnt->nR;
        cur ^= 1;
        ++done_rounds;
        if (hooks == 0 && changed == 0) break;
    }
    MSF_HIP(hipStreamSynchronize(s));
    if (rounds) *rounds = done_rounds;
    return MSF_OK;
}

size_t msf_request_footprint(int32_t n, int64_t m)
{
    // the most any path of a solve holds, per edge: input copy (12),
    // two-level build staging (two 16-byte records and a 2-byte row per
    // stored direction: 68), adjacency (24), the filtered twin of the full
    // sweep or the head sweep's run arrays (at most 24.2), forest flags (1)
    // -> 131; per vertex: row pointers (8), p, h, hedge, three lists, hook
    // weights, ids (32), r (8), the head sweep's per-row runs and counts
    // (36) -> 84; plus chunk tables, partials and allocation slack
    const size_t nn = (size_t)std::max(n, 1), mm = (size_t)std::max<int64_t>(m, 1);
    return 131 * mm + 84 * nn + ((size_t)32 << 20);
}

}  // extern "C"
