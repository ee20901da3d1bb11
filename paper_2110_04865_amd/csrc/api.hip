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
            MSF_HIP(hipStreamSynchronize(c->stream));
            MSF_HIP(hipFree(b.ptr));
            b.ptr = nullptr;
            b.cap = 0;
        }
        size_t cap = (bytes + (1u << 20) - 1) & ~(size_t)((1u << 20) - 1);
        hipError_t e = hipMalloc(&b.ptr, cap);
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

static void zero_counters(Ctx *c)
{
    launch_fill_u32(c->stream, reinterpret_cast<uint32_t *>(c->dcnt), 0u,
                    sizeof(Counters) / sizeof(uint32_t));
}

static msf_status decode_err(uint32_t err)
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

// ---------------------------------------------------------------- solve --

struct SolveBufs {
    uint2 *slot;
    uint32_t *deg, *rp[2], *col[2], *crow[2], *p, *h, *hedge, *R[2], *F, *blive;
    uint64_t *key[2], *r, *status;
    uint8_t *flags;
    void *part;
};

static msf_status get_solve_bufs(Ctx *c, int32_t n, int64_t m, SolveBufs *b)
{
    const size_t nn = (size_t)std::max(n, 1), mm = (size_t)std::max<int64_t>(m, 1);
    const size_t nnz_cap = 2 * mm;
    const size_t nch = sweep_nchunks((uint32_t)std::min<size_t>(nnz_cap, 0xFFFFFFFFull)) + 2;
    size_t st = std::max<size_t>(nch, (size_t)output_tiles((int64_t)mm) + 1);
    st = std::max<size_t>(st, nn / 2048 + 2);
    const size_t part_bytes = std::max<size_t>(output_part_bytes((int64_t)mm), 4 * 4096 + 256);
    void *v[22];
    msf_status rc;
#define GET(i, slot, bytes)                                  \
    if ((rc = ws_get(c, slot, (bytes), &v[i])) != MSF_OK) return rc;
    GET(2, WS_ROWPTR, 4 * (nn + 1));
    GET(3, WS_COL, 4 * nnz_cap);
    GET(4, WS_KEY, 8 * nnz_cap);
    GET(5, WS_CHUNKROW, 4 * nch);
    GET(6, WS_P, 4 * nn);
    GET(7, WS_R, 8 * nn);
    GET(8, WS_H, 4 * nn);
    GET(9, WS_HEDGE, 4 * nn);
    GET(10, WS_RL, 4 * nn);
    GET(11, WS_RL2, 4 * nn);
    GET(12, WS_FL, 4 * nn);
    GET(13, WS_FLAGS, (mm + 16) & ~(size_t)3);
    GET(14, WS_STATUS, 8 * st);
    GET(15, WS_SCRATCH, 4 * nch);
    GET(16, WS_PART, part_bytes);
#undef GET
    b->rp[0] = (uint32_t *)v[2];
    b->col[0] = (uint32_t *)v[3];
    b->key[0] = (uint64_t *)v[4];
    b->crow[0] = (uint32_t *)v[5];
    b->p = (uint32_t *)v[6];
    b->r = (uint64_t *)v[7];
    b->h = (uint32_t *)v[8];
    b->hedge = (uint32_t *)v[9];
    b->R[0] = (uint32_t *)v[10];
    b->R[1] = (uint32_t *)v[11];
    b->F = (uint32_t *)v[12];
    b->flags = (uint8_t *)v[13];
    b->status = (uint64_t *)v[14];
    b->blive = (uint32_t *)v[15];
    b->part = v[16];
    b->rp[1] = b->col[1] = b->crow[1] = nullptr;
    b->key[1] = nullptr;
    return MSF_OK;
}

static msf_status get_filter_bufs(Ctx *c, int32_t n, int64_t m, SolveBufs *b)
{
    if (b->rp[1]) return MSF_OK;
    const size_t nn = (size_t)std::max(n, 1), mm = (size_t)std::max<int64_t>(m, 1);
    const size_t nnz_cap = 2 * mm;
    const size_t nch = sweep_nchunks((uint32_t)std::min<size_t>(nnz_cap, 0xFFFFFFFFull)) + 2;
    void *v[4];
    msf_status rc;
    if ((rc = ws_get(c, WS_ROWPTR2, 4 * (nn + 1), &v[0]))) return rc;
    if ((rc = ws_get(c, WS_COL2, 4 * nnz_cap, &v[1]))) return rc;
    if ((rc = ws_get(c, WS_KEY2, 8 * nnz_cap, &v[2]))) return rc;
    if ((rc = ws_get(c, WS_CHUNKROW2, 4 * nch, &v[3]))) return rc;
    b->rp[1] = (uint32_t *)v[0];
    b->col[1] = (uint32_t *)v[1];
    b->key[1] = (uint64_t *)v[2];
    b->crow[1] = (uint32_t *)v[3];
    return MSF_OK;
}

msf_status solve_device(Ctx *c, int32_t n, int64_t m, const int32_t *d_edges, const void *d_w,
                        msf_wtype wt, int32_t *d_ids, int64_t *count, msf_total *total)
{
    hipStream_t s = c->stream;
    msf_stats st{};
    SolveBufs b{};
    msf_status rc = get_solve_bufs(c, n, m, &b);
    if (rc) return rc;

    MSF_HIP(hipEventRecord(c->ev[0], s));
    zero_counters(c);
    Adj a;
    rc = build_adjacency(c, n, m, d_edges, d_w, wt, &a, b.rp[0], b.col[0], b.key[0], b.crow[0]);
    if (rc) return rc;
    MSF_TRY(read_counters(c));
    if ((rc = decode_err(c->hcnt->err))) return rc;
    a.nnz = c->hcnt->count;
    a.nchunks = sweep_nchunks(a.nnz);
    launch_chunk_rows(s, a.row_ptr, n, a.nnz, a.chunk_row, a.nchunks);
    MSF_HIP(hipEventRecord(c->ev[1], s));

    // round state
    launch_iota_u32(s, b.p, (size_t)n);
    launch_iota_u32(s, b.h, (size_t)n);
    launch_fill_u64(s, b.r, KEY_INF, (size_t)n);
    launch_fill_u32(s, reinterpret_cast<uint32_t *>(b.flags), 0u, ((size_t)m + 3) / 4);
    launch_init_roots(s, a.row_ptr, n, b.R[0], b.status, c->dcnt);
    MSF_HIP(hipGetLastError());
    MSF_TRY(read_counters(c));
    uint32_t nR = c->hcnt->nR;
    uint32_t rows = nR;  // rows with entries (every non-isolated vertex)
    bool rows_pending = false;
    int ri = 0;    // which R buffer is current
    int ai = 0;    // which adjacency buffer set is current
    double live_frac = 1.0;
    int rounds = 0;
    // fewer than two live roots: no outgoing edge can remain
    while (nR >= 2 && a.nnz > 0 && rounds < 1000) {
        bool compact = false;
        if (c->filter_mode == 2) compact = true;
        else if (c->filter_mode == 1) compact = live_frac < c->filter_threshold;
        Adj nxt = a;
        const int ev_k = rounds < 64 ? rounds : -1;
        if (ev_k >= 0) {
            MSF_HIP(hipEventRecord(c->sev[2 * ev_k], s));
            st.sweep_bytes[ev_k] = 12.0 * a.nnz + 8.0 * rows + 8.0 * nR;
        }
        if (compact) {
            if ((rc = get_filter_bufs(c, n, m, &b))) return rc;
            nxt.row_ptr = b.rp[ai ^ 1];
            nxt.col = b.col[ai ^ 1];
            nxt.key = b.key[ai ^ 1];
            nxt.chunk_row = b.crow[ai ^ 1];
            launch_sweep_compact(s, a, b.p, b.r, nxt.row_ptr, nxt.col, nxt.key, b.status,
                                 c->dcnt);
        } else {
            // round 1: p is the identity and nothing has been filtered
            launch_sweep(s, a, b.p, b.r, b.blive, c->dcnt, rounds == 0 && c->first_round_kernel);
        }
        if (ev_k >= 0) MSF_HIP(hipEventRecord(c->sev[2 * ev_k + 1], s));
        launch_hook(s, b.R[ri], nR, b.r, b.p, d_edges, b.h, b.hedge);
        launch_fill_u32(s, &c->dcnt->nR, 0u, 3);  // nR, nF, hooks
        launch_tiebreak(s, b.R[ri], nR, b.h, b.hedge, b.flags, b.R[ri ^ 1], b.F, b.status,
                        c->dcnt);
        MSF_HIP(hipGetLastError());
        MSF_TRY(read_counters(c));
        const uint32_t nF = c->hcnt->nF, nRn = c->hcnt->nR;
        if (rows_pending && ev_k >= 0) {
            st.sweep_bytes[ev_k] += 8.0 * c->hcnt->rows;  // rows of the swept CSR
            rows_pending = false;
        }
        if (rounds < 64) {
            st.hooks[rounds] = nF;
            st.active_nnz[rounds] = a.nnz;
        }
        ++rounds;
        if (nF) ++st.hook_rounds;
        if (compact) {
            const uint32_t nnz2 = c->hcnt->nnz_out;
            live_frac = a.nnz ? (double)nnz2 / (double)a.nnz : 0.0;
            nxt.nnz = nnz2;
            nxt.nchunks = sweep_nchunks(nnz2);
            if (nnz2) launch_chunk_rows(s, nxt.row_ptr, n, nnz2, nxt.chunk_row, nxt.nchunks);
            a = nxt;
            ai ^= 1;
            ++st.filtered;
        } else {
            live_frac = a.nnz ? (double)c->hcnt->live / (double)a.nnz : 0.0;
        }
        if (nF == 0) break;
        launch_chase(s, b.F, nF, b.h, (uint32_t *)b.part, c->dcnt);
        if (c->check_rounds) {
            MSF_TRY(read_counters(c));
            if (c->hcnt->err) {
                set_error("internal error: hook cycle in round %d", rounds);
                return MSF_EDEVICE;
            }
        }
        launch_update_parents(s, a.row_ptr, n, b.p, b.h, (uint32_t *)b.part, c->dcnt);
        ri ^= 1;
        nR = nRn;
        rows = 0;  // read back with the next round's counters
        rows_pending = true;
    }
    st.rounds = rounds;

    // output
    launch_output(s, b.flags, m, d_w, wt, d_ids, b.status, b.part, c->dcnt);
    MSF_HIP(hipEventRecord(c->ev[2], s));
    MSF_HIP(hipGetLastError());
    MSF_TRY(read_counters(c));
    if (c->hcnt->err) {
        set_error("internal error: hook cycle detected");
        return MSF_EDEVICE;
    }
    float ms_build = 0.f, ms_rounds = 0.f;
    (void)hipEventElapsedTime(&ms_build, c->ev[0], c->ev[1]);
    (void)hipEventElapsedTime(&ms_rounds, c->ev[1], c->ev[2]);
    st.build_ms = ms_build;
    st.rounds_ms = ms_rounds;
    for (int k = 0; k < rounds && k < 64; ++k) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, c->sev[2 * k], c->sev[2 * k + 1]);
        st.sweep_ms[k] = ms;
    }
    st.max_chase = (int32_t)c->hcnt->max_chase;
    c->stats = st;
    *count = (m > 0) ? (int64_t)c->hcnt->count : 0;
    if (total) {
        total->u64 = (wt == MSF_W_U32) ? c->hcnt->total_u64 : 0;
        total->f64 = (m > 0) ? c->hcnt->total_f64 : 0.0;
    }
    return MSF_OK;
}

}  // namespace msf

using namespace msf;

// ------------------------------------------------------------------ ABI --

extern "C" {

const char *msf_last_error(void) { return g_err.c_str(); }

const char *msf_version(void) { return "msf-gfx950 0.1"; }

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
    Ctx *c = &x->c;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (hipMalloc(&c->dcnt, sizeof(Counters)) != hipSuccess ||
        hipHostMalloc(&c->hcnt, sizeof(Counters), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        if (c->dcnt) (void)hipFree(c->dcnt);
        delete x;
        set_error("counter allocation failed");
        return MSF_ENOMEM;
    }
    for (auto &ev : c->sev) {
        if (hipEventCreate(&ev) != hipSuccess) {
            set_error("event creation failed");
            msf_ctx_destroy(x);
            return MSF_EDEVICE;
        }
    }
    for (auto &ev : c->ev) {
        if (hipEventCreate(&ev) != hipSuccess) {
            set_error("event creation failed");
            msf_ctx_destroy(x);
            return MSF_EDEVICE;
        }
    }
    if (const char *f = getenv("MSF_FILTER")) c->filter_mode = atoi(f);
    if (const char *f = getenv("MSF_CHECK_ROUNDS")) c->check_rounds = atoi(f) != 0;
    if (const char *f = getenv("MSF_FIRST_ROUND")) c->first_round_kernel = atoi(f) != 0;
    if (const char *f = getenv("MSF_BUCKETED_BUILD")) c->bucketed_build = atoi(f) != 0;
    if (const char *f = getenv("MSF_FILTER_THRESHOLD")) c->filter_threshold = atof(f);
    *out = x;
    return MSF_OK;
}

void msf_ctx_destroy(msf_ctx *x)
{
    if (!x) return;
    Ctx *c = &x->c;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto &b : c->ws)
        if (b.ptr) (void)hipFree(b.ptr);
    for (auto &ev : c->ev)
        if (ev) (void)hipEventDestroy(ev);
    for (auto &ev : c->sev)
        if (ev) (void)hipEventDestroy(ev);
    if (c->dcnt) (void)hipFree(c->dcnt);
    if (c->hcnt) (void)hipHostFree(c->hcnt);
    delete x;
}

static msf_status check_graph_args(msf_ctx *ctx, int32_t n, int64_t m, const int32_t *edges,
                                   const void *weights, msf_wtype wt, msf_mem mem)
{
    if (!ctx) {
        set_error("ctx is NULL");
        return MSF_EINVAL;
    }
    if (n < 0 || m < 0 || m > 0x7FFFFFFFll) {
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
    rc = solve_device(c, n, m, d_edges, d_w, wt, d_ids, &cnt, &tot);
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
    *out = ctx->c.stats;
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
    const size_t nch = sweep_nchunks((uint32_t)std::min<size_t>(2 * mm, 0xFFFFFFFFull)) + 2;
    const size_t sizes[6] = {8 * mm, 4 * mm, 4 * (nn + 1), 4 * 2 * mm, 8 * 2 * mm, 4 * nch};
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
    zero_counters(c);
    rc = build_adjacency(c, n, m, (const int32_t *)g->bufs[0], g->bufs[1], wt, &g->a,
                         (uint32_t *)g->bufs[2], (uint32_t *)g->bufs[3], (uint64_t *)g->bufs[4],
                         (uint32_t *)g->bufs[5]);
    if (rc == MSF_OK) rc = read_counters(c);
    if (rc == MSF_OK) rc = decode_err(c->hcnt->err);
    if (rc) {
        msf_graph_destroy(g);
        return rc;
    }
    g->a.nnz = c->hcnt->count;
    g->a.nchunks = sweep_nchunks(g->a.nnz);
    launch_chunk_rows(c->stream, g->a.row_ptr, n, g->a.nnz, g->a.chunk_row, g->a.nchunks);
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
    launch_fill_u32(c->stream, &c->dcnt->err, 0u, 1);
    launch_check_parents(c->stream, p, n, c->dcnt);
    msf_status rc = read_counters(c);
    if (rc) return rc;
    if ((rc = decode_err(c->hcnt->err))) return rc;
    launch_fill_u64(c->stream, r, KEY_INF, (size_t)n);
    launch_sweep(c->stream, g->a, p, r);
    MSF_HIP(hipGetLastError());
    return MSF_OK;
}

msf_status msf_shortcut(msf_ctx *ctx, int32_t n, uint32_t *p, int32_t *sub_iters)
{
    if (!ctx || n < 0 || (n > 0 && !p)) {
        set_error("bad arguments");
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
    launch_jump_init(s, q, n, F[0], status, c->dcnt);
    if ((rc = read_counters(c))) return rc;
    uint32_t nF = c->hcnt->nF;
    int cap = 2;
    while ((1ll << (cap - 1)) < (long long)n) ++cap;  // ceil(log2 n) + 1
    int passes = 0, fi = 0;
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

size_t msf_request_footprint(int32_t n, int64_t m)
{
    // edges + weights (12m), slots (8m), CSR (12 * 2m + 4(n+1)), chunk rows,
    // per-vertex state p, h, hedge, r, lists (32n), forest flags (m)
    const size_t nn = (size_t)std::max(n, 1), mm = (size_t)std::max<int64_t>(m, 1);
    return 12 * mm + 8 * mm + 24 * mm + 4 * (nn + 1) + (2 * mm / SWEEP_CHUNK + 2) * 4 + 32 * nn +
           mm + (1u << 16);
}

}  // extern "C"
