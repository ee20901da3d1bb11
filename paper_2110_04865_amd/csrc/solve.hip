// The round loop of Algorithm 2 with complete shortcutting (section 4.2), as
// a resumable state machine per context.
//
// Step sequence (each step ends with an asynchronous copy of the counters
// to pinned host memory and an event):
//   build   adjacency build (validation flags, stored-entry count)
//   roots   round state: p = identity, r = empty, forest flags cleared, R
//   round   multilinear sweep (+ filtering when the live fraction is low),
//           hook, tie break; the counters say how many roots hooked (nF)
//           and how many stay roots (nR)
//   -> if some root hooked: shortcut chase + parent update are enqueued in
//      front of the next round's sweep
//   output  ascending forest ids, count, exact total
//
// The loop stops after a round in which nothing hooks (the parent vector is
// then unchanged, the paper's termination test), or earlier when fewer than
// two roots can still have an outgoing edge.
#include <algorithm>
#include <cmath>

#include "msf_internal.hpp"

namespace msf {

// Chunk-table capacity: every slice may add two partial chunks.
static size_t chunk_cap(size_t nnz_cap)
{
    return sweep_nchunks((uint32_t)std::min<size_t>(nnz_cap, 0xFFFFFFFFull)) + 2 * MAX_SLICES + 2;
}

// adj: also the buffers the adjacency is built into (not for a kept graph's)
static msf_status get_solve_bufs(Ctx *c, int32_t n, int64_t m, int S, SolveBufs *b,
                                 bool adj = true)
{
    const size_t nn = (size_t)std::max(n, 1), mm = (size_t)std::max<int64_t>(m, 1);
    const size_t nnz_cap = 2 * mm;
    const size_t nch = chunk_cap(nnz_cap);
    size_t st = std::max<size_t>(nch, (size_t)output_tiles((int64_t)mm) + 1);
    // a one-pass scan of n items takes its look-back status from this slot
    // (it must not grow under the solve's pointer), and the root list's
    // per-tile counts and their scan live here too
    st = std::max<size_t>(st, nn / 2048 + 2);
    st = std::max<size_t>(st, (size_t)compaction_tiles((uint64_t)nn) + 1);
    const size_t part_bytes = std::max<size_t>(
        {output_part_bytes((int64_t)mm), chase_part_bytes(), 4 * 4096 + 256});
    struct Req {
        Slot s;
        size_t bytes;
    } req[] = {
        {WS_ROWPTR, 4 * (size_t)S * (nn + 1)}, {WS_COL, 4 * (nnz_cap + SWEEP_PAD)},
        {WS_KEY, 8 * (nnz_cap + SWEEP_PAD)},
        {WS_CHUNKROW, 4 * nch},    {WS_P, 4 * nn},        {WS_R, 8 * nn},
        {WS_H, 4 * nn},            {WS_HEDGE, 4 * nn},    {WS_RL, 4 * nn},
        {WS_RL2, 4 * nn},          {WS_FL, 4 * nn},       {WS_FLAGS, (mm + 16) & ~(size_t)3},
        {WS_STATUS, 8 * st},       {WS_WLIVE, 4 * (SWEEP_BLOCK / 64) * nch},
        {WS_PART, part_bytes},     {WS_HWK, 4 * nn},
    };
    void *v[sizeof(req) / sizeof(req[0])];
    for (size_t i = 0; i < sizeof(req) / sizeof(req[0]); ++i) {
        const bool adjacency = req[i].s == WS_ROWPTR || req[i].s == WS_COL ||
                               req[i].s == WS_KEY || req[i].s == WS_CHUNKROW;
        v[i] = nullptr;
        if (adj || !adjacency) MSF_TRY(ws_get(c, req[i].s, req[i].bytes, &v[i]));
    }
    b->rp[0] = (uint32_t *)v[0];
    b->col[0] = (uint32_t *)v[1];
    b->key[0] = (uint64_t *)v[2];
    b->crow[0] = (uint32_t *)v[3];
    b->p = (uint32_t *)v[4];
    b->r = (uint64_t *)v[5];
    b->h = (uint32_t *)v[6];
    b->hedge = (uint32_t *)v[7];
    b->R[0] = (uint32_t *)v[8];
    b->R[1] = (uint32_t *)v[9];
    b->F = (uint32_t *)v[10];
    b->flags = (uint8_t *)v[11];
    b->status = (uint64_t *)v[12];
    b->wlive = (uint32_t *)v[13];
    b->part = v[14];
    b->hwk = (uint32_t *)v[15];
    b->rp[1] = b->col[1] = b->crow[1] = nullptr;
    b->key[1] = nullptr;
    return MSF_OK;
}

static msf_status get_filter_bufs(Ctx *c, int32_t n, int64_t m, int S, SolveBufs *b)
{
    if (b->rp[1]) return MSF_OK;
    const size_t nn = (size_t)std::max(n, 1), mm = (size_t)std::max<int64_t>(m, 1);
    const size_t nnz_cap = 2 * mm;
    const size_t nch = chunk_cap(nnz_cap);
    void *v[5];
    MSF_TRY(ws_get(c, WS_ROWPTR2, 4 * (size_t)S * (nn + 1), &v[0]));
    MSF_TRY(ws_get(c, WS_COL2, 4 * (nnz_cap + SWEEP_PAD), &v[1]));
    MSF_TRY(ws_get(c, WS_KEY2, 8 * (nnz_cap + SWEEP_PAD), &v[2]));
    MSF_TRY(ws_get(c, WS_CHUNKROW2, 4 * nch, &v[3]));
    MSF_TRY(ws_get(c, WS_CHUNKINFO, 4 * chunk_info_words((uint32_t)nch), &v[4]));
    b->cinfo = (uint32_t *)v[4];
    b->rp[1] = (uint32_t *)v[0];
    b->col[1] = (uint32_t *)v[1];
    b->key[1] = (uint64_t *)v[2];
    b->crow[1] = (uint32_t *)v[3];
    return MSF_OK;
}

// Buffers of the head sweep: per-chunk first runs,
// per-row run counts and offsets, run descriptors and the phase-B queue.
static msf_status get_runs_bufs(Ctx *c, int32_t n, int64_t m, Runs *R)
{
    const size_t mm = (size_t)std::max<int64_t>(m, 1), nn = (size_t)std::max(n, 1);
    const size_t nnz_cap = 2 * mm;
    const size_t nch = (nnz_cap + 63) / 64 + 1;
    const size_t rc = heads_runs_cap(nnz_cap, n);
    void *v[4];
    MSF_TRY(ws_get(c, WS_RUNCHUNK, 4 * nch + 8, &v[0]));
    MSF_TRY(ws_get(c, WS_RUNROW, 4 * nn + 4 * (nn + 1), &v[1]));  // roff: nn + 1 (scan total)
    MSF_TRY(ws_get(c, WS_RUNS, 28 * rc + 8, &v[2]));
    MSF_TRY(ws_get(c, WS_RUNPERM, 64 * nch + 64, &v[3]));
    R->perm = (uint8_t *)v[3];
    R->cfirst = (uint32_t *)v[0];
    R->rc = (uint32_t *)v[1];
    R->roff = R->rc + nn;
    R->hkey = (uint64_t *)v[2];
    R->cur = (uint32_t *)(R->hkey + rc);
    R->end = R->cur + rc;
    R->row = R->end + rc;
    R->hcol = R->row + rc;
    R->queue = R->hcol + rc;
    return MSF_OK;
}

// Default use of the head sweep: from HEADS_MIN_NNZ stored entries (below,
// the run set-up's five launches cost more than they save) and from
// HEADS_MIN_DEG stored entries per vertex on average (a run then covers
// enough entries: R-MAT s22 has 30.6 per vertex and the head sweep takes a
// solve from 7.5 to 5.6 ms; the 256^3 grid, 5.7, is even (10.3 vs 10.6 ms);
// the 10^4-graph Erdos-Renyi batch, 8, loses (139 vs 104 ms): one gather
// and one descriptor per run cost about what 14 streamed entries do).
constexpr int64_t HEADS_MIN_NNZ = (int64_t)1 << 20;
constexpr int64_t HEADS_MIN_DEG = 16;

// End a step: counters to pinned host memory, then the step event.
static msf_status end_step(Ctx *c, int next_phase)
{
    MSF_HIP(hipGetLastError());
    MSF_HIP(hipMemcpyAsync(c->hcnt, c->dcnt, sizeof(Counters), hipMemcpyDeviceToHost, c->stream));
    MSF_HIP(hipEventRecord(c->ev[3], c->stream));
    c->ss.phase = next_phase;
    return MSF_OK;
}

static msf_status enqueue_round_state(Ctx *c);
static int edge_bits(int64_t m);

msf_status solve_start(Ctx *c, int32_t n, int64_t m, const int32_t *d_edges, const void *d_w,
                       msf_wtype wt, int32_t *d_ids)
{
    SolveState &S = c->ss;
    S = SolveState{};
    c->ml_pending = false;  // this solve's statistics replace the last sweep's
    S.n = n;
    S.m = m;
    S.edges = d_edges;
    S.w = d_w;
    S.wt = wt;
    S.ids = d_ids;
    const int slices = choose_slices(n, m, c->slices);
    MSF_TRY(get_solve_bufs(c, n, m, slices, &S.b));
    // head sweep: 1 from HEADS_MIN_NNZ stored entries on, 2 always
    S.heads = slices == 1 && m > 0 && n > 0 &&
              (c->heads == 2 || (c->heads == 1 && 2 * m >= HEADS_MIN_NNZ &&
                                 2 * m >= HEADS_MIN_DEG * (int64_t)n));
    if (S.heads) MSF_TRY(get_runs_bufs(c, n, m, &S.runs));
    // rounds on the device: the full sweep without filtering, one slice
    S.graph = !S.heads && slices == 1 && c->graph_rounds > 0 && m > 0 && n > 1 &&
              (int64_t)n <= c->graph_rounds_max_n && c->filter_mode != 2 && !c->check_rounds;
    MSF_HIP(hipEventRecord(c->ev[0], c->stream));
    zero_counters(c);
    c->pass_done = 0;
    MSF_TRY(build_adjacency(c, n, m, d_edges, d_w, wt, slices, &S.a, S.b.rp[0], S.b.col[0],
                            S.b.key[0], S.b.crow[0], c->first_round == 2 ? S.b.r : nullptr,
                            &S.first_done));
    // the build may have fallen back to another slice count
    if (S.a.sl.S != 1) S.heads = S.graph = false;
    if (S.heads) {
        // the run set-up and the round state need nothing the host would
        // read back from the build (the run sort takes the entry count on
        // the device), so they follow at once: one host step fewer, and
        // the build's counters are read with the set-up's
        MSF_TRY(build_runs(c, S.runs, S.a.row_ptr, S.n, S.a.col, S.a.key,
                           (uint32_t)std::min<int64_t>(2 * m, UINT32_MAX), edge_bits(m)));
        MSF_TRY(enqueue_round_state(c));
        return end_step(c, 7);
    }
    return end_step(c, 1);
}

// Round state: p = identity, h = identity, r = empty (unless the build
// wrote round 1's minima), forest flags cleared, R = the rows with entries.
static msf_status enqueue_round_state(Ctx *c)
{
    SolveState &S = c->ss;
    hipStream_t s = c->stream;
    MSF_HIP(hipEventRecord(c->ev[1], s));
    launch_round_state(s, S.b.p, S.b.h, S.first_done ? nullptr : S.b.r, (size_t)S.n,
                       reinterpret_cast<uint32_t *>(S.b.flags), ((size_t)S.m + 3) / 4);
    MSF_TRY(launch_init_roots(c, S.a.row_ptr, S.n, S.a.sl.S, S.b.R[0], S.b.status));
    return MSF_OK;
}

// Bits of the edge ids in the keys of a graph with m edges.
static int edge_bits(int64_t m)
{
    int eb = 1;
    while (eb < 64 && ((uint64_t)(m > 1 ? m - 1 : 1) >> eb)) ++eb;
    return eb;
}

bool kept_heads_eligible(const Ctx *c, const Adj &a)
{
    const int64_t nnz = (int64_t)a.nnz;
    return a.sl.S == 1 && nnz > 0 && a.n > 0 &&
           (c->heads == 2 ||
            (c->heads == 1 && nnz >= HEADS_MIN_NNZ && nnz >= HEADS_MIN_DEG * (int64_t)a.n));
}

msf_status solve_start_kept(Ctx *c, const Adj &a, const uint32_t *perm, uint32_t *labels)
{
    SolveState &S = c->ss;
    S = SolveState{};
    c->ml_pending = false;
    S.n = a.n;
    S.m = a.m;
    S.edges = a.edges;
    S.wt = MSF_W_U32;  // the weight sum of the hooks is not read
    S.kept = true;
    S.labels = labels;
    S.perm = perm;
    MSF_TRY(get_solve_bufs(c, S.n, S.m, a.sl.S, &S.b, false));
    // the head sweep where msf_solve would take it, else the full sweep
    // without filtering; the graph is only read (the run order goes to the
    // workspace)
    S.heads = kept_heads_eligible(c, a);
    if (S.heads) MSF_TRY(get_runs_bufs(c, S.n, S.m, &S.runs));
    S.a = a;
    MSF_HIP(hipEventRecord(c->ev[0], c->stream));
    zero_counters(c);
    c->pass_done = 0;
    if (S.heads)
        MSF_TRY(build_runs(c, S.runs, a.row_ptr, S.n, a.col, a.key, a.nnz, edge_bits(S.m)));
    MSF_TRY(enqueue_round_state(c));
    return end_step(c, 2);
}

bool solve_ready(Ctx *c) { return hipEventQuery(c->ev[3]) == hipSuccess; }

bool solve_done(const Ctx *c) { return c->ss.phase == 5; }

// Enqueue one round: sweep (+ filtering), hook, tie break.
// Live roots below which the sweep reads r before each atomic (measured:
// with 200 roots the read saves 2.6x; with millions it costs up to 1.6x).
#ifndef SWEEP_READ_FILTER_ROOTS
#define SWEEP_READ_FILTER_ROOTS (1u << 16)
#endif
constexpr uint32_t READ_FILTER_ROOTS = SWEEP_READ_FILTER_ROOTS;
// A sweep with that read counts every entry it passed over as live, so
// once the roots are that few its count stops showing how many entries
// turned internal.  Then, when the trees average at least
// FILTER_ROOTS_RATIO vertices, the adaptive policy filters once anyway
// (0: never).  Measured on the 256^3 grid: the filtering sweep in round 5
// (46K roots) costs 1.3 ms, as in later rounds, and keeps 32% of the
// entries; the six later sweeps take 0.24-0.31 ms instead of 0.43-0.48
// (solve 9.13-9.18 -> 8.91-8.94 ms; waiting for fewer roots, 2^12 or 2^14,
// gave 9.31-9.33 ms).
#ifndef FILTER_ROOTS_RATIO
#define FILTER_ROOTS_RATIO 16
#endif

static msf_status enqueue_round(Ctx *c)
{
    SolveState &S = c->ss;
    hipStream_t s = c->stream;
    S.compact = false;
    if (S.heads) S.compact = false;  // the head sweep passes internal entries over by itself
    // a kept graph's rows all stay, so every vertex's parent is updated to
    // the end (its final root is its label)
    else if (S.kept) S.compact = false;
    else if (c->filter_mode == 2) S.compact = true;
    else if (c->filter_mode == 1) {
        S.compact = S.live_frac < c->filter_threshold;
        if (!S.compact && FILTER_ROOTS_RATIO > 0 && S.st.filtered == 0 && S.rounds > 0 &&
            S.nR < READ_FILTER_ROOTS && (int64_t)S.nR * FILTER_ROOTS_RATIO <= (int64_t)S.n)
            S.compact = true;
    }
    const int ev_k = S.rounds < 64 ? S.rounds : -1;
    if (ev_k >= 0) {
        S.sweep_events = ev_k + 1;
        MSF_HIP(hipEventRecord(c->sev[2 * ev_k], s));
        S.st.sweep_bytes[ev_k] = (S.rounds == 0 && S.first_done) || S.heads
                                     ? 0.0
                                     : 12.0 * S.a.nnz + 8.0 * S.a.segs + 8.0 * S.nR;
    }
    // with many live roots few runs share one: atomics without a read first
    const bool read_filter = S.nR < READ_FILTER_ROOTS;
    if (c->check_rounds) {
        // roots at the start of the round (p is exact for every vertex in
        // this mode), compared on the host with the hooks of the last round
        launch_fill_u32(s, &c->dcnt->roots, 0u, 1);
        launch_count_roots(s, S.b.p, S.n, c->dcnt);
    }
    if (S.compact) {
        MSF_TRY(get_filter_bufs(c, S.n, S.m, S.a.sl.S, &S.b));
        Adj nxt = S.a;
        nxt.row_ptr = S.b.rp[S.ai ^ 1];
        nxt.col = S.b.col[S.ai ^ 1];
        nxt.key = S.b.key[S.ai ^ 1];
        launch_sweep_compact(s, S.a, S.b.p, S.b.r, nxt.row_ptr, nxt.col, nxt.key, S.b.cinfo,
                             S.b.status, c->dcnt, read_filter);
        launch_slice_info(s, nxt, c->dcnt);  // boundaries of the filtered adjacency
    } else if (S.rounds == 0 && S.first_done) {
        // round 1's minima were written by the build; every entry is live
        launch_fill_u64(s, &c->dcnt->live, (uint64_t)S.a.nnz, 1);
    } else if (S.heads) {
        ++S.st.head_sweeps;
        launch_heads(s, S.runs, S.nruns, S.a.col, S.a.key, S.b.p, S.b.r, c->dcnt, S.rounds);
    } else {
        // round 1: p is the identity and nothing has been filtered
        launch_sweep(s, S.a, S.b.p, S.b.r, c->dcnt, S.rounds == 0 && c->first_round >= 1,
                     S.b.wlive, read_filter);
    }
    if (ev_k >= 0) MSF_HIP(hipEventRecord(c->sev[2 * ev_k + 1], s));
    launch_hook(s, S.b.R[S.ri], S.nR, S.b.r, S.b.p, S.edges, S.b.h, S.b.hedge, S.b.hwk,
                S.rounds == 0, S.heads ? S.a.row_ptr : nullptr, S.heads ? S.a.col : nullptr,
                S.heads ? S.runs.perm : nullptr, c->dcnt);
    launch_tiebreak(s, S.b.R[S.ri], S.nR, S.b.h, S.b.hedge, S.b.flags, S.b.R[S.ri ^ 1], S.b.F,
                    S.b.status, c->dcnt, S.nR > 0);
    return end_step(c, 3);
}

static msf_status enqueue_output(Ctx *c)
{
    SolveState &S = c->ss;
    S.st.rounds = S.rounds;
    if (!S.kept)
        MSF_TRY(launch_output(c, S.b.flags, S.m, S.w, S.wt, S.ids, S.b.part));
    else if (S.perm)
        launch_relabel_labels(c->stream, S.b.p, S.perm, S.n, S.labels);
    else
        MSF_HIP(hipMemcpyAsync(S.labels, S.b.p, 4 * (size_t)S.n, hipMemcpyDeviceToDevice,
                               c->stream));
    MSF_HIP(hipEventRecord(c->ev[2], c->stream));
    return end_step(c, 4);
}

static bool more_rounds(const SolveState &S)
{
    // fewer than two live roots: no outgoing edge can remain
    return S.nR >= 2 && S.a.nnz > 0 && S.rounds < 1000;
}

// Rounds enqueued per host round trip on the device-driven path.
constexpr int GRAPH_K = 4;

static GraphRound graph_round_args(const Ctx *c)
{
    const SolveState &S = c->ss;
    GraphRound g;
    g.a = S.a;
    g.p = S.b.p;
    g.h = S.b.h;
    g.hedge = S.b.hedge;
    g.hwk = S.b.hwk;
    g.r = S.b.r;
    g.flags = S.b.flags;
    g.part = (uint32_t *)S.b.part;
    g.wt = S.wt;
    return g;
}

// The captured K rounds for this solve's arguments (captured on a private
// stream, instantiated, and kept in the context while the arguments stay
// the same).
static msf_status graph_rounds_exec(Ctx *c)
{
    const SolveState &S = c->ss;
    const uint64_t key[16] = {(uint64_t)S.n, (uint64_t)S.m, (uint64_t)S.a.nnz,
                              (uint64_t)S.a.nchunks, (uint64_t)(uintptr_t)S.a.row_ptr,
                              (uint64_t)(uintptr_t)S.a.col, (uint64_t)(uintptr_t)S.a.key,
                              (uint64_t)(uintptr_t)S.a.chunk_row, (uint64_t)(uintptr_t)S.b.p,
                              (uint64_t)(uintptr_t)S.b.r, (uint64_t)(uintptr_t)S.b.part,
                              (uint64_t)(uintptr_t)S.b.flags, (uint64_t)(uintptr_t)S.edges,
                              (uint64_t)S.wt, (uint64_t)(uintptr_t)c->dcnt,
                              (uint64_t)S.a.sl.sstart[1]};
    if (c->gexec && std::equal(key, key + 16, c->gkey)) return MSF_OK;
    if (c->gexec) {
        MSF_HIP(hipGraphExecDestroy(c->gexec));
        c->gexec = nullptr;
    }
    if (!c->cap_stream) MSF_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    const GraphRound g = graph_round_args(c);
    MSF_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < GRAPH_K; ++k) enqueue_graph_round(c->cap_stream, g, c->dcnt, true);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->cap_stream, &graph);
    if (ec != hipSuccess || !graph) return hip_fail(ec, "hipStreamEndCapture");
    const hipError_t ei = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        c->gexec = nullptr;
        return hip_fail(ei, "hipGraphInstantiate");
    }
    std::copy(key, key + 16, c->gkey);
    return MSF_OK;
}

// K more device-driven rounds on the context's stream.
static msf_status enqueue_graph_rounds(Ctx *c)
{
    if (c->graph_rounds == 2) {
        MSF_TRY(graph_rounds_exec(c));
        MSF_HIP(hipGraphLaunch(c->gexec, c->stream));
    } else {
        const GraphRound g = graph_round_args(c);
        for (int k = 0; k < GRAPH_K; ++k) enqueue_graph_round(c->stream, g, c->dcnt, true);
    }
    return end_step(c, 6);
}

msf_status solve_advance(Ctx *c)
{
    SolveState &S = c->ss;
    hipStream_t s = c->stream;
    const Counters *h = c->hcnt;
    switch (S.phase) {
    case 7:  // adjacency built and the head sweep's runs set up
    case 1: {  // adjacency built
        MSF_TRY(decode_err(h->err));
        for (int q = 0; q <= S.a.sl.S; ++q) S.a.sl.sstart[q] = h->sstart[q];
        set_chunks(&S.a);
        S.a.segs = h->segs;
        if (S.phase == 7) {
            S.phase = 2;
            return solve_advance(c);  // the root list is ready too
        }
        // the chunk-row table serves the full sweep only
        if (S.a.nnz && !S.heads) launch_chunk_rows_sliced(s, S.a);
        MSF_TRY(enqueue_round_state(c));
        MSF_TRY(end_step(c, 2));
        // capture the device-driven rounds while the GPU runs the set-up
        if (S.graph && c->graph_rounds == 2) MSF_TRY(graph_rounds_exec(c));
        return MSF_OK;
    }
    case 2: {  // root list ready
        S.nR = h->nR;
        S.nruns = h->nruns;
        S.st.runs = S.heads ? (int64_t)S.nruns : 0;
        if (!more_rounds(S)) return enqueue_output(c);
        if (S.graph) {
            // round 1 (its minima from the build when it kept them), then
            // the replays
            enqueue_graph_round(s, graph_round_args(c), c->dcnt, !S.first_done);
            return enqueue_graph_rounds(c);
        }
        return enqueue_round(c);
    }
    case 6: {  // device-driven rounds: counters after the last replay
        if (!h->gdone && !h->err) return enqueue_graph_rounds(c);
        S.rounds = (int)h->grounds;
        for (int k = 0; k < S.rounds && k < 64; ++k) {
            S.st.hooks[k] = h->ghist[k];
            S.st.active_nnz[k] = S.a.nnz;
            if (h->ghist[k]) ++S.st.hook_rounds;
        }
        S.st.path = c->graph_rounds == 2 ? 3 : 2;
        // the flag stays set only while device-driven rounds run (other
        // calls on this context launch the sweep, which tests it)
        launch_fill_u32(s, &c->dcnt->gdone, 0u, 1);
        return enqueue_output(c);
    }
    case 3: {  // round counters ready
        const uint32_t nF = h->nF, nRn = h->nR;
        const int k = S.rounds;
        if (k < 64) {
            S.st.hooks[k] = nF;
            S.st.active_nnz[k] = S.a.nnz;
        }
        if (c->check_rounds) {
            if (h->err & ERR_STAR) {
                set_error("internal error: a tree is not a star at the start of round %d", k + 1);
                return MSF_EDEVICE;
            }
            if (k < 64) S.st.roots[k] = h->roots;
            // every kept hook removes exactly one root
            if (k > 0 && k <= 64 && S.st.roots[k - 1] - S.st.hooks[k - 1] != (int64_t)h->roots) {
                set_error("internal error: roots %lld -> %u over round %d with %lld hooks",
                          (long long)S.st.roots[k - 1], h->roots, k, (long long)S.st.hooks[k - 1]);
                return MSF_EDEVICE;
            }
        }
        ++S.rounds;
        if (nF) ++S.st.hook_rounds;
        if (S.compact) {
            const uint32_t nnz2 = h->nnz_out;
            S.live_frac = S.a.nnz ? (double)nnz2 / (double)S.a.nnz : 0.0;
            Adj nxt = S.a;
            nxt.row_ptr = S.b.rp[S.ai ^ 1];
            nxt.col = S.b.col[S.ai ^ 1];
            nxt.key = S.b.key[S.ai ^ 1];
            nxt.chunk_row = S.b.crow[S.ai ^ 1];
            for (int q = 0; q <= nxt.sl.S; ++q) nxt.sl.sstart[q] = h->sstart[q];
            set_chunks(&nxt);
            nxt.segs = h->segs;
            if (nnz2) launch_chunk_rows_sliced(s, nxt);
            S.a = nxt;
            S.ai ^= 1;
            ++S.st.filtered;
        } else {
            S.live_frac = S.a.nnz ? (double)h->live / (double)S.a.nnz : 0.0;
        }
        if (nF == 0) return enqueue_output(c);
        launch_chase(s, S.b.F, nF, S.b.h, S.b.hwk, S.wt, (uint32_t *)S.b.part, c->dcnt);
        if (c->check_rounds) {
            MSF_TRY(read_counters(c));
            if (c->hcnt->err) {
                set_error("internal error: hook cycle in round %d", S.rounds);
                return MSF_EDEVICE;
            }
        }
        // every vertex until the adjacency is filtered: a vertex without
        // entries keeps p = h = itself, and skipping the row pointers costs
        // less than reading them
        launch_update_parents(s, S.a.row_ptr, S.n, S.a.sl.S, S.b.p, S.b.h, (uint32_t *)S.b.part,
                              c->dcnt, c->check_rounds || S.st.filtered == 0);
        if (c->check_rounds) launch_check_stars(s, S.b.p, S.n, c->dcnt);
        S.ri ^= 1;
        S.nR = nRn;
        return more_rounds(S) ? enqueue_round(c) : enqueue_output(c);
    }
    case 4: {  // output ready
        if (h->err & ERR_STAR) {
            set_error("internal error: a tree is not a star after the last round");
            return MSF_EDEVICE;
        }
        if (h->err) {
            set_error("internal error: hook cycle detected");
            return MSF_EDEVICE;
        }
        float ms_build = 0.f, ms_rounds = 0.f;
        (void)hipEventElapsedTime(&ms_build, c->ev[0], c->ev[1]);
        (void)hipEventElapsedTime(&ms_rounds, c->ev[1], c->ev[2]);
        S.st.build_ms = ms_build;
        S.st.rounds_ms = ms_rounds;
        float ms_adj = 0.f;
        if (c->pass_done & 1u) (void)hipEventElapsedTime(&ms_adj, c->ev[0], c->kev[1]);
        S.st.adjacency_ms = ms_adj;
        // only the rounds that recorded their sweep events (none when the
        // rounds ran on the device)
        for (int k = 0; k < S.sweep_events; ++k) {
            float ms = 0.f;
            MSF_HIP(hipEventElapsedTime(&ms, c->sev[2 * k], c->sev[2 * k + 1]));
            S.st.sweep_ms[k] = ms;
        }
        const double nnz = (double)S.a.nnz;
        const double pass_bytes[4] = {
            nnz * (c->rec2 + c->sub2 + 12) + (double)S.n * (4.0 + (S.first_done ? 8.0 : 0.0)),
            13.0 * nnz + 16.0 * S.nruns + 4.0 * std::ceil(nnz / 64.0),
            nnz * (c->rec1 + c->rec2 + c->sub2),
            12.0 * (double)S.m + nnz * (c->rec1 + 1),
        };
        for (int q = 0; q < 4; ++q) {
            if (!(c->pass_done & (1u << q))) continue;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, c->kev[2 * q], c->kev[2 * q + 1]);
            S.st.pass_ms[q] = ms;
            S.st.pass_bytes[q] = pass_bytes[q];
        }
        S.st.max_chase = (int32_t)h->max_chase;
        c->stats = S.st;
        S.phase = 5;
        return MSF_OK;
    }
    default:
        set_error("solve_advance in phase %d", S.phase);
        return MSF_EINVAL;
    }
}

void solve_result(const Ctx *c, int64_t *count, msf_total *total)
{
    const SolveState &S = c->ss;
    const Counters *h = c->hcnt;
    *count = (S.m > 0) ? (int64_t)h->count : 0;
    if (total) {
        total->u64 = (S.wt == MSF_W_U32) ? h->total_u64 : 0;
        total->f64 = (S.m > 0) ? h->total_f64 : 0.0;
    }
}

msf_status solve_device(Ctx *c, int32_t n, int64_t m, const int32_t *d_edges, const void *d_w,
                        msf_wtype wt, int32_t *d_ids, int64_t *count, msf_total *total)
{
    MSF_TRY(solve_start(c, n, m, d_edges, d_w, wt, d_ids));
    while (!solve_done(c)) {
        MSF_HIP(hipEventSynchronize(c->ev[3]));
        MSF_TRY(solve_advance(c));
    }
    solve_result(c, count, total);
    return MSF_OK;
}

}  // namespace msf
