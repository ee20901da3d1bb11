// Batched solve of many independent graphs.
//
// The disjoint union of the graphs is itself a graph whose minimum spanning
// forest is the union of their forests.  Vertex v of graph g becomes
// vtx_off[g] + v and edge e becomes edge_off[g] + e; since the offset is the
// same for every edge of a graph, keys (wkey, id) compare within a graph
// exactly as they do alone, so every per-graph result equals its solo solve.
// One round loop then advances all graphs at once: each sweep, hook and
// shortcut launch covers every graph, and a graph that is finished simply
// stops contributing live roots and (after filtering) stored entries.
#include <algorithm>
#include <vector>
#include <cstring>

#include "exact_sum.hpp"
#include "msf_internal.hpp"
#include "persist.hpp"
#include "wave.hpp"

namespace msf {

namespace {

__device__ __forceinline__ int32_t graph_of(const int64_t *__restrict__ off, int32_t G, int64_t x)
{
    // largest g with off[g] <= x (off[0] == 0, off[G] > x)
    int32_t lo = 0, hi = G - 1;
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo + 1) / 2;
        if (off[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace

// Local endpoints -> global ids; local ids outside [0, n_g) are rejected.
__global__ void k_globalize(const int32_t *__restrict__ edges, int64_t M,
                            const int64_t *__restrict__ vtx_off, const int64_t *__restrict__ edge_off,
                            int32_t G, int32_t *__restrict__ out, Counters *cnt)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < M; e += stride) {
        const int32_t g = graph_of(edge_off, G, e);
        const int64_t v0 = vtx_off[g];
        const int64_t ng = vtx_off[g + 1] - v0;
        const int32_t u = edges[2 * e], v = edges[2 * e + 1];
        const bool ok = u >= 0 && v >= 0 && (int64_t)u < ng && (int64_t)v < ng;
        bad |= !ok;
        out[2 * e] = ok ? (int32_t)(v0 + u) : -1;
        out[2 * e + 1] = ok ? (int32_t)(v0 + v) : -1;
    }
    if (__ballot(bad) && __lane_id() == 0) atomicOr(&cnt->err, ERR_ENDPOINT);
}

// One workgroup per graph: locate the graph's slice of the ascending global
// forest ids, write local ids from vtx_off[g], and total its weights (exact
// u64 for uint32; exact 32-bit-digit accumulation rounded once for float32).
template <int WT>
__global__ __launch_bounds__(256) void k_split(const int32_t *__restrict__ gids, int64_t count,
                                               const int64_t *__restrict__ vtx_off,
                                               const int64_t *__restrict__ edge_off,
                                               const void *__restrict__ w, int32_t *__restrict__ out,
                                               int64_t *__restrict__ counts,
                                               uint64_t *__restrict__ tot_u64,
                                               double *__restrict__ tot_f64)
{
    __shared__ int64_t s_sum[(256 / 64) * (ACC_DIGITS + 1)];
    __shared__ int64_t s_tot[WS_WORDS];
    const int32_t g = blockIdx.x;
    const int64_t e0 = edge_off[g], e1 = edge_off[g + 1];
    // lower bounds of e0 and e1 in gids[0..count)
    auto lb = [&](int64_t x) {
        int64_t lo = 0, hi = count;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)gids[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    const int64_t a = lb(e0), b = lb(e1);
    const int64_t base = vtx_off[g];
    WSum ws;
    for (int64_t k = a + threadIdx.x; k < b; k += blockDim.x) {
        const int64_t e = gids[k];
        out[base + (k - a)] = (int32_t)(e - e0);
        const uint32_t bits = ((const uint32_t *)w)[e];
        if (WT == MSF_W_U32) ws.su += bits;
        else wsum_add_bits(ws, bits);
    }
    wsum_block<256, WT>(ws, s_sum, s_tot, 1);
    if (threadIdx.x != 0) return;
    counts[g] = b - a;
    tot_u64[g] = WT == MSF_W_U32 ? (uint64_t)s_tot[0] : 0;
    tot_f64[g] = exact_total_f64((uint64_t)s_tot[0], s_tot + 1, (uint32_t)s_tot[1 + ACC_DIGITS],
                                 (uint32_t)s_tot[2 + ACC_DIGITS], WT);
}


// Batched solve by the persistent kernel (kernels_persist.hip) for every
// graph it takes, and one msf_solve-equivalent per graph for the rest.
// Writes each graph's ids into d_stage (device, at vtx_off[g]) and its
// count and totals into hres (host: counts, then u64 totals, then f64
// totals as bits); on any error nothing outside the workspace is written.
msf_status batched_persistent(Ctx *c, int32_t G, const int64_t *vtx_off, const int64_t *edge_off,
                              const int64_t *d_voff, const int64_t *d_eoff,
                              const int32_t *d_edges, const void *d_w, msf_wtype wt,
                              int32_t *d_stage, int64_t *d_counts, uint64_t *d_tu,
                              double *d_tf, int64_t *hres)
{
    hipStream_t s = c->stream;
    std::vector<uint32_t> order, large;
    uint32_t n_cap = 1, m_cap = 1;
    double sum_n = 0.0, sum_m = 0.0;
    for (int32_t g = 0; g < G; ++g) {
        const int64_t n = vtx_off[g + 1] - vtx_off[g], m = edge_off[g + 1] - edge_off[g];
        if (n <= (int64_t)PERSIST_MAX_N && m <= (int64_t)PERSIST_MAX_M) {
            order.push_back((uint32_t)g);
            n_cap = std::max(n_cap, (uint32_t)n);
            m_cap = std::max(m_cap, (uint32_t)m);
            sum_n += (double)n;
            sum_m += (double)m;
        } else {
            large.push_back((uint32_t)g);
        }
    }
    c->stats = msf_stats{};
    c->stats.batch_config = -1;
    c->stats.batch_graphs = (int64_t)order.size();
    c->stats.batch_large = (int64_t)large.size();
    const uint32_t Gs = (uint32_t)order.size();
    msf_status rc;
    if (Gs > 0) {
        // largest first, so the last graphs to start are the small ones
        std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
            const int64_t mx = edge_off[x + 1] - edge_off[x], my = edge_off[y + 1] - edge_off[y];
            if (mx != my) return mx > my;
            return vtx_off[x + 1] - vtx_off[x] > vtx_off[y + 1] - vtx_off[y];
        });
        // a sample with the batch's size mix for the tuner: every k-th graph
        std::vector<uint32_t> sample;
        const uint32_t step = std::max<uint32_t>(1, Gs / 256);
        for (uint32_t i = 0; i < Gs; i += step) sample.push_back(order[i]);
        int cus = 0;
        MSF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
        int ncand = 0;
        const PersistCfg *cand = persist_candidates(&ncand);
        std::vector<int> bpc(ncand, 0);
        uint32_t slots = 1;
        for (int i = 0; i < ncand; ++i) {
            if (!persist_cfg_fits(c->device, cand[i])) continue;
            bpc[i] = persist_blocks_per_cu(cand[i], wt);
            slots = std::max<uint32_t>(slots, (uint32_t)std::max(1, cus * bpc[i]));
        }
        // at most four workgroups per compute unit keep a slot (a slot holds
        // two live-edge lists of the largest graph: 32 bytes per edge)
        slots = std::min({slots, Gs, (uint32_t)std::max(1, 4 * cus)});
        const size_t slot_bytes = persist_slot_bytes(n_cap, m_cap);
        void *vord, *vctl, *vscr;
        if ((rc = ws_get(c, WS_PORDER, 4 * ((size_t)Gs + sample.size()), &vord))) return rc;
        if ((rc = ws_get(c, WS_PCTL, 256, &vctl))) return rc;
        if ((rc = ws_get(c, WS_PSCRATCH, slot_bytes * slots, &vscr))) return rc;
        uint32_t *d_order = (uint32_t *)vord, *d_sample = d_order + Gs;
        uint32_t *d_ctl = (uint32_t *)vctl;
        MSF_HIP(hipMemcpyAsync(d_order, order.data(), 4 * (size_t)Gs, hipMemcpyHostToDevice, s));
        MSF_HIP(hipMemcpyAsync(d_sample, sample.data(), 4 * sample.size(), hipMemcpyHostToDevice,
                               s));
        PersistArgs A;
        A.queue = d_ctl;
        A.err = d_ctl + 1;
        A.vtx_off = d_voff;
        A.edge_off = d_eoff;
        A.edges = d_edges;
        A.w = (const uint32_t *)d_w;
        A.out = d_stage;
        A.counts = d_counts;
        A.tot_u64 = d_tu;
        A.tot_f64 = d_tf;
        A.scratch = (uint8_t *)vscr;
        A.slot_bytes = slot_bytes;
        A.m_cap = m_cap;
        auto grid_of = [&](int i, uint32_t graphs) {
            return (unsigned)std::max<uint32_t>(
                1, std::min<uint32_t>({graphs, slots, (uint32_t)std::max(1, cus * bpc[i])}));
        };
        auto run = [&](int i, float *ms) -> msf_status {
            PersistArgs T = A;
            T.G = (int32_t)sample.size();
            T.order = d_sample;
            T.lds_bytes = cand[i].lds;
            if (ms) MSF_HIP(hipEventRecord(c->ev[0], s));
            MSF_HIP(launch_persist(s, T, cand[i], (int)wt, grid_of(i, T.G)));
            if (ms) {
                MSF_HIP(hipEventRecord(c->ev[1], s));
                MSF_HIP(hipEventSynchronize(c->ev[1]));
                MSF_HIP(hipEventElapsedTime(ms, c->ev[0], c->ev[1]));
            }
            return MSF_OK;
        };
        BatchShape shape;
        shape.mean_n = sum_n / Gs;
        shape.mean_deg = sum_n > 0 ? 2.0 * sum_m / sum_n : 0.0;
        int ci = 0;
        if ((rc = persist_pick(c, shape, (int)wt, run, &ci))) return rc;
        A.G = (int32_t)Gs;
        A.order = d_order;
        A.lds_bytes = cand[ci].lds;
        const unsigned grid = grid_of(ci, Gs);
        MSF_HIP(hipEventRecord(c->ev[0], s));
        MSF_HIP(launch_persist(s, A, cand[ci], (int)wt, grid));
        MSF_HIP(hipEventRecord(c->ev[1], s));
        c->stats.batch_config = ci;
        c->stats.batch_grid = (int32_t)grid;
    }
    MSF_HIP(hipMemcpyAsync(hres, d_counts, 24 * (size_t)G, hipMemcpyDeviceToHost, s));
    uint32_t herr = 0;
    if (Gs > 0) {
        void *vctl;
        if ((rc = ws_get(c, WS_PCTL, 256, &vctl))) return rc;
        MSF_HIP(hipMemcpyAsync(&herr, (uint32_t *)vctl + 1, 4, hipMemcpyDeviceToHost, s));
    }
    MSF_HIP(hipStreamSynchronize(s));
    if (Gs > 0) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
        c->stats.batch_ms = ms;
    }
    if ((rc = decode_err(herr))) return rc;
    // graphs too large for one workgroup: one solve each, into the staging
    for (uint32_t g : large) {
        const int64_t v0 = vtx_off[g], e0 = edge_off[g];
        int64_t cnt = 0;
        msf_total tot{0, 0.0};
        const msf_stats keep = c->stats;
        rc = solve_device(c, (int32_t)(vtx_off[g + 1] - v0), edge_off[g + 1] - e0,
                          d_edges + 2 * e0, (const uint32_t *)d_w + e0, wt, d_stage + v0, &cnt,
                          &tot);
        c->stats = keep;
        if (rc) return rc;
        hres[g] = cnt;
        hres[G + g] = (int64_t)tot.u64;
        std::memcpy(&hres[2 * (size_t)G + g], &tot.f64, sizeof(double));
    }
    return MSF_OK;
}


bool small_eligible(const Ctx *c, int32_t n, int64_t m)
{
    return c->small_m > 0 && m > 0 && m <= c->small_m && (uint32_t)n <= PERSIST_MAX_N &&
           persist_state_bytes((uint32_t)n, (uint32_t)m) <= SMALL_LDS &&
           persist_cfg_fits(c->device, PersistCfg{1024, 4, SMALL_LDS});
}

msf_status solve_small(Ctx *c, int32_t n, int64_t m, const int32_t *d_edges, const void *d_w,
                       msf_wtype wt, int32_t *d_ids, int64_t *count, msf_total *total)
{
    hipStream_t s = c->stream;
    c->ml_pending = false;
    void *vctl, *vscr;
    msf_status rc;
    if ((rc = ws_get(c, WS_PCTL, 512, &vctl))) return rc;
    if ((rc = ws_get(c, WS_PSCRATCH, persist_slot_bytes((uint32_t)n, (uint32_t)m), &vscr)))
        return rc;
    // control block: queue, error word; at byte 64 the offsets, then the
    // count, totals, the order and the per-round hooks
    uint8_t *ctl = (uint8_t *)vctl;
    PersistArgs A;
    A.G = 1;
    A.queue = (uint32_t *)ctl;
    A.err = (uint32_t *)ctl + 1;
    A.vtx_off = (int64_t *)(ctl + 64);
    A.edge_off = (int64_t *)(ctl + 80);
    A.counts = (int64_t *)(ctl + 96);
    A.tot_u64 = (uint64_t *)(ctl + 104);
    A.tot_f64 = (double *)(ctl + 112);
    A.order = (uint32_t *)(ctl + 120);
    A.round_hooks = (uint32_t *)(ctl + 128);
    A.edges = d_edges;
    A.w = (const uint32_t *)d_w;
    A.out = d_ids;
    A.scratch = (uint8_t *)vscr;
    A.slot_bytes = persist_slot_bytes((uint32_t)n, (uint32_t)m);
    A.m_cap = (uint32_t)m;
    A.lds_bytes = SMALL_LDS;
    launch_small_setup(s, (int64_t *)A.vtx_off, (int64_t *)A.edge_off, (uint32_t *)A.order, n, m);
    MSF_HIP(hipEventRecord(c->ev[0], s));
    MSF_HIP(launch_persist(s, A, PersistCfg{1024, 4, SMALL_LDS}, (int)wt, 1));
    MSF_HIP(hipEventRecord(c->ev[1], s));
    alignas(8) uint8_t h[512];
    MSF_HIP(hipMemcpyAsync(h, ctl, 512, hipMemcpyDeviceToHost, s));
    MSF_HIP(hipStreamSynchronize(s));
    uint32_t err;
    std::memcpy(&err, h + 4, 4);
    if ((rc = decode_err(err))) return rc;
    const uint32_t *hooks = (const uint32_t *)(h + 128);
    msf_stats st{};
    st.batch_config = -1;
    st.path = 1;
    st.rounds = (int32_t)hooks[64];
    for (int k = 0; k < st.rounds && k < 64; ++k) {
        st.hooks[k] = hooks[k];
        st.hook_rounds += hooks[k] != 0;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
    st.rounds_ms = ms;
    c->stats = st;
    std::memcpy(count, h + 96, 8);
    if (total) {
        std::memcpy(&total->u64, h + 104, 8);
        std::memcpy(&total->f64, h + 112, 8);
    }
    return MSF_OK;
}

}  // namespace msf

using namespace msf;

extern "C" msf_status msf_solve_batched(msf_ctx *ctx, int32_t G, const int64_t *vtx_off,
                                        const int64_t *edge_off, const int32_t *edges,
                                        const void *weights, msf_wtype wt, msf_mem mem,
                                        int32_t *forest_ids, int64_t *counts, msf_total *totals)
{
    if (!ctx || G < 0 || (G > 0 && (!vtx_off || !edge_off || !counts))) {
        set_error("bad arguments");
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
    if (G == 0) return MSF_OK;
    if (vtx_off[0] != 0 || edge_off[0] != 0) {
        set_error("offsets must start at 0");
        return MSF_EINVAL;
    }
    for (int32_t g = 0; g < G; ++g) {
        if (vtx_off[g + 1] < vtx_off[g] || edge_off[g + 1] < edge_off[g]) {
            set_error("offsets must be non-decreasing (graph %d)", (int)g);
            return MSF_EINVAL;
        }
    }
    const int64_t N = vtx_off[G], M = edge_off[G];
    if (N > 0x7FFFFFFFll || M > MSF_MAX_EDGES) {
        set_error("batch too large: %lld vertices, %lld edges", (long long)N, (long long)M);
        return MSF_EINVAL;
    }
    if (M > 0 && (!edges || !weights)) {
        set_error("NULL edges/weights");
        return MSF_EINVAL;
    }
    if (N > 0 && !forest_ids) {
        set_error("NULL forest_ids");
        return MSF_EINVAL;
    }
    Ctx *c = &ctx->c;
    MSF_HIP(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const size_t mm = (size_t)std::max<int64_t>(M, 1), nn = (size_t)std::max<int64_t>(N, 1);
    void *voff, *vge = nullptr, *vgid, *vout = nullptr, *vw = nullptr, *vin = nullptr, *vres;
    msf_status rc;
    if ((rc = ws_get(c, WS_BATCH0, 8 * 2 * (size_t)(G + 1), &voff))) return rc;
    if ((rc = ws_get(c, WS_BATCH2, 4 * nn, &vgid))) return rc;
    if ((rc = ws_get(c, WS_BATCH3, (8 + 8 + 8) * (size_t)G, &vres))) return rc;
    int64_t *d_voff = (int64_t *)voff, *d_eoff = d_voff + (G + 1);
    MSF_HIP(hipMemcpyAsync(d_voff, vtx_off, 8 * (size_t)(G + 1), hipMemcpyHostToDevice, s));
    MSF_HIP(hipMemcpyAsync(d_eoff, edge_off, 8 * (size_t)(G + 1), hipMemcpyHostToDevice, s));
    const int32_t *d_edges = edges;
    const void *d_w = weights;
    int32_t *d_out = forest_ids;
    if (mem == MSF_MEM_HOST) {
        if ((rc = ws_get(c, WS_EDGES, 8 * mm, &vin))) return rc;
        if ((rc = ws_get(c, WS_W, 4 * mm, &vw))) return rc;
        if (c->batch_mode == 0 && (rc = ws_get(c, WS_IDS, 4 * nn, &vout))) return rc;
        if (M > 0) {
            MSF_HIP(hipMemcpyAsync(vin, edges, 8 * (size_t)M, hipMemcpyHostToDevice, s));
            MSF_HIP(hipMemcpyAsync(vw, weights, 4 * (size_t)M, hipMemcpyHostToDevice, s));
        }
        d_edges = (const int32_t *)vin;
        d_w = vw;
        d_out = (int32_t *)vout;
    }
    int64_t *d_counts = (int64_t *)vres;
    uint64_t *d_tu = (uint64_t *)(d_counts + G);
    double *d_tf = (double *)(d_tu + G);
    std::vector<int64_t> hres(3 * (size_t)G);
    if (c->batch_mode == 0) {
        // the disjoint union through the round loop of msf_solve
        if ((rc = ws_get(c, WS_BATCH1, 8 * mm, &vge))) return rc;
        launch_fill_u32(s, &c->dcnt->err, 0u, 1);
        if (M > 0) {
            size_t g = (size_t)(M + 255) / 256;
            k_globalize<<<(unsigned)std::min<size_t>(g, 16384), 256, 0, s>>>(
                d_edges, M, d_voff, d_eoff, G, (int32_t *)vge, c->dcnt);
        }
        MSF_HIP(hipGetLastError());
        if ((rc = read_counters(c))) return rc;
        if (c->hcnt->err & ERR_ENDPOINT) {
            set_error("edge endpoint outside its graph's vertex range");
            return MSF_EINVAL;
        }
        int64_t cnt = 0;
        msf_total tot;
        rc = solve_device(c, (int32_t)N, M, (const int32_t *)vge, d_w, wt, (int32_t *)vgid, &cnt,
                          &tot);
        if (rc) return rc;
        if (wt == MSF_W_F32)
            k_split<MSF_W_F32><<<G, 256, 0, s>>>((const int32_t *)vgid, cnt, d_voff, d_eoff, d_w,
                                                 d_out, d_counts, d_tu, d_tf);
        else
            k_split<MSF_W_U32><<<G, 256, 0, s>>>((const int32_t *)vgid, cnt, d_voff, d_eoff, d_w,
                                                 d_out, d_counts, d_tu, d_tf);
        MSF_HIP(hipGetLastError());
        MSF_HIP(hipMemcpyAsync(hres.data(), vres, 24 * (size_t)G, hipMemcpyDeviceToHost, s));
        c->stats = msf_stats{};
        c->stats.batch_config = -1;
    } else {
        // persistent launch into the staging buffer (vgid); the caller's
        // forest ids are written only once every graph has succeeded
        rc = batched_persistent(c, G, vtx_off, edge_off, d_voff, d_eoff, d_edges, d_w, wt,
                                (int32_t *)vgid, d_counts, d_tu, d_tf, hres.data());
        if (rc) return rc;
        if (mem == MSF_MEM_HOST) d_out = (int32_t *)vgid;  // downloaded from there below
        else if (N > 0)
            MSF_HIP(hipMemcpyAsync(d_out, vgid, 4 * (size_t)N, hipMemcpyDeviceToDevice, s));
    }
    if (mem == MSF_MEM_HOST && N > 0)
        MSF_HIP(hipMemcpyAsync(forest_ids, d_out, 4 * (size_t)N, hipMemcpyDeviceToHost, s));
    MSF_HIP(hipStreamSynchronize(s));
    for (int32_t g = 0; g < G; ++g) {
        counts[g] = hres[g];
        if (totals) {
            totals[g].u64 = (uint64_t)hres[G + g];
            double f;
            std::memcpy(&f, &hres[2 * (size_t)G + g], sizeof f);
            totals[g].f64 = f;
        }
    }
    return MSF_OK;
}
