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

#include "msf_internal.hpp"
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
    constexpr int D = 10;
    __shared__ int64_t s_acc[D][4];
    __shared__ uint64_t s_u[4];
    __shared__ uint32_t s_inf[2];
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
    uint64_t su = 0;
    int64_t acc[D];
#pragma unroll
    for (int d = 0; d < D; ++d) acc[d] = 0;
    uint32_t pinf = 0, ninf = 0;
    for (int64_t k = a + threadIdx.x; k < b; k += blockDim.x) {
        const int64_t e = gids[k];
        out[base + (k - a)] = (int32_t)(e - e0);
        const uint32_t bits = ((const uint32_t *)w)[e];
        if (WT == MSF_W_U32) {
            su += bits;
        } else {
            const uint32_t ex = (bits >> 23) & 0xFFu;
            const bool neg = (bits >> 31) != 0;
            if (ex == 0xFFu) {
                if (neg) ++ninf;
                else ++pinf;
                continue;
            }
            const uint64_t mant = ex ? ((bits & 0x7FFFFFu) | 0x800000u) : (bits & 0x7FFFFFu);
            const uint32_t sh = ex ? ex - 1u : 0u;
            const uint64_t x = mant << (sh & 31u);
            const uint32_t di = sh >> 5;
            const int64_t lo = (int64_t)(x & 0xFFFFFFFFull), hi = (int64_t)(x >> 32);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                int64_t add = (d == (int)di) ? lo : ((d == (int)di + 1) ? hi : 0);
                acc[d] += neg ? -add : add;
            }
        }
    }
    const int wv = threadIdx.x >> 6;
    if (WT == MSF_W_U32) {
        su = wave_sum(su);
        if (__lane_id() == 0) s_u[wv] = su;
    } else {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int64_t v = wave_sum(acc[d]);
            if (__lane_id() == 0) s_acc[d][wv] = v;
        }
        pinf = wave_sum(pinf);
        ninf = wave_sum(ninf);
        if (threadIdx.x == 0) s_inf[0] = s_inf[1] = 0;
    }
    __syncthreads();
    if (WT != MSF_W_U32 && __lane_id() == 0 && (pinf | ninf)) {
        atomicAdd(&s_inf[0], pinf);
        atomicAdd(&s_inf[1], ninf);
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    counts[g] = b - a;
    if (WT == MSF_W_U32) {
        const uint64_t s = s_u[0] + s_u[1] + s_u[2] + s_u[3];
        tot_u64[g] = s;
        tot_f64[g] = (double)s;
        return;
    }
    tot_u64[g] = 0;
    if (s_inf[0] || s_inf[1]) {
        tot_f64[g] = (s_inf[0] && s_inf[1]) ? __builtin_nan("")
                     : (s_inf[0] ? __builtin_inf() : -__builtin_inf());
        return;
    }
    uint32_t dig[D];
    int64_t carry = 0;
    for (int d = 0; d < D; ++d) {
        const int64_t v = s_acc[d][0] + s_acc[d][1] + s_acc[d][2] + s_acc[d][3] + carry;
        dig[d] = (uint32_t)(v & 0xFFFFFFFFll);
        carry = v >> 32;
    }
    const bool neg = carry < 0;
    if (neg) {
        uint64_t c = 1;
        for (int d = 0; d < D; ++d) {
            const uint64_t v = (uint64_t)(uint32_t)~dig[d] + c;
            dig[d] = (uint32_t)v;
            c = v >> 32;
        }
    }
    int top = -1;
    for (int d = D - 1; d >= 0 && top < 0; --d)
        if (dig[d]) top = d * 32 + 31 - __builtin_clz(dig[d]);
    double outv = 0.0;
    if (top >= 0) {
        auto bit = [&](int i) -> uint32_t { return i < 0 ? 0u : (dig[i >> 5] >> (i & 31)) & 1u; };
        uint64_t q = 0;
        const int lo = top - 52;
        int scale = lo;
        if (lo < 0) {
            scale = 0;
            for (int i = top; i >= 0; --i) q = (q << 1) | bit(i);
        } else {
            for (int i = top; i >= lo; --i) q = (q << 1) | bit(i);
            const uint32_t rb = bit(lo - 1);
            uint32_t sticky = 0;
            for (int i = lo - 2; i >= 0 && !sticky; --i) sticky |= bit(i);
            if (rb && (sticky || (q & 1u))) {
                ++q;
                if (q == (1ull << 53)) {
                    q >>= 1;
                    ++scale;
                }
            }
        }
        outv = ldexp((double)q, scale - 149);
    }
    tot_f64[g] = neg ? -outv : outv;
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
    void *voff, *vge, *vgid, *vout, *vw = nullptr, *vin = nullptr, *vres;
    msf_status rc;
    if ((rc = ws_get(c, WS_BATCH0, 8 * 2 * (size_t)(G + 1), &voff))) return rc;
    if ((rc = ws_get(c, WS_BATCH1, 8 * mm, &vge))) return rc;
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
        if ((rc = ws_get(c, WS_IDS, 4 * nn, &vout))) return rc;
        if (M > 0) {
            MSF_HIP(hipMemcpyAsync(vin, edges, 8 * (size_t)M, hipMemcpyHostToDevice, s));
            MSF_HIP(hipMemcpyAsync(vw, weights, 4 * (size_t)M, hipMemcpyHostToDevice, s));
        }
        d_edges = (const int32_t *)vin;
        d_w = vw;
        d_out = (int32_t *)vout;
    }
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
    rc = solve_device(c, (int32_t)N, M, (const int32_t *)vge, d_w, wt, (int32_t *)vgid, &cnt, &tot);
    if (rc) return rc;
    int64_t *d_counts = (int64_t *)vres;
    uint64_t *d_tu = (uint64_t *)(d_counts + G);
    double *d_tf = (double *)(d_tu + G);
    if (wt == MSF_W_F32)
        k_split<MSF_W_F32><<<G, 256, 0, s>>>((const int32_t *)vgid, cnt, d_voff, d_eoff, d_w, d_out,
                                             d_counts, d_tu, d_tf);
    else
        k_split<MSF_W_U32><<<G, 256, 0, s>>>((const int32_t *)vgid, cnt, d_voff, d_eoff, d_w, d_out,
                                             d_counts, d_tu, d_tf);
    MSF_HIP(hipGetLastError());
    std::vector<int64_t> hres(3 * (size_t)G);
    MSF_HIP(hipMemcpyAsync(hres.data(), vres, 24 * (size_t)G, hipMemcpyDeviceToHost, s));
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
