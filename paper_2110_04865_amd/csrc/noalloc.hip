// msf_solve_batched_noalloc: the batched solve for callers that cannot
// allocate device memory.
//
// Every scratch buffer of the persistent batched kernel (queue cursor,
// error and size words, the workgroups' live-edge lists and state slots)
// lives in `scratch`, one file-scope device array per GPU, held until the
// process ends.  Its device address is taken once per device with
// hipGetSymbolAddress when a context is created on that device, and only
// that address is ever used by host code.  A call clears the control words
// it relies on, checks every graph (offsets, endpoints, NaN weights, fit in
// a slot) in a validation pass before anything is solved, and then runs the
// persistent kernel with as many workgroups as the array holds slots for.
// Calls that overlap in time on one GPU share the array and race.
#include <algorithm>
#include <mutex>

#include "msf_internal.hpp"
#include "persist.hpp"
#include "wave.hpp"

namespace msf {

namespace {

constexpr size_t CTRL_BYTES = 256;
// control words: [0] queue, [1] error flags, [2] largest n, [3] largest m
enum { C_QUEUE = 0, C_ERR = 1, C_MAXN = 2, C_MAXM = 3, C_WORDS = 4 };
enum : uint32_t { ERR_SHAPE = 1u << 8 };  // bad offsets or a graph too large

__attribute__((used)) __device__ __align__(256) uint8_t scratch[MSF_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_ptr[MAX_DEVICES] = {};

__global__ void k_na_clear(uint32_t *ctl)
{
    if (threadIdx.x < C_WORDS) ctl[threadIdx.x] = 0;
}

// One workgroup per graph (grid-stride): offsets of graph g, its sizes
// against the persistent kernel's limits, then every edge's endpoints and
// weight.  The largest n and m go to the control words.
template <int WT>
__global__ __launch_bounds__(256) void k_na_validate(int32_t G, const int64_t *__restrict__ vo,
                                                     const int64_t *__restrict__ eo,
                                                     const int32_t *__restrict__ edges,
                                                     const uint32_t *__restrict__ w,
                                                     uint32_t *ctl)
{
    for (int32_t g = blockIdx.x; g < G; g += gridDim.x) {
        const int64_t v0 = vo[g], v1 = vo[g + 1], e0 = eo[g], e1 = eo[g + 1];
        const bool shape_ok = v0 >= 0 && e0 >= 0 && v1 >= v0 && e1 >= e0 &&
                              (g > 0 || (v0 == 0 && e0 == 0)) &&
                              v1 - v0 <= (int64_t)PERSIST_MAX_N &&
                              e1 - e0 <= (int64_t)PERSIST_MAX_M && v1 <= 0x7FFFFFFFll;
        if (!shape_ok) {
            if (threadIdx.x == 0) atomicOr(ctl + C_ERR, ERR_SHAPE);
            continue;
        }
        const uint32_t n = (uint32_t)(v1 - v0);
        if (threadIdx.x == 0) {
            atomicMax(ctl + C_MAXN, n);
            atomicMax(ctl + C_MAXM, (uint32_t)(e1 - e0));
        }
        uint32_t bad = 0;
        for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
            const uint32_t u = (uint32_t)edges[2 * e], v = (uint32_t)edges[2 * e + 1];
            if (u >= n || v >= n) bad |= ERR_ENDPOINT;
            if (WT == MSF_W_F32 && (w[e] & 0x7FFFFFFFu) > 0x7F800000u) bad |= ERR_NAN;
        }
        if (__ballot(bad != 0)) {
            for (int d = 32; d >= 1; d >>= 1) bad |= __shfl_xor(bad, d, 64);
            if (__lane_id() == 0) atomicOr(ctl + C_ERR, bad);
        }
    }
}

}  // namespace

msf_status noalloc_init(int device)
{
    if (device < 0 || device >= MAX_DEVICES) {
        set_error("device %d beyond the static scratch table", device);
        return MSF_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return MSF_OK;
    void *p = nullptr;
    MSF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
        set_error("no device address for the static scratch array");
        return MSF_EDEVICE;
    }
    g_ptr[device] = p;
    return MSF_OK;
}

}  // namespace msf

using namespace msf;

extern "C" msf_status msf_solve_batched_noalloc(msf_ctx *ctx, int32_t G, const int64_t *vtx_off,
                                                const int64_t *edge_off, const int32_t *edges,
                                                const void *weights, msf_wtype wt,
                                                int32_t *forest_ids, int64_t *counts,
                                                msf_total *totals)
{
    if (!ctx || G < 0 || (G > 0 && (!vtx_off || !edge_off || !counts || !totals))) {
        set_error("bad arguments");
        return MSF_EINVAL;
    }
    if (wt != MSF_W_U32 && wt != MSF_W_F32) {
        set_error("bad weight type");
        return MSF_EINVAL;
    }
    if (G == 0) return MSF_OK;
    Ctx *c = &ctx->c;
    MSF_HIP(hipSetDevice(c->device));
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (c->device >= 0 && c->device < MAX_DEVICES) base = g_ptr[c->device];
    }
    if (!base) {
        set_error("static scratch not set up on device %d", c->device);
        return MSF_EDEVICE;
    }
    hipStream_t s = c->stream;
    // totals of the batch: NULL arrays are allowed only where nothing is read
    // or written
    int64_t tail[2] = {0, 0};
    MSF_HIP(hipMemcpyAsync(&tail[0], vtx_off + G, 8, hipMemcpyDeviceToHost, s));
    MSF_HIP(hipMemcpyAsync(&tail[1], edge_off + G, 8, hipMemcpyDeviceToHost, s));
    MSF_HIP(hipStreamSynchronize(s));
    if ((tail[1] > 0 && (!edges || !weights)) || (tail[0] > 0 && !forest_ids)) {
        set_error("NULL edges, weights or forest_ids with a nonzero size");
        return MSF_EINVAL;
    }
    uint32_t *ctl = (uint32_t *)base;
    k_na_clear<<<1, 64, 0, s>>>(ctl);
    const unsigned vgrid = (unsigned)std::min<int64_t>(G, 4096);
    if (wt == MSF_W_F32)
        k_na_validate<MSF_W_F32><<<vgrid, 256, 0, s>>>(G, vtx_off, edge_off, edges,
                                                       (const uint32_t *)weights, ctl);
    else
        k_na_validate<MSF_W_U32><<<vgrid, 256, 0, s>>>(G, vtx_off, edge_off, edges,
                                                       (const uint32_t *)weights, ctl);
    MSF_HIP(hipGetLastError());
    uint32_t h[C_WORDS];
    MSF_HIP(hipMemcpyAsync(h, ctl, sizeof h, hipMemcpyDeviceToHost, s));
    MSF_HIP(hipStreamSynchronize(s));
    if (h[C_ERR] & ERR_SHAPE) {
        set_error("offsets must start at 0 and not decrease, and every graph must have at most "
                  "%u vertices and %u edges",
                  PERSIST_MAX_N, PERSIST_MAX_M);
        return MSF_EINVAL;
    }
    msf_status rc;
    if ((rc = decode_err(h[C_ERR]))) return rc;
    const size_t slot = persist_slot_bytes(std::max(h[C_MAXN], 1u), std::max(h[C_MAXM], 1u));
    const size_t room = MSF_NOALLOC_SCRATCH_BYTES - CTRL_BYTES;
    if (slot > room) {
        set_error("a graph needs %zu bytes of scratch; the static array holds %zu", slot, room);
        return MSF_EINVAL;
    }
    PersistCfg cfg{1024, 4, 64u << 10};
    if (persist_cfg_fits(c->device, PersistCfg{1024, 4, SMALL_LDS})) cfg.lds = SMALL_LDS;
    int cus = 0;
    MSF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
    const int bpc = std::max(1, persist_blocks_per_cu(cfg, (int)wt));
    const size_t slots = std::min<size_t>({room / slot, (size_t)G, (size_t)cus * bpc});
    PersistArgs A;
    A.G = G;
    A.order = nullptr;
    A.queue = ctl + C_QUEUE;
    A.err = ctl + C_ERR;
    A.vtx_off = vtx_off;
    A.edge_off = edge_off;
    A.edges = edges;
    A.w = (const uint32_t *)weights;
    A.out = forest_ids;
    A.counts = counts;
    A.tot_u64 = &totals[0].u64;
    A.tot_f64 = &totals[0].f64;
    A.tot_stride = sizeof(msf_total) / sizeof(uint64_t);
    A.scratch = (uint8_t *)base + CTRL_BYTES;
    A.slot_bytes = slot;
    A.m_cap = std::max(h[C_MAXM], 1u);
    A.lds_bytes = cfg.lds;
    MSF_HIP(launch_persist(s, A, cfg, (int)wt, (unsigned)slots));
    c->stats = msf_stats{};
    c->stats.batch_config = -1;
    c->stats.batch_grid = (int32_t)slots;
    c->stats.batch_graphs = G;
    return MSF_OK;
}
