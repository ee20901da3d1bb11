// Persistent batched solve: one workgroup runs every round of one graph.
//
// A batch of many small and medium graphs (the batched pattern) is solved
// by one launch of a persistent grid (a few workgroups per compute unit).
// Each workgroup takes graphs from a queue, largest first, and runs
// Algorithm 2 with complete shortcutting (section 4.2) on its graph alone,
// with a workgroup barrier between the steps of a round and a per-graph
// termination test, so no round boundary involves the host:
//
//   sweep     the multilinear kernel of section 3.1 with the projection of
//             Algorithm 2, over the graph's edge list: an edge {u, v} with
//             key k and roots a = p[u] != b = p[v] lowers r[a] and r[b] to k
//             (both stored directions of the adjacency matrix at once).
//             From the second round on, the sweep also writes the edges it
//             found live, as (a, b, key), and the next round sweeps only
//             those (their endpoints are roots of the previous round, whose
//             parents are the current roots): intra-component edges are
//             filtered out round by round.
//   hook      every root with r != empty hooks onto the root at the other
//             end of its minimum edge (Algorithm 2, hooking step);
//   tie break of two roots that hooked onto each other, the smaller id
//             stays root (Algorithm 2, tie-breaking step; section 2.3); the
//             kept hooks' edges are flagged and their weights summed;
//   shortcut  pointer jumping over the hook forest until every tree is a
//             star (complete shortcutting, section 4.2), then p <- h[p];
//   stop      after a round in which nothing hooks.
//
// State of a graph with n vertices and m edges: r u64[n], p u32[n] (a
// parent chain: a vertex that stops being a root points to the root that
// absorbed it), h u32[n], the list of roots that can still hook u32[n] and
// the forest flags as a bitmask u32[ceil(m/32)], in LDS when
// 20 n + 4 ceil(m/32) bytes fit the launch's dynamic LDS, else in the
// workgroup's slot of a global scratch area (same code, the address space
// is fixed per instantiation).  The live-edge lists of the later rounds
// (16 bytes per edge, two buffers) are always in the slot.  Keys use the
// graph's local edge ids, so each graph's forest is the one msf_solve finds
// on that graph alone.  Outputs: the forest's local edge ids in ascending
// order from out + vtx_off[g], count and exact totals.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "exact_sum.hpp"
#include "msf_internal.hpp"
#include "persist.hpp"
#include "wave.hpp"

// Graphs whose state does not fit the launch's LDS keep their parent
// vector there as 16-bit ids when it fits (1).
#ifndef PERSIST_P16
#define PERSIST_P16 1
#endif

namespace msf {

namespace {

// One live edge of a later round: roots of the previous round and the key.
struct __align__(16) LiveEdge {
    uint32_t a, b;
    uint64_t key;
};

__device__ __forceinline__ uint64_t ld_min_u64(uint64_t *p, uint64_t v)
{
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// r[i] <- min(r[i], key) where a read of r[i] (cur) shows that the key can
// lower it: r only decreases during a sweep, so a stale read can cost an
// atomic, never a miss, and most atomics are skipped (measured: sending
// every atomic to global memory made the sweep 3x slower).
__device__ __forceinline__ void lower(uint64_t *r, uint32_t i, uint64_t cur, uint64_t key)
{
    if (key < cur) ld_min_u64(r + i, key);
}

__device__ __forceinline__ uint32_t weight_key(uint32_t bits, int wt)
{
    return wt == MSF_W_F32 ? wkey_f32_bits(bits) : bits;
}

// Shared control words of a workgroup.
struct Ctl {
    uint32_t g;          // graph being solved (NONE32: queue empty)
    uint32_t live;       // live edges written by the current sweep
    uint32_t hooks;      // kept hooks of the current round
    uint32_t changed[2]; // shortcut passes, alternating
    uint32_t err;        // ERR_* seen by this workgroup
    uint32_t gerr;       // the current graph failed validation
};

// P16: the state is in the workgroup's slot except p, which is kept in LDS
// as 16-bit vertex ids (pstate; graphs of at most 2^16 vertices): the sweep
// looks up p at both ends of every edge, and the hook follows p chains.
template <int NT, int EPT, int WT, bool IN_LDS, bool P16>
__device__ __forceinline__ void solve_graph(const PersistArgs &A, uint32_t g, uint8_t *state,
                                            uint16_t *pstate, LiveEdge *buf0, LiveEdge *buf1,
                                            Ctl &ctl, int64_t *s_sum, int64_t *s_tot,
                                            uint32_t *s_scan)
{
    static_assert(!(IN_LDS && P16), "p in LDS on its own only when the rest is not");
    using PT = typename std::conditional<P16, uint16_t, uint32_t>::type;
    const uint32_t tid = threadIdx.x;
    const int64_t v0 = A.vtx_off[g];
    const uint32_t n = (uint32_t)(A.vtx_off[g + 1] - v0);
    const int64_t e0 = A.edge_off[g];
    const uint32_t m = (uint32_t)(A.edge_off[g + 1] - e0);
    const uint32_t nw = (m + 31) / 32;
    // r: root minima; p: parent chain (a root points to itself; a vertex
    // that stopped being a root points to the root that absorbed it, after
    // that round's shortcut); h: hook targets; L: the current roots
    uint64_t *r = reinterpret_cast<uint64_t *>(state);
    PT *p;
    uint32_t *h;
    if constexpr (P16) {
        p = pstate;
        h = reinterpret_cast<uint32_t *>(state + 8 * (size_t)n);
    } else {
        p = reinterpret_cast<PT *>(state + 8 * (size_t)n);
        h = reinterpret_cast<uint32_t *>(p + n);
    }
    uint32_t *L = h + n;
    uint32_t *fb = L + n;
    const int2 *E = reinterpret_cast<const int2 *>(A.edges) + e0;
    const uint32_t *W = A.w + e0;

    for (uint32_t i = tid; i < n; i += NT) {
        r[i] = KEY_INF;
        p[i] = (PT)i;
        L[i] = i;
    }
    uint32_t nroots = n;
    for (uint32_t k = tid; k < nw; k += NT) fb[k] = 0u;
    if (tid == 0) ctl.gerr = 0;
    uint32_t err = 0;
    WSum ws;
    uint32_t nlive = m;
    __syncthreads();

    for (uint32_t round = 0;; ++round) {
        if (tid == 0) {
            ctl.live = 0;
            ctl.hooks = 0;
        }
        __syncthreads();
        // ---- sweep -------------------------------------------------------
        LiveEdge *dst = (round & 1) ? buf0 : buf1;
        const LiveEdge *src = (round & 1) ? buf1 : buf0;
        // Each step of a sweep runs in phases over the thread's EPT edges:
        // every load first, then the parent lookups, then the minima, so
        // the loads of all EPT edges are in flight together.  Indices past
        // the end are clamped (the loads stay in bounds) and the edge is
        // masked off.
        if (round <= 1) {
            for (uint32_t base = 0; base < m; base += NT * EPT) {
                int2 uv[EPT];
                uint32_t wb[EPT];
#pragma unroll
                for (int k = 0; k < EPT; ++k) {
                    const uint32_t e = base + k * NT + tid;
                    const uint32_t ec = e < m ? e : m - 1;
                    uv[k] = E[ec];
                    wb[k] = W[ec];
                }
                uint32_t a[EPT], b[EPT];
                bool ok[EPT];
#pragma unroll
                for (int k = 0; k < EPT; ++k) {
                    const uint32_t e = base + k * NT + tid;
                    a[k] = (uint32_t)uv[k].x;
                    b[k] = (uint32_t)uv[k].y;
                    ok[k] = e < m;
                    if (ok[k] && (a[k] >= n || b[k] >= n)) {
                        err |= ERR_ENDPOINT;
                        ok[k] = false;
                    }
                    if (ok[k] && WT == MSF_W_F32 && (wb[k] & 0x7FFFFFFFu) > 0x7F800000u) {
                        err |= ERR_NAN;
                        ok[k] = false;
                    }
                    if (!ok[k]) a[k] = b[k] = 0;
                }
                if (round == 1) {
#pragma unroll
                    for (int k = 0; k < EPT; ++k) {
                        a[k] = p[a[k]];
                        b[k] = p[b[k]];
                    }
                }
                uint64_t ra[EPT], rb[EPT];
#pragma unroll
                for (int k = 0; k < EPT; ++k) {
                    ra[k] = r[a[k]];
                    rb[k] = r[b[k]];
                }
#pragma unroll
                for (int k = 0; k < EPT; ++k) {
                    const uint32_t e = base + k * NT + tid;
                    const uint64_t key = ((uint64_t)weight_key(wb[k], WT) << 32) | e;
                    const bool live = ok[k] && a[k] != b[k];
                    if (live) {
                        lower(r, a[k], ra[k], key);
                        lower(r, b[k], rb[k], key);
                    }
                    if (round == 1) {
                        // keep the live edges for the next round
                        const uint64_t mask = __ballot(live);
                        uint32_t at = 0;
                        if (__lane_id() == 0 && mask)
                            at = atomicAdd(&ctl.live, (uint32_t)__popcll(mask));
                        at = __shfl(at, 0, 64);
                        if (live)
                            dst[at + __popcll(mask & lanemask_lt())] = LiveEdge{a[k], b[k], key};
                    }
                }
            }
        } else {
            for (uint32_t base = 0; base < nlive; base += NT * EPT) {
                LiveEdge x[EPT];
#pragma unroll
                for (int k = 0; k < EPT; ++k) {
                    const uint32_t j = base + k * NT + tid;
                    x[k] = src[j < nlive ? j : nlive - 1];
                }
                uint32_t a[EPT], b[EPT];
#pragma unroll
                for (int k = 0; k < EPT; ++k) {
                    a[k] = p[x[k].a];
                    b[k] = p[x[k].b];
                }
                uint64_t ra[EPT], rb[EPT];
#pragma unroll
                for (int k = 0; k < EPT; ++k) {
                    ra[k] = r[a[k]];
                    rb[k] = r[b[k]];
                }
#pragma unroll
                for (int k = 0; k < EPT; ++k) {
                    const uint32_t j = base + k * NT + tid;
                    const bool live = j < nlive && a[k] != b[k];
                    if (live) {
                        lower(r, a[k], ra[k], x[k].key);
                        lower(r, b[k], rb[k], x[k].key);
                    }
                    const uint64_t mask = __ballot(live);
                    uint32_t at = 0;
                    if (__lane_id() == 0 && mask)
                        at = atomicAdd(&ctl.live, (uint32_t)__popcll(mask));
                    at = __shfl(at, 0, 64);
                    if (live)
                        dst[at + __popcll(mask & lanemask_lt())] = LiveEdge{a[k], b[k], x[k].key};
                }
            }
        }
        __syncthreads();
        if (round >= 1) nlive = ctl.live;
        // ---- hook: every root onto the root across its minimum edge ------
        // The other endpoint's root at the start of this round is the end
        // of its parent chain (one step per round since it stopped being a
        // root); p is not written in this step, so the chains are stable.
        for (uint32_t k = tid; k < nroots; k += NT) {
            const uint32_t i = L[k];
            const uint64_t key = r[i];
            uint32_t t = i;
            if (key != KEY_INF) {
                const int2 uv = E[(uint32_t)key];
                uint32_t a = (uint32_t)uv.x, b = (uint32_t)uv.y;
                while (p[a] != a) a = p[a];
                while (p[b] != b) b = p[b];
                t = a == i ? b : a;
            }
            h[i] = t;
        }
        __syncthreads();
        // ---- tie break, forest flags and weights -------------------------
        // The larger root of a mutual pair never reverts, whatever it reads,
        // so reverting the smaller one in place is race-free.
        uint32_t kept = 0;
        for (uint32_t k = tid; k < nroots; k += NT) {
            const uint32_t i = L[k];
            const uint32_t t = h[i];
            if (t == i) continue;
            if (i < t && h[t] == i) {
                h[i] = i;
                continue;
            }
            const uint64_t key = r[i];
            const uint32_t e = (uint32_t)key;
            atomicOr(fb + (e >> 5), 1u << (e & 31));
            wsum_add<WT>(ws, (uint32_t)(key >> 32));
            ++kept;
        }
        kept = wave_sum(kept);
        if (__lane_id() == 0 && kept) atomicAdd(&ctl.hooks, kept);
        __syncthreads();
        if (A.round_hooks && tid == 0 && round < 64) A.round_hooks[round] = ctl.hooks;
        if (ctl.hooks == 0) {
            if (A.round_hooks && tid == 0) A.round_hooks[64] = round + 1;
            break;
        }
        // the roots that can still hook at least halve every round, so a
        // graph of at most 2^31 vertices needs fewer than 33 rounds
        if (round >= 40) {
            err |= ERR_CYCLE;
            break;
        }
        // ---- complete shortcutting over the roots ------------------------
        for (uint32_t pass = 0;; ++pass) {
            if (tid == 0) ctl.changed[pass & 1] = 0;
            __syncthreads();
            uint32_t any = 0;
            for (uint32_t k = tid; k < nroots; k += NT) {
                const uint32_t i = L[k];
                const uint32_t x = h[i];
                const uint32_t y = h[x];
                if (y != x) {
                    h[i] = y;
                    any = 1;
                }
            }
            if (__ballot(any) && __lane_id() == 0) ctl.changed[pass & 1] = 1;
            __syncthreads();
            if (!ctl.changed[pass & 1]) break;
            if (pass > 64) {  // the hook forest is acyclic: cannot happen
                err |= ERR_CYCLE;
                break;
            }
        }
        if (err & ERR_CYCLE) break;
        // ---- p <- h at the old roots; the roots that stay, compacted -----
        // in place, one tile at a time: every read of a tile happens before
        // the barrier, and writes land below the tile's end (at most as
        // many roots stay as were read so far)
        if (tid == 0) ctl.live = 0;
        __syncthreads();
        for (uint32_t base = 0; base < nroots; base += NT) {
            const uint32_t k = base + tid;
            const uint32_t i = k < nroots ? L[k] : NONE32;
            bool stay = false;
            if (i != NONE32) {
                const uint32_t t = h[i];
                p[i] = (PT)t;
                // a root without an outgoing edge spans its whole component:
                // no edge can reach it again, so it leaves the list
                stay = t == i && r[i] != KEY_INF;
                r[i] = KEY_INF;
            }
            __syncthreads();
            const uint64_t mask = __ballot(stay);
            uint32_t at = 0;
            if (__lane_id() == 0 && mask) at = atomicAdd(&ctl.live, (uint32_t)__popcll(mask));
            at = __shfl(at, 0, 64);
            if (stay) L[at + __popcll(mask & lanemask_lt())] = i;
        }
        __syncthreads();
        nroots = ctl.live;
        __syncthreads();
    }

    // ---- output: ascending forest ids, count, totals ----------------------
    // a graph that failed validation writes no ids (the call fails); its
    // count is minus its error flags
    if (err) atomicOr(&ctl.gerr, err);
    __syncthreads();
    const bool bad = ctl.gerr != 0;
    // each thread owns a contiguous range of flag words
    const uint32_t per = (nw + NT - 1) / NT;
    const uint32_t w_lo = tid * per, w_hi = min(nw, w_lo + per);
    uint32_t cnt = 0;
    for (uint32_t k = w_lo; k < w_hi; ++k) cnt += __popc(fb[k]);
    uint32_t total;
    uint32_t pos = block_excl_sum<NT>(cnt, s_scan, &total);
    int32_t *out = A.out + v0;
    for (uint32_t k = w_lo; k < w_hi && !bad; ++k) {
        uint32_t bits = fb[k];
        while (bits) {
            const uint32_t b = __builtin_ctz(bits);
            bits &= bits - 1;
            out[pos++] = (int32_t)(k * 32 + b);
        }
    }
    wsum_block<NT, WT>(ws, s_sum, s_tot, 1);
    if (err) atomicOr(&ctl.err, err);
    if (tid == 0) {
        A.counts[g] = bad ? -(int64_t)ctl.gerr : (int64_t)total;
        A.tot_u64[(size_t)g * A.tot_stride] = WT == MSF_W_U32 ? (uint64_t)s_tot[0] : 0;
        A.tot_f64[(size_t)g * A.tot_stride] = exact_total_f64((uint64_t)s_tot[0], s_tot + 1,
                                       (uint32_t)s_tot[1 + ACC_DIGITS],
                                       (uint32_t)s_tot[2 + ACC_DIGITS], WT);
    }
    __syncthreads();
}

}  // namespace

template <int NT, int EPT, int WT>
__global__ __launch_bounds__(NT) void k_persist(PersistArgs A)
{
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ Ctl ctl;
    __shared__ int64_t s_sum[(NT / 64) * (ACC_DIGITS + 1)];
    __shared__ int64_t s_tot[WS_WORDS];
    __shared__ uint32_t s_scan[NT / 64 + 1];
    uint8_t *slot = A.scratch + (size_t)blockIdx.x * A.slot_bytes;
    LiveEdge *buf0 = reinterpret_cast<LiveEdge *>(slot);
    LiveEdge *buf1 = buf0 + A.m_cap;
    uint8_t *gstate = reinterpret_cast<uint8_t *>(buf1 + A.m_cap);
    if (threadIdx.x == 0) ctl.err = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t k = atomicAdd(A.queue, 1u);
            ctl.g = k < (uint32_t)A.G ? (A.order ? A.order[k] : k) : NONE32;
        }
        __syncthreads();
        const uint32_t g = ctl.g;
        if (g == NONE32) break;
        const uint32_t n = (uint32_t)(A.vtx_off[g + 1] - A.vtx_off[g]);
        const uint32_t m = (uint32_t)(A.edge_off[g + 1] - A.edge_off[g]);
        if (persist_state_bytes(n, m) <= A.lds_bytes)
            solve_graph<NT, EPT, WT, true, false>(A, g, smem, nullptr, buf0, buf1, ctl, s_sum,
                                                  s_tot, s_scan);
        else if (PERSIST_P16 && n <= 65536u && 2 * (size_t)n <= A.lds_bytes)
            solve_graph<NT, EPT, WT, false, true>(A, g, gstate,
                                                  reinterpret_cast<uint16_t *>(smem), buf0,
                                                  buf1, ctl, s_sum, s_tot, s_scan);
        else
            solve_graph<NT, EPT, WT, false, false>(A, g, gstate, nullptr, buf0, buf1, ctl,
                                                   s_sum, s_tot, s_scan);
    }
    if (threadIdx.x == 0 && ctl.err) atomicOr(A.err, ctl.err);
}

// Queue counter and error word to zero (a kernel, not a memset, so the
// launch sequence can be captured into a graph).
__global__ void k_persist_reset(uint32_t *queue, uint32_t *err)
{
    if (threadIdx.x == 0) {
        *queue = 0;
        *err = 0;
    }
}

// Offsets and order of a one-graph launch: vertices [0, n), edges [0, m).
__global__ void k_small_setup(int64_t *vo, int64_t *eo, uint32_t *order, int64_t n, int64_t m)
{
    if (threadIdx.x == 0) {
        vo[0] = 0;
        vo[1] = n;
        eo[0] = 0;
        eo[1] = m;
        order[0] = 0;
    }
}

void launch_small_setup(hipStream_t s, int64_t *vo, int64_t *eo, uint32_t *order, int64_t n,
                        int64_t m)
{
    k_small_setup<<<1, 64, 0, s>>>(vo, eo, order, n, m);
}

namespace {

template <int NT, int EPT>
hipError_t launch_cfg(hipStream_t s, const PersistArgs &A, int wt, unsigned grid)
{
    const size_t dyn = A.lds_bytes;
    if (wt == MSF_W_F32) {
        (void)hipFuncSetAttribute((const void *)k_persist<NT, EPT, MSF_W_F32>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
        k_persist<NT, EPT, MSF_W_F32><<<grid, NT, dyn, s>>>(A);
    } else {
        (void)hipFuncSetAttribute((const void *)k_persist<NT, EPT, MSF_W_U32>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
        k_persist<NT, EPT, MSF_W_U32><<<grid, NT, dyn, s>>>(A);
    }
    return hipGetLastError();
}

}  // namespace

int persist_blocks_per_cu(const PersistCfg &cfg, int wt)
{
    // one occupancy query per (device, configuration, weight type)
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, uint32_t, int>, int> known;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const auto key = std::make_tuple(dev, cfg.nt, cfg.ept, (uint32_t)cfg.lds, wt);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = known.find(key);
        if (it != known.end()) return it->second;
    }
    const void *f = nullptr;
#define MSF_PERSIST_FN(NT_, EPT_)                                                            \
    if (cfg.nt == NT_ && cfg.ept == EPT_)                                                   \
        f = wt == MSF_W_F32 ? (const void *)k_persist<NT_, EPT_, MSF_W_F32>                  \
                            : (const void *)k_persist<NT_, EPT_, MSF_W_U32>;
    MSF_PERSIST_FN(256, 4)
    MSF_PERSIST_FN(512, 2)
    MSF_PERSIST_FN(512, 4)
    MSF_PERSIST_FN(1024, 2)
    MSF_PERSIST_FN(1024, 4)
#undef MSF_PERSIST_FN
    if (!f) return 0;
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cfg.lds);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, cfg.nt, cfg.lds) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    std::lock_guard<std::mutex> lk(mu);
    known[key] = nb;
    return nb;
}

const PersistCfg *persist_candidates(int *count)
{
    // threads per workgroup x edges per thread and load round x dynamic LDS
    // (which sets how many workgroups share a compute unit)
    static const PersistCfg c[] = {
        {256, 4, 32 << 10},  {512, 2, 32 << 10},  {512, 4, 64 << 10},  {512, 4, 32 << 10},
        {1024, 2, 64 << 10}, {1024, 4, 64 << 10}, {1024, 2, 150 << 10}, {1024, 4, 150 << 10},
    };
    *count = (int)(sizeof(c) / sizeof(c[0]));
    return c;
}

hipError_t launch_persist(hipStream_t s, const PersistArgs &A, const PersistCfg &cfg, int wt,
                          unsigned grid)
{
    k_persist_reset<<<1, 64, 0, s>>>(A.queue, A.err);
    if (cfg.nt == 256 && cfg.ept == 4) return launch_cfg<256, 4>(s, A, wt, grid);
    if (cfg.nt == 512 && cfg.ept == 2) return launch_cfg<512, 2>(s, A, wt, grid);
    if (cfg.nt == 512 && cfg.ept == 4) return launch_cfg<512, 4>(s, A, wt, grid);
    if (cfg.nt == 1024 && cfg.ept == 2) return launch_cfg<1024, 2>(s, A, wt, grid);
    if (cfg.nt == 1024 && cfg.ept == 4) return launch_cfg<1024, 4>(s, A, wt, grid);
    return hipErrorInvalidValue;
}

}  // namespace msf
