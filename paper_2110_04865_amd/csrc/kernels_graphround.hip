// One round of Algorithm 2 with complete shortcutting (section 4.2) driven
// entirely on the device, for enqueueing several rounds without waiting for
// the host between them (directly, or captured once per solve into a HIP
// graph and replayed).
//
// Every launch size is fixed (it depends on n, not on how many roots are
// left), and every kernel reads the device flag gdone first: once a round
// has kept no hook (the termination test of Algorithm 2: p no longer
// changes), the round-end kernel sets it and every later kernel of the
// sequence returns at once.  The steps are those of the host-stepped loop,
// over all vertices instead of compacted lists:
//   sweep          the multilinear kernel + projection (kernels_sweep.hip)
//   k_gr_hook      every root hooks across its minimum edge (hooking step)
//   k_gr_tiebreak  the smaller root of a mutual pair reverts; the kept
//                  hooks' edges are flagged and counted (tie-breaking step)
//   k_gr_chase     complete shortcutting by chasing every kept hook to its
//                  final root, summing the hooks' weights exactly
//   fold, update   the weight partials into the counters; p <- h[p]
//   k_gr_round_end records the round's hooks and sets gdone when none
#include <algorithm>

#include "exact_sum.hpp"
#include "msf_internal.hpp"
#include "wave.hpp"

namespace msf {

namespace {

unsigned vgrid(int64_t n, unsigned cap)
{
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap));
}

__global__ __launch_bounds__(256) void k_gr_hook(const uint32_t *__restrict__ p,
                                                 uint64_t *__restrict__ r,
                                                 const int32_t *__restrict__ edges, int32_t n,
                                                 uint32_t *__restrict__ h,
                                                 uint32_t *__restrict__ hedge,
                                                 uint32_t *__restrict__ hwk, const Counters *cnt)
{
    if (cnt->gdone) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        if (p[v] != (uint32_t)v) continue;
        const uint64_t key = r[v];
        if (key == KEY_INF) {
            h[v] = (uint32_t)v;
            continue;
        }
        r[v] = KEY_INF;  // empty again for the next round's sweep
        const uint32_t e = (uint32_t)key;
        const uint32_t a = p[(uint32_t)edges[2 * (size_t)e]];
        const uint32_t b = p[(uint32_t)edges[2 * (size_t)e + 1]];
        h[v] = a == (uint32_t)v ? b : a;
        hedge[v] = e;
        hwk[v] = (uint32_t)(key >> 32);
    }
}

// The larger root of a mutual pair never reverts whatever it reads, so the
// smaller one reverts in place without a race.
__global__ __launch_bounds__(256) void k_gr_tiebreak(const uint32_t *__restrict__ p, int32_t n,
                                                     uint32_t *h,
                                                     const uint32_t *__restrict__ hedge,
                                                     uint8_t *__restrict__ flags, Counters *cnt)
{
    if (cnt->gdone) return;
    __shared__ uint32_t s_lds[256 / 64 + 1];
    uint32_t kept = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        if (p[v] != (uint32_t)v) continue;
        const uint32_t t = h[v];
        if (t == (uint32_t)v) continue;
        if ((uint32_t)v < t && h[t] == (uint32_t)v) {
            h[v] = (uint32_t)v;
            continue;
        }
        flags[hedge[v]] = 1;
        ++kept;
    }
    kept = block_sum<256>(kept, s_lds);
    if (threadIdx.x == 0 && kept) atomicAdd(&cnt->ghooks, kept);
}

// Every kept hook (a root at the round start whose h moved) chases its
// chain to the final root, writing each improvement back; the cap of n
// steps turns an impossible cycle into the error flag.  Its edge's weight
// goes into this workgroup's exact partial sums (folded afterwards).
template <int WT>
__global__ __launch_bounds__(256) void k_gr_chase(const uint32_t *__restrict__ p, int32_t n,
                                                  uint32_t *h, const uint32_t *__restrict__ hwk,
                                                  uint32_t *part, int64_t *wpart,
                                                  const Counters *cnt)
{
    if (cnt->gdone) return;
    __shared__ uint32_t s_lds[256 / 64 + 1];
    __shared__ int64_t s_sum[(256 / 64) * (ACC_DIGITS + 1)];
    uint32_t longest = 0, broken = 0;
    WSum ws;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        if (p[v] != (uint32_t)v) continue;
        uint32_t x = load_relaxed_u32(h + v);
        if (x == (uint32_t)v) continue;
        wsum_add<WT>(ws, hwk[v]);
        uint32_t steps = 0;
        for (;;) {
            const uint32_t y = load_relaxed_u32(h + x);
            if (y == x) break;
            x = y;
            store_relaxed_u32(h + v, x);
            if (++steps > (uint32_t)n) {
                broken = 1;
                break;
            }
        }
        longest = steps > longest ? steps : longest;
    }
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t o = __shfl_xor(longest, d, 64);
        longest = o > longest ? o : longest;
        broken |= __shfl_xor(broken, d, 64);
    }
    if (__lane_id() == 0) s_lds[threadIdx.x >> 6] = longest | (broken << 31);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t v = 0, br = 0;
        for (int i = 0; i < 4; ++i) {
            const uint32_t o = s_lds[i];
            v = (o & 0x7FFFFFFFu) > v ? (o & 0x7FFFFFFFu) : v;
            br |= o >> 31;
        }
        part[blockIdx.x] = v | (br << 31);
    }
    wsum_block<256, WT>(ws, s_sum, wpart + blockIdx.x, CHASE_MAX_BLOCKS);
}

// p[v] <- h[p[v]] where the adjacency still has a row for v (S == 1), or
// for every vertex (S > 1).
__global__ __launch_bounds__(256) void k_gr_update(const uint32_t *__restrict__ row_ptr,
                                                   int32_t n, int S, uint32_t *__restrict__ p,
                                                   const uint32_t *__restrict__ h,
                                                   const Counters *cnt)
{
    if (cnt->gdone) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        if (S > 1 || row_ptr[i + 1] > row_ptr[i]) p[i] = h[p[i]];
}

__global__ void k_gr_round_end(Counters *cnt)
{
    if (threadIdx.x != 0 || cnt->gdone) return;
    const uint32_t k = cnt->grounds, hooks = cnt->ghooks;
    if (k < 64) cnt->ghist[k] = hooks;
    cnt->grounds = k + 1;
    cnt->ghooks = 0;
    // the roots that can still hook at least halve every round: more than
    // 40 rounds means a defect, reported as a cycle
    if (hooks == 0 || k + 1 > 40) cnt->gdone = 1;
    if (hooks != 0 && k + 1 > 40) cnt->err |= ERR_CYCLE;
}

}  // namespace

void enqueue_graph_round(hipStream_t s, const GraphRound &g, Counters *dcnt, bool sweep)
{
    const int32_t n = g.a.n;
    if (sweep) launch_sweep(s, g.a, g.p, g.r, dcnt);
    k_gr_hook<<<vgrid(n, 4096), 256, 0, s>>>(g.p, g.r, g.a.edges, n, g.h, g.hedge, g.hwk, dcnt);
    k_gr_tiebreak<<<vgrid(n, 4096), 256, 0, s>>>(g.p, n, g.h, g.hedge, g.flags, dcnt);
    const unsigned cg = vgrid(n, CHASE_MAX_BLOCKS);
    int64_t *wpart = reinterpret_cast<int64_t *>(
        ((uintptr_t)(g.part + CHASE_MAX_BLOCKS) + 7) & ~(uintptr_t)7);
    if (g.wt == MSF_W_F32)
        k_gr_chase<MSF_W_F32><<<cg, 256, 0, s>>>(g.p, n, g.h, g.hwk, g.part, wpart, dcnt);
    else
        k_gr_chase<MSF_W_U32><<<cg, 256, 0, s>>>(g.p, n, g.h, g.hwk, g.part, wpart, dcnt);
    launch_chase_fold(s, g.part, cg, dcnt);
    k_gr_update<<<vgrid(n, 4096), 256, 0, s>>>(g.a.row_ptr, n, g.a.sl.S, g.p, g.h, dcnt);
    k_gr_round_end<<<1, 64, 0, s>>>(dcnt);
}

}  // namespace msf
