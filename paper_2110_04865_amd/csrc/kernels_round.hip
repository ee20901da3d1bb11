// Per-round kernels of Algorithm 2 with complete shortcutting (section 4.2),
// plus output compaction and the standalone shortcut of an arbitrary parent
// vector.
//
// State between kernels (see msf_internal.hpp): p is a star forest at the
// start of every round; R lists the roots that may still have an outgoing
// edge; r[i] holds root i's minimum outgoing key after the sweep.
//
// The root lists (R, F) are built by ordered tile compaction: each
// workgroup takes a tile from a ticket, counts, and gets its output offset
// from a decoupled look-back, so one counter atomic is issued per tile
// rather than per wave, and list order is deterministic.  The output ids
// (up to m/8192 tiles) are counted, scanned and written in separate passes
// instead: a long chain of tickets and look-backs costs more there than a
// second read of the flags.
#include "exact_sum.hpp"
#include "msf_internal.hpp"
#include "wave.hpp"

namespace msf {

namespace {

unsigned grid_for(size_t n, unsigned block = 256, unsigned cap = 8192)
{
    size_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

constexpr int CT_NT = 256;                 // compaction tile: threads
#ifndef ROUND_ITEMS_PER_THREAD
#define ROUND_ITEMS_PER_THREAD 8
#endif
constexpr int CT_IT = ROUND_ITEMS_PER_THREAD;  // items per thread
constexpr int CT_TILE = CT_NT * CT_IT;     // items per tile
static_assert(CT_IT <= 32, "a thread's items are kept in 32-bit masks");
constexpr uint64_t M31 = (1ull << 31) - 1ull;

uint32_t ct_tiles(uint64_t n) { return (uint32_t)((n + CT_TILE - 1) / CT_TILE); }

}  // namespace

uint32_t compaction_tiles(uint64_t n) { return ct_tiles(n); }

// Zero the look-back status of `tiles` tiles and the ticket (one launch).
static void prep_lookback(hipStream_t s, uint64_t *status, uint32_t tiles, Counters *dcnt)
{
    launch_zero_lookback(s, status, tiles, &dcnt->ticket, 1, nullptr, 0);
}

// A solve's round state in one launch: p = h = identity over n vertices,
// r = empty when given, and `words` words of forest flags cleared.
__global__ void k_round_state(uint32_t *p, uint32_t *h, uint64_t *r, size_t n, uint32_t *flags,
                              size_t words)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t top = n > words ? n : words;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < top; i += stride) {
        if (i < n) {
            p[i] = (uint32_t)i;
            h[i] = (uint32_t)i;
            if (r) r[i] = KEY_INF;
        }
        if (i < words) flags[i] = 0u;
    }
}

void launch_round_state(hipStream_t s, uint32_t *p, uint32_t *h, uint64_t *r, size_t n,
                        uint32_t *flags, size_t words)
{
    const size_t top = n > words ? n : words;
    if (top) k_round_state<<<grid_for(top), 256, 0, s>>>(p, h, r, n, flags, words);
}

// ----------------------------------------------------------- root list --
// R = vertices with at least one stored entry (isolated vertices are
// finished roots from the start).  Counted per tile, scanned, then written
// (a launch of this size has all its tiles resident at once, where a ticket
// and a look-back per tile would chain them: 37 us for 1024 tiles).

// Active vertices of this thread's CT_IT items, as a mask.
__device__ __forceinline__ uint32_t roots_mask(const uint32_t *__restrict__ row_ptr, int32_t n,
                                               int S, int64_t base)
{
    uint32_t act = 0;
    for (int q = 0; q < S; ++q) {
        const uint32_t *rp = row_ptr + (size_t)q * ((size_t)n + 1);
        uint32_t prev = (base <= n) ? rp[base] : 0u;
#pragma unroll
        for (int k = 0; k < CT_IT; ++k) {
            const uint32_t nx = (base + k + 1 <= n) ? rp[base + k + 1] : 0u;
            if (base + k < n && nx > prev) act |= 1u << k;
            prev = nx;
        }
    }
    return act;
}

__global__ __launch_bounds__(CT_NT) void k_roots_count(const uint32_t *__restrict__ row_ptr,
                                                       int32_t n, int S,
                                                       uint32_t *__restrict__ tcnt)
{
    __shared__ uint32_t s_lds[CT_NT / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * CT_TILE + (int64_t)threadIdx.x * CT_IT;
    const uint32_t c = (uint32_t)__popc(roots_mask(row_ptr, n, S, base));
    const uint32_t tot = block_sum<CT_NT>(c, s_lds);
    if (threadIdx.x == 0) tcnt[blockIdx.x] = tot;
}

__global__ __launch_bounds__(CT_NT) void k_roots_write(const uint32_t *__restrict__ row_ptr,
                                                       int32_t n, int S,
                                                       const uint32_t *__restrict__ toff,
                                                       uint32_t *__restrict__ R)
{
    __shared__ uint32_t s_lds[CT_NT / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * CT_TILE + (int64_t)threadIdx.x * CT_IT;
    const uint32_t act = roots_mask(row_ptr, n, S, base);
    uint32_t tot;
    uint32_t o = toff[blockIdx.x] + block_excl_sum<CT_NT>((uint32_t)__popc(act), s_lds, &tot);
#pragma unroll
    for (int k = 0; k < CT_IT; ++k)
        if (act & (1u << k)) R[o++] = (uint32_t)(base + k);
}

msf_status launch_init_roots(Ctx *c, const uint32_t *row_ptr, int32_t n, int S, uint32_t *R,
                             uint64_t *status)
{
    const uint32_t tiles = ct_tiles((uint64_t)n);
    hipStream_t s = c->stream;
    if (!tiles) {
        launch_fill_u32(s, &c->dcnt->nR, 0u, 1);
        return MSF_OK;
    }
    // per-tile counts and their scan in the status buffer (8 bytes per
    // tile and one more); at most 2^20 tiles, so the scan takes its
    // three-launch form, whose workspace is not the status buffer
    uint32_t *tcnt = reinterpret_cast<uint32_t *>(status);
    uint32_t *toff = tcnt + tiles;
    k_roots_count<<<tiles, CT_NT, 0, s>>>(row_ptr, n, S, tcnt);
    MSF_TRY(scan_u32(c, tcnt, toff, (int64_t)tiles, &c->dcnt->nR));
    k_roots_write<<<tiles, CT_NT, 0, s>>>(row_ptr, n, S, toff, R);
    MSF_HIP(hipGetLastError());
    return MSF_OK;
}

// ---------------------------------------------------------------- hook --
// Hooking step of Algorithm 2: root i takes the parent of the far endpoint of its
// minimum outgoing edge.  The EDGE pair carries the edge id; the target is
// recovered from the edge's endpoints (exactly one of them is in i's star).
// Writes go to h, never to p, so concurrent readers of p see one version.
// r[i] is reset to empty for the next round.

// IDENTITY: p is the identity (round 1); with row_ptr, col and perm (every
// 64-entry chunk ordered by (row, key), perm[j] the chunk offset of the
// entry at sorted position j), a root whose row lies in one chunk takes its
// hook target from the row's first entry in that order (its smallest key)
// instead of gathering the edge's endpoints.
// Items per thread of the hook: IT (item k of a thread is entry
// block * 256 * IT + k * 256 + thread of R: coalesced loads, issued in
// phases so that the chains R -> r -> edge endpoints -> parents of
// different items overlap).  Several items per thread only pay with many
// roots; with fewer, one item per thread keeps every compute unit busy.
#ifndef HOOK_MANY_ROOTS
#define HOOK_MANY_ROOTS (1u << 22)
#endif
constexpr uint32_t HK_MANY = HOOK_MANY_ROOTS;

template <bool IDENTITY, int HK_IT>
__global__ __launch_bounds__(256) void k_hook(const uint32_t *__restrict__ R, uint32_t nR,
                                              uint64_t *__restrict__ r,
                                              const uint32_t *__restrict__ p,
                                              const int32_t *__restrict__ edges,
                                              uint32_t *__restrict__ h,
                                              uint32_t *__restrict__ hedge,
                                              uint32_t *__restrict__ hwk,
                                              const uint32_t *__restrict__ row_ptr,
                                              const uint32_t *__restrict__ col,
                                              const uint8_t *__restrict__ perm, Counters *tb_cnt)
{
    // the tie break that follows counts into these (no kernel between reads them)
    if (tb_cnt && blockIdx.x == 0 && threadIdx.x == 0) {
        tb_cnt->rf = 0;
        tb_cnt->tdone = 0;
        tb_cnt->nR = tb_cnt->nF = tb_cnt->hooks = 0;
    }
    const uint32_t base = blockIdx.x * (256u * HK_IT) + threadIdx.x;
    uint32_t id[HK_IT];
    uint64_t key[HK_IT];
#pragma unroll
    for (int k = 0; k < HK_IT; ++k) {
        const uint32_t j = base + (uint32_t)k * 256u;
        id[k] = j < nR ? R[j] : NONE32;
    }
#pragma unroll
    for (int k = 0; k < HK_IT; ++k) key[k] = id[k] != NONE32 ? r[id[k]] : KEY_INF;
    // the target: with p the identity and the root's row inside one sorted
    // chunk, the row's first entry; otherwise the endpoint of the edge that
    // is not in the root's star
    uint32_t tgt[HK_IT];
    bool done[HK_IT];
    if (IDENTITY && row_ptr) {
        uint32_t rs[HK_IT], re[HK_IT];
#pragma unroll
        for (int k = 0; k < HK_IT; ++k) {
            const bool v = key[k] != KEY_INF;
            rs[k] = v ? row_ptr[id[k]] : 0u;
            re[k] = v ? row_ptr[id[k] + 1] : 0u;
        }
#pragma unroll
        for (int k = 0; k < HK_IT; ++k) {
            done[k] = key[k] != KEY_INF && (rs[k] >> 6) == ((re[k] - 1u) >> 6);
            tgt[k] = done[k] ? col[(rs[k] & ~63u) | perm[rs[k]]] : 0u;
        }
    } else {
#pragma unroll
        for (int k = 0; k < HK_IT; ++k) done[k] = false;
    }
    uint32_t ea[HK_IT], eb[HK_IT];
#pragma unroll
    for (int k = 0; k < HK_IT; ++k) {
        const bool need = key[k] != KEY_INF && !done[k];
        const uint32_t e = (uint32_t)key[k];
        ea[k] = need ? (uint32_t)edges[2 * (size_t)e] : 0u;
        eb[k] = need ? (uint32_t)edges[2 * (size_t)e + 1] : 0u;
    }
    if (!IDENTITY) {
#pragma unroll
        for (int k = 0; k < HK_IT; ++k) {
            const bool need = key[k] != KEY_INF;
            ea[k] = need ? p[ea[k]] : 0u;
            eb[k] = need ? p[eb[k]] : 0u;
        }
    }
#pragma unroll
    for (int k = 0; k < HK_IT; ++k) {
        const uint32_t i = id[k];
        if (i == NONE32) continue;
        if (key[k] != KEY_INF) {
            r[i] = KEY_INF;  // empty again for the next round's sweep
            // with p the identity (round 1) the endpoints are their own roots
            h[i] = done[k] ? tgt[k] : (ea[k] == i ? eb[k] : ea[k]);
            hedge[i] = (uint32_t)key[k];
            hwk[i] = (uint32_t)(key[k] >> 32);  // the hooked edge's weight key
        } else {
            h[i] = i;
            hedge[i] = NONE32;
        }
    }
}

void launch_hook(hipStream_t s, const uint32_t *R, uint32_t nR, uint64_t *r, const uint32_t *p,
                 const int32_t *edges, uint32_t *h, uint32_t *hedge, uint32_t *hwk,
                 bool identity, const uint32_t *row_ptr, const uint32_t *col,
                 const uint8_t *run_perm, Counters *tb_cnt)
{
    if (!nR) return;
    const bool many = nR >= HK_MANY;
    const unsigned g4 = (nR + 1023u) / 1024u, g1 = (nR + 255u) / 256u;
    // the shortcut through the ordered chunks needs all three
    if (!row_ptr || !col || !run_perm) row_ptr = nullptr;
    if (identity && many)
        k_hook<true, 4><<<g4, 256, 0, s>>>(R, nR, r, p, edges, h, hedge, hwk, row_ptr, col,
                                           run_perm, tb_cnt);
    else if (identity)
        k_hook<true, 1><<<g1, 256, 0, s>>>(R, nR, r, p, edges, h, hedge, hwk, row_ptr, col,
                                           run_perm, tb_cnt);
    else if (many)
        k_hook<false, 4><<<g4, 256, 0, s>>>(R, nR, r, p, edges, h, hedge, hwk, nullptr, nullptr,
                                            nullptr, tb_cnt);
    else
        k_hook<false, 1><<<g1, 256, 0, s>>>(R, nR, r, p, edges, h, hedge, hwk, nullptr, nullptr,
                                            nullptr, tb_cnt);
}

// ------------------------------------------------------- forest weight --
// The forest weight is summed exactly as the hooks are kept: uint32 weights
// in u64; float32 weights as integers in units of 2^-149 (the smallest
// float32 subnormal) split over 32-bit digits held in int64 lanes, so the
// sum does not depend on the order of additions; infinities are counted
// separately.  The shortcut chase visits every kept hook once; each of its
// workgroups writes its partial sums to its own slot, k_chase_fold adds the
// slots into the counters, and k_total rounds once at the end.  The weight
// comes back from the key's high word: for float32 the key map is undone.

// Most blocks a chase launch uses (each leaves one partial).
#ifndef CHASE_WORKGROUPS
#define CHASE_WORKGROUPS 2048
#endif
constexpr unsigned CHASE_BLOCKS = CHASE_WORKGROUPS;

// ----------------------------------------------------------- tie break --
// Tie-breaking step of Algorithm 2: a 2-cycle (i hooks on k and k on i) is the only
// cycle hooking can form (section 2.3, with keys distinct); its smaller id
// reverts to being a root and the larger keeps the hook, so the shared edge
// enters the forest once.  Roots without an outgoing edge are finished for
// good (their component is complete) and leave R.  Kept hooks flag their
// edge and join the shortcut frontier F; reverted roots stay in R.
//
// A revert writes h[i] while other roots may read it; they read either the
// old target (which is not them unless they are i's partner, and the
// partner has the larger id so it never reverts) or i itself, and decide
// the same either way.

__global__ __launch_bounds__(CT_NT) void k_tiebreak(const uint32_t *__restrict__ R, uint32_t nR,
                                                    uint32_t *h, const uint32_t *__restrict__ hedge,
                                                    uint8_t *__restrict__ in_forest,
                                                    uint32_t *__restrict__ Rnext,
                                                    uint32_t *__restrict__ F, Counters *cnt)
{
    __shared__ uint64_t s_lds[CT_NT / 64 + 1];
    __shared__ uint64_t s_pre;
    const uint32_t tile = blockIdx.x;
    // item k of a thread is entry tile * CT_TILE + k * CT_NT + thread of R,
    // so every load below is one coalesced access per wave; the loads come
    // in phases (ids, targets, the targets' targets and hooked edges), all
    // issued before any store, instead of one dependent chain per item
    const uint32_t base = tile * CT_TILE + threadIdx.x;
    uint32_t id[CT_IT], t[CT_IT], back[CT_IT], e[CT_IT];
#pragma unroll
    for (int k = 0; k < CT_IT; ++k) {
        const uint32_t j = base + (uint32_t)k * CT_NT;
        id[k] = j < nR ? R[j] : NONE32;
    }
#pragma unroll
    for (int k = 0; k < CT_IT; ++k) t[k] = id[k] != NONE32 ? load_relaxed_u32(h + id[k]) : NONE32;
#pragma unroll
    for (int k = 0; k < CT_IT; ++k) {
        const bool hk = id[k] != NONE32 && t[k] != id[k];
        back[k] = hk ? load_relaxed_u32(h + t[k]) : NONE32;
        e[k] = hk ? hedge[id[k]] : 0u;
    }
    uint32_t stay = 0, hooked = 0, ca = 0, cb = 0;
#pragma unroll
    for (int k = 0; k < CT_IT; ++k) {
        const uint32_t i = id[k];
        if (i == NONE32 || t[k] == i) continue;
        if (back[k] == i && i < t[k]) {
            store_relaxed_u32(h + i, i);
            stay |= 1u << k;
            ++ca;
        } else {
            in_forest[e[k]] = 1;
            hooked |= 1u << k;
            ++cb;
        }
    }
    // Both lists keep the tile's order of R (k-major, then wave, then lane:
    // the order of the entries), so the shortcut and the next hook read h
    // and r of nearby vertices together.  Per (item k, wave): counts by
    // ballot, a scan of the 2 x CT_IT x waves counts in LDS, and ranks from
    // the lane masks.  Across tiles the lists are sets: a block takes its
    // slots with one atomic on the packed (roots << 31 | hooks) count; the
    // last block to finish publishes the totals (each block's slot atomic
    // has returned before it counts itself done).
    constexpr int NW = CT_NT / 64;
    __shared__ uint32_t s_off[2][CT_IT][NW];
    const uint32_t w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < CT_IT; ++k) {
        const uint64_t ma = __ballot((stay >> k) & 1u), mb = __ballot((hooked >> k) & 1u);
        if (__lane_id() == 0) {
            s_off[0][k][w] = (uint32_t)__popcll(ma);
            s_off[1][k][w] = (uint32_t)__popcll(mb);
        }
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        // exclusive scan of one list's counts in (k, wave) order
        uint32_t run = 0;
        for (int k = 0; k < CT_IT; ++k)
            for (int v = 0; v < NW; ++v) {
                const uint32_t c = s_off[threadIdx.x][k][v];
                s_off[threadIdx.x][k][v] = run;
                run += c;
            }
        s_lds[threadIdx.x] = run;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint64_t btot = (s_lds[0] << 31) | s_lds[1];
        const uint64_t pre = atomicAdd((unsigned long long *)&cnt->rf, (unsigned long long)btot);
        s_pre = pre;
        if (atomicAdd(&cnt->tdone, pre == ~0ull ? 0u : 1u) == gridDim.x - 1) {
            const uint64_t tot = atomicAdd((unsigned long long *)&cnt->rf, 0ull);
            cnt->nR = (uint32_t)(tot >> 31);
            cnt->nF = (uint32_t)(tot & M31);
        }
    }
    __syncthreads();
    const uint32_t pa = (uint32_t)(s_pre >> 31), pb = (uint32_t)(s_pre & M31);
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int k = 0; k < CT_IT; ++k) {
        const bool a = (stay >> k) & 1u, b = (hooked >> k) & 1u;
        const uint64_t ma = __ballot(a), mb = __ballot(b);
        if (a) Rnext[pa + s_off[0][k][w] + (uint32_t)__popcll(ma & lt)] = id[k];
        else if (b) F[pb + s_off[1][k][w] + (uint32_t)__popcll(mb & lt)] = id[k];
    }
    (void)ca;
    (void)cb;
}

void launch_tiebreak(hipStream_t s, const uint32_t *R, uint32_t nR, uint32_t *h,
                     const uint32_t *hedge, uint8_t *in_forest, uint32_t *Rnext, uint32_t *F,
                     uint64_t *status, Counters *dcnt, bool counts_cleared)
{
    const uint32_t tiles = ct_tiles(nR);
    (void)status;
    // the slot count, the done count and nR, nF, hooks start at zero: cleared
    // by the hook launched just before (it runs whenever nR > 0), else here
    if (!counts_cleared)
        launch_zero_lookback(s, nullptr, 0, reinterpret_cast<uint32_t *>(&dcnt->rf), 4,
                             &dcnt->nR, 3);
    if (!tiles) return;
    k_tiebreak<<<tiles, CT_NT, 0, s>>>(R, nR, h, hedge, in_forest, Rnext, F, dcnt);
}

// ------------------------------------------------------------- shortcut --
// Complete shortcutting restricted to the roots that hooked (the "changed"
// set of Algorithm 3): each thread chases its hook chain to the final root,
// writing every improvement back so other chases jump further.  Every value
// read of h[x] is an ancestor of x (or x itself for a final root, which is
// never written), and the hook forest is acyclic after tie breaking, so each
// chase ends after at most the height of its tree; a hard cap of nF steps
// turns a (theoretically impossible) cycle into an error flag.  F lists the
// kept hooks, so the chase also adds their edges' weights to the forest
// weight (hwk: the hook's weight key).

template <int WT>
__global__ __launch_bounds__(256) void k_chase(const uint32_t *__restrict__ F, uint32_t nF,
                                               uint32_t *h, const uint32_t *__restrict__ hwk,
                                               uint32_t *part, int64_t *wpart)
{
    __shared__ uint32_t s_lds[256 / 64 + 1];
    __shared__ int64_t s_sum[(256 / 64) * (ACC_DIGITS + 1)];
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t longest = 0, broken = 0;
    WSum ws;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < nF; k += stride) {
        const uint32_t i = F[k];
        wsum_add<WT>(ws, hwk[i]);
        uint32_t x = load_relaxed_u32(h + i);
        uint32_t steps = 0;
        for (;;) {
            const uint32_t y = load_relaxed_u32(h + x);
            if (y == x) break;
            x = y;
            store_relaxed_u32(h + i, x);
            if (++steps > nF) {
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
    wsum_block<256, WT>(ws, s_sum, wpart + blockIdx.x, CHASE_BLOCKS);
}

// Fold per-block chase results into the counters: the longest chase, the
// cycle flag and the kept hooks' weight sums (wpart[j * CHASE_BLOCKS + b]).
__global__ __launch_bounds__(256) void k_chase_fold(const uint32_t *__restrict__ part,
                                                    const int64_t *__restrict__ wpart,
                                                    uint32_t nb, Counters *cnt)
{
    if (cnt->gdone) return;  // rounds driven on the device: nothing was chased
    __shared__ int64_t s_w[4][WS_WORDS + 1];
    uint32_t v = 0, br = 0;
    int64_t w[WS_WORDS] = {};
    for (uint32_t i = threadIdx.x; i < nb; i += 256) {
        const uint32_t o = part[i];
        v = (o & 0x7FFFFFFFu) > v ? (o & 0x7FFFFFFFu) : v;
        br |= o >> 31;
#pragma unroll
        for (int j = 0; j < WS_WORDS; ++j) w[j] += wpart[(size_t)j * CHASE_BLOCKS + i];
    }
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t o = __shfl_xor(v, d, 64);
        v = o > v ? o : v;
        br |= __shfl_xor(br, d, 64);
    }
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < WS_WORDS; ++j) {
        const int64_t t = wave_sum(w[j]);
        if (__lane_id() == 0) s_w[wv][j] = t;
    }
    if (__lane_id() == 0) s_w[wv][WS_WORDS] = (int64_t)(v | (br << 31));
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int i = 1; i < 4; ++i) {
        for (int j = 0; j < WS_WORDS; ++j) s_w[0][j] += s_w[i][j];
        const uint32_t o = (uint32_t)s_w[i][WS_WORDS];
        v = (o & 0x7FFFFFFFu) > v ? (o & 0x7FFFFFFFu) : v;
        br |= o >> 31;
    }
    atomicMax(&cnt->max_chase, v);
    if (br) atomicOr(&cnt->err, ERR_CYCLE);
    cnt->total_u64 += (uint64_t)s_w[0][0];
    for (int d = 0; d < ACC_DIGITS; ++d) cnt->acc[d] += s_w[0][1 + d];
    cnt->inf_pos += (uint32_t)s_w[0][1 + ACC_DIGITS];
    cnt->inf_neg += (uint32_t)s_w[0][2 + ACC_DIGITS];
}


void launch_chase_fold(hipStream_t s, const uint32_t *part, uint32_t nb, Counters *dcnt)
{
    const int64_t *wpart = reinterpret_cast<const int64_t *>(
        ((uintptr_t)(part + CHASE_BLOCKS) + 7) & ~(uintptr_t)7);
    k_chase_fold<<<1, 256, 0, s>>>(part, wpart, nb, dcnt);
}

void launch_chase(hipStream_t s, const uint32_t *F, uint32_t nF, uint32_t *h,
                  const uint32_t *hwk, msf_wtype wt, uint32_t *part, Counters *dcnt)
{
    if (!nF) return;
    const unsigned g = grid_for(nF, 256, CHASE_BLOCKS);
    // part: the per-block chase words, then per-block weight sums (aligned)
    int64_t *wpart = reinterpret_cast<int64_t *>(
        ((uintptr_t)(part + CHASE_BLOCKS) + 7) & ~(uintptr_t)7);
    if (wt == MSF_W_F32)
        k_chase<MSF_W_F32><<<g, 256, 0, s>>>(F, nF, h, hwk, part, wpart);
    else
        k_chase<MSF_W_U32><<<g, 256, 0, s>>>(F, nF, h, hwk, part, wpart);
    k_chase_fold<<<1, 256, 0, s>>>(part, wpart, g, dcnt);
}

// p[v] <- h[p[v]] for every vertex that still has stored entries: p[v] is an
// old root and h maps it to its new root, so p is again a star forest.
// Vertices without entries are never read again.  Per-block row counts go
// to part[] (folded by k_fold_rows) for the sweep's byte accounting.

__global__ __launch_bounds__(256) void k_update_parents(const uint32_t *__restrict__ row_ptr,
                                                        int32_t n, int S, uint32_t *__restrict__ p,
                                                        const uint32_t *__restrict__ h)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (S > 1 || row_ptr[i + 1] > row_ptr[i]) {
            const uint32_t x = p[i], y = h[x];
            if (y != x) p[i] = y;  // most roots keep their place in a round
        }
    }
}

void launch_update_parents(hipStream_t s, const uint32_t *row_ptr, int32_t n, int S, uint32_t *p,
                           const uint32_t *h, uint32_t *part, Counters *dcnt, bool all)
{
    (void)part;
    (void)dcnt;
    if (!n) return;
    const unsigned g = grid_for((size_t)n, 256, 4096);
    k_update_parents<<<g, 256, 0, s>>>(row_ptr, n, all ? 2 : S, p, h);
}

// --------------------------------------------------------------- output --
// Forest flags -> ascending edge ids and their count (count per tile, scan,
// write); the forest weight was summed by the tie breaks and is rounded once
// by k_total.

constexpr int OUT_NT = 256;
constexpr int OUT_IT = 32;
constexpr int OUT_TILE = OUT_NT * OUT_IT;

// A thread's OUT_IT flags as OUT_IT/4 words (one byte per flag).
__device__ __forceinline__ void load_flags(const uint8_t *__restrict__ flags, int64_t m,
                                           int64_t base, uint32_t (&fw)[OUT_IT / 4])
{
    if (base + OUT_IT <= m) {
#pragma unroll
        for (int q = 0; q < OUT_IT / 16; ++q) {
            const uint4 v = *reinterpret_cast<const uint4 *>(flags + base + 16 * q);
            fw[4 * q] = v.x;
            fw[4 * q + 1] = v.y;
            fw[4 * q + 2] = v.z;
            fw[4 * q + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < OUT_IT / 4; ++q) {
            uint32_t x = 0;
            for (int b = 0; b < 4; ++b) {
                const int64_t e = base + 4 * q + b;
                if (e < m && flags[e]) x |= 1u << (8 * b);
            }
            fw[q] = x;
        }
    }
}

__device__ __forceinline__ uint32_t count_flags(const uint32_t (&fw)[OUT_IT / 4])
{
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < OUT_IT / 4; ++q)
        for (int b = 0; b < 4; ++b) c += ((fw[q] >> (8 * b)) & 0xFFu) ? 1u : 0u;
    return c;
}

// Pass 1 (tile = workgroup): the tile's forest-edge count.
__global__ __launch_bounds__(OUT_NT) void k_output_count(const uint8_t *__restrict__ flags,
                                                        int64_t m,
                                                        uint32_t *__restrict__ tile_cnt)
{
    __shared__ uint64_t s_lds[OUT_NT / 64 + 1];
    const uint32_t tile = blockIdx.x;
    const int64_t base = (int64_t)tile * OUT_TILE + (int64_t)threadIdx.x * OUT_IT;
    uint32_t fw[OUT_IT / 4];
    load_flags(flags, m, base, fw);
    const uint64_t tot = block_sum<OUT_NT>((uint64_t)count_flags(fw), s_lds);
    if (threadIdx.x == 0) tile_cnt[tile] = (uint32_t)tot;
}

// Pass 2: the tile's ids, ascending, from its scanned offset.
__global__ __launch_bounds__(OUT_NT) void k_output_ids(const uint8_t *__restrict__ flags,
                                                      int64_t m,
                                                      const uint32_t *__restrict__ tile_off,
                                                      int32_t *__restrict__ ids)
{
    __shared__ uint32_t s_lds[OUT_NT / 64 + 1];
    const uint32_t tile = blockIdx.x;
    const int64_t base = (int64_t)tile * OUT_TILE + (int64_t)threadIdx.x * OUT_IT;
    uint32_t fw[OUT_IT / 4];
    load_flags(flags, m, base, fw);
    const uint32_t c = count_flags(fw);
    uint32_t tot;
    uint32_t pos = tile_off[tile] + block_excl_sum<OUT_NT>(c, s_lds, &tot);
    if (c) {
        for (int k = 0; k < OUT_IT; ++k) {
            if (!((fw[k >> 2] >> (8 * (k & 3))) & 0xFFu)) continue;
            ids[pos++] = (int32_t)(base + k);
        }
    }
}

// Round the exact forest weight once (one thread).
__global__ void k_total(Counters *cnt, int wt)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t acc[ACC_DIGITS];
    for (int d = 0; d < ACC_DIGITS; ++d) acc[d] = cnt->acc[d];
    cnt->total_f64 = exact_total_f64(cnt->total_u64, acc, cnt->inf_pos, cnt->inf_neg, wt);
}

int64_t output_tiles(int64_t m) { return (m + OUT_TILE - 1) / OUT_TILE; }
size_t chase_part_bytes()
{
    return 4 * (size_t)CHASE_BLOCKS + 8 + 8 * (size_t)CHASE_BLOCKS * WS_WORDS;
}

size_t output_part_bytes(int64_t m)
{
    // per-tile counts and their scan
    return 4 * (2 * (size_t)output_tiles(m) + 2);
}

msf_status launch_output(Ctx *c, const uint8_t *in_forest, int64_t m, const void *w,
                         msf_wtype wt, int32_t *ids, void *part)
{
    const int64_t ntiles = output_tiles(m);
    if (ntiles == 0) return MSF_OK;
    hipStream_t s = c->stream;
    (void)w;
    // per-tile counts, then their exclusive scan
    uint32_t *tcnt = reinterpret_cast<uint32_t *>(part);
    uint32_t *toff = tcnt + ntiles;
    k_output_count<<<(unsigned)ntiles, OUT_NT, 0, s>>>(in_forest, m, tcnt);
    MSF_TRY(scan_u32(c, tcnt, toff, ntiles, &c->dcnt->count));
    k_output_ids<<<(unsigned)ntiles, OUT_NT, 0, s>>>(in_forest, m, toff, ids);
    k_total<<<1, 64, 0, s>>>(c->dcnt, (int)wt);
    MSF_HIP(hipGetLastError());
    return MSF_OK;
}

// ------------------------------------------- shortcut of arbitrary p ----
// Complete shortcutting of a caller's parent vector: in-place pointer
// jumping q[i] <- q[q[i]] over a shrinking frontier of vertices whose
// parent is not yet a fixed point.  A rooted forest of height d converges
// in at most ceil(log2 d) + 1 passes.  Cycles are detected afterwards: every
// final target must be a root of the input (p[q[i]] == q[i]); an even cycle
// may collapse onto false fixed points, an odd one never settles, and both
// fail that test.

__global__ void k_check_parents(const uint32_t *__restrict__ p, int32_t n, Counters *cnt)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        bad |= p[i] >= (uint32_t)n;
    if (__ballot(bad) && __lane_id() == 0) atomicOr(&cnt->err, ERR_PARENT);
}

void launch_check_parents(hipStream_t s, const uint32_t *p, int32_t n, Counters *dcnt)
{
    if (n) k_check_parents<<<grid_for((size_t)n, 256, 1024), 256, 0, s>>>(p, n, dcnt);
}

__global__ __launch_bounds__(CT_NT) void k_jump_init(const uint32_t *__restrict__ q, int32_t n,
                                                     uint32_t *__restrict__ F, uint64_t *status,
                                                     Counters *cnt)
{
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_lds[CT_NT / 64 + 1];
    __shared__ uint64_t s_pre;
    if (threadIdx.x == 0) s_tile = atomicAdd(&cnt->ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t base = (int64_t)tile * CT_TILE + (int64_t)threadIdx.x * CT_IT;
    uint32_t act = 0, c = 0;
#pragma unroll
    for (int k = 0; k < CT_IT; ++k) {
        if (base + k < n) {
            const uint32_t x = q[base + k];
            if (q[x] != x) {
                act |= 1u << k;
                ++c;
            }
        }
    }
    uint32_t oa, ob;
    uint64_t tot;
    tile_offsets2<CT_NT>(tile, c, 0u, status, s_lds, &s_pre, &oa, &ob, &tot);
#pragma unroll
    for (int k = 0; k < CT_IT; ++k)
        if (act & (1u << k)) F[oa++] = (uint32_t)(base + k);
    if (tile == gridDim.x - 1 && threadIdx.x == 0) cnt->nF = (uint32_t)(tot >> 31);
}

void launch_jump_init(hipStream_t s, const uint32_t *q, int32_t n, uint32_t *F, uint64_t *status,
                      Counters *dcnt)
{
    const uint32_t tiles = ct_tiles((uint64_t)n);
    if (!tiles) return;
    prep_lookback(s, status, tiles, dcnt);
    k_jump_init<<<tiles, CT_NT, 0, s>>>(q, n, F, status, dcnt);
}

__global__ __launch_bounds__(CT_NT) void k_jump_pass(const uint32_t *__restrict__ Fin, uint32_t nF,
                                                     uint32_t *q, uint32_t *__restrict__ Fout,
                                                     uint64_t *status, Counters *cnt)
{
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_lds[CT_NT / 64 + 1];
    __shared__ uint64_t s_pre;
    if (threadIdx.x == 0) s_tile = atomicAdd(&cnt->ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t base = tile * CT_TILE + threadIdx.x * CT_IT;
    uint32_t again = 0, c = 0;
    uint32_t id[CT_IT];
#pragma unroll
    for (int k = 0; k < CT_IT; ++k) {
        id[k] = 0;
        if (base + k < nF) {
            const uint32_t i = Fin[base + k];
            id[k] = i;
            const uint32_t x = load_relaxed_u32(q + i);
            const uint32_t y = load_relaxed_u32(q + x);
            store_relaxed_u32(q + i, y);
            if (load_relaxed_u32(q + y) != y) {
                again |= 1u << k;
                ++c;
            }
        }
    }
    uint32_t oa, ob;
    uint64_t tot;
    tile_offsets2<CT_NT>(tile, c, 0u, status, s_lds, &s_pre, &oa, &ob, &tot);
#pragma unroll
    for (int k = 0; k < CT_IT; ++k)
        if (again & (1u << k)) Fout[oa++] = id[k];
    if (tile == gridDim.x - 1 && threadIdx.x == 0) cnt->nR = (uint32_t)(tot >> 31);
}

void launch_jump_pass(hipStream_t s, const uint32_t *Fin, uint32_t nF, uint32_t *q, uint32_t *Fout,
                      uint64_t *status, Counters *dcnt)
{
    const uint32_t tiles = ct_tiles(nF);
    if (!tiles) return;
    prep_lookback(s, status, tiles, dcnt);
    k_jump_pass<<<tiles, CT_NT, 0, s>>>(Fin, nF, q, Fout, status, dcnt);
}

// One full pass of pointer jumping: every vertex takes q[i] <- q[q[i]] in
// place (the baseline of the shortcut study, section 7.1); vertices whose
// new parent is still not a root are counted into cnt->nR, one atomic per
// workgroup.  In-place jumps only move a pointer up its own tree, so any
// interleaving of the relaxed loads and stores gets at least as far as a
// synchronous pass.
__global__ __launch_bounds__(256) void k_jump_full(uint32_t *q, int32_t n, Counters *cnt)
{
    __shared__ uint64_t s_lds[256 / 64 + 1];
    uint64_t c = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t x = load_relaxed_u32(q + i);
        const uint32_t y = load_relaxed_u32(q + x);
        if (y != x) store_relaxed_u32(q + i, y);
        if (load_relaxed_u32(q + y) != y) ++c;
    }
    c = block_sum<256>(c, s_lds);
    if (threadIdx.x == 0 && c) atomicAdd(&cnt->nR, (uint32_t)c);
}

void launch_jump_full(hipStream_t s, uint32_t *q, int32_t n, Counters *dcnt)
{
    if (n <= 0) return;
    size_t g = ((size_t)n + 255) / 256;
    if (g > 8192) g = 8192;
    k_jump_full<<<(unsigned)g, 256, 0, s>>>(q, n, dcnt);
}

// Connected components by the same rounds (the connectivity variant of
// section 2.4: a star root hooks along any edge leaving its star; the
// minimum-key one found by the sweep is such an edge).  p is a star forest,
// so r[k] is set only for roots.  Hooked roots are counted into cnt->nR,
// one atomic per workgroup.
// With star (original AS rounds, section 2.3): only roots of stars hook, the
// target is the parent of the outside endpoint (a vertex of its tree, not
// necessarily the root), and the hooking edge is marked in in_forest.
__global__ __launch_bounds__(256) void k_cc_hook(const uint32_t *__restrict__ p,
                                                 const uint64_t *__restrict__ r,
                                                 const int32_t *__restrict__ edges, int32_t n,
                                                 uint32_t *__restrict__ h, Counters *cnt,
                                                 const uint32_t *__restrict__ star,
                                                 uint8_t *__restrict__ in_forest)
{
    __shared__ uint64_t s_lds[256 / 64 + 1];
    uint64_t c = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        uint32_t t = (uint32_t)k;
        const uint64_t rk = r[k];
        if (rk != KEY_INF && p[k] == (uint32_t)k && (!star || star[k])) {
            // one endpoint lies in k's star, the other outside it
            const size_t e = (size_t)(uint32_t)rk;
            const uint32_t a = p[edges[2 * e]], b = p[edges[2 * e + 1]];
            t = a == (uint32_t)k ? b : a;
            if (in_forest) in_forest[e] = 1;
            ++c;
        }
        h[k] = t;
    }
    c = block_sum<256>(c, s_lds);
    if (threadIdx.x == 0 && c) atomicAdd(&cnt->nR, (uint32_t)c);
}

// Apply the hooks; of two roots that hooked onto each other (they chose the
// same edge) the smaller stays root.  Minimum keys leave no longer cycles.
__global__ void k_cc_apply(const uint32_t *__restrict__ h, int32_t n, uint32_t *__restrict__ p)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const uint32_t t = h[k];
        if (t != (uint32_t)k && !(h[t] == (uint32_t)k && (uint32_t)k < t)) p[k] = t;
    }
}

void launch_cc_hook(hipStream_t s, const uint32_t *p, const uint64_t *r, const int32_t *edges,
                    int32_t n, uint32_t *h, Counters *dcnt, const uint32_t *star,
                    uint8_t *in_forest)
{
    if (n <= 0) return;
    size_t g = ((size_t)n + 255) / 256;
    if (g > 8192) g = 8192;
    k_cc_hook<<<(unsigned)g, 256, 0, s>>>(p, r, edges, n, h, dcnt, star, in_forest);
}

// Star check (section 2.3): star[i] = 1 iff i's tree has depth at most one.
// Pass 1 clears i and its grandparent where i is two levels down; pass 2
// takes the parent's flag (a vertex still flagged after pass 1 has a root
// for parent, whose flag pass 2 does not change).
__global__ void k_star_clear(const uint32_t *__restrict__ p, int32_t n, uint32_t *star)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t x = p[i], y = p[x];
        if (y != x) {
            star[i] = 0u;
            star[y] = 0u;
        }
    }
}

__global__ void k_star_parent(const uint32_t *__restrict__ p, int32_t n, uint32_t *star)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        if (star[i] && !star[p[i]]) star[i] = 0u;
}

// One synchronous shortcut step (section 2.3): dst[i] = src[src[i]];
// changed entries are counted into cnt->nR.
__global__ __launch_bounds__(256) void k_jump_once(const uint32_t *__restrict__ src, int32_t n,
                                                   uint32_t *__restrict__ dst, Counters *cnt)
{
    __shared__ uint64_t s_lds[256 / 64 + 1];
    uint64_t c = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t x = src[i], y = src[x];
        dst[i] = y;
        c += y != x ? 1u : 0u;
    }
    c = block_sum<256>(c, s_lds);
    if (threadIdx.x == 0 && c) atomicAdd(&cnt->nR, (uint32_t)c);
}

void launch_star_check(hipStream_t s, const uint32_t *p, int32_t n, uint32_t *star)
{
    if (n <= 0) return;
    size_t g = ((size_t)n + 255) / 256;
    if (g > 8192) g = 8192;
    launch_fill_u32(s, star, 1u, (size_t)n);
    k_star_clear<<<(unsigned)g, 256, 0, s>>>(p, n, star);
    k_star_parent<<<(unsigned)g, 256, 0, s>>>(p, n, star);
}

void launch_jump_once(hipStream_t s, const uint32_t *src, int32_t n, uint32_t *dst,
                      Counters *dcnt)
{
    if (n <= 0) return;
    size_t g = ((size_t)n + 255) / 256;
    if (g > 8192) g = 8192;
    k_jump_once<<<(unsigned)g, 256, 0, s>>>(src, n, dst, dcnt);
}

void launch_cc_apply(hipStream_t s, const uint32_t *h, int32_t n, uint32_t *p)
{
    if (n <= 0) return;
    size_t g = ((size_t)n + 255) / 256;
    if (g > 8192) g = 8192;
    k_cc_apply<<<(unsigned)g, 256, 0, s>>>(h, n, p);
}

__global__ void k_check_roots(const uint32_t *__restrict__ p, const uint32_t *__restrict__ q,
                              int32_t n, Counters *cnt)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t x = q[i];
        bad |= p[x] != x;
    }
    if (__ballot(bad) && __lane_id() == 0) atomicOr(&cnt->err, ERR_CYCLE);
}

// ---------------------------------------------------------- round checks --
// Invariants of a round, checked when MSF_CHECK_ROUNDS is set: every tree is
// a star after complete shortcutting (section 4.2), and the number of roots
// drops by exactly the number of kept hooks (the host compares the counts).

__global__ __launch_bounds__(256) void k_count_roots(const uint32_t *__restrict__ p, int32_t n,
                                                     Counters *cnt)
{
    __shared__ uint32_t s_lds[256 / 64 + 1];
    uint32_t c = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        c += p[i] == (uint32_t)i ? 1u : 0u;
    c = block_sum<256>(c, s_lds);
    if (threadIdx.x == 0 && c) atomicAdd(&cnt->roots, c);
}

__global__ void k_check_stars(const uint32_t *__restrict__ p, int32_t n, Counters *cnt)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t x = p[i];
        bad |= p[x] != x;
    }
    if (__ballot(bad) && __lane_id() == 0) atomicOr(&cnt->err, ERR_STAR);
}

void launch_count_roots(hipStream_t s, const uint32_t *p, int32_t n, Counters *dcnt)
{
    if (n) k_count_roots<<<grid_for((size_t)n, 256, 1024), 256, 0, s>>>(p, n, dcnt);
}

void launch_check_stars(hipStream_t s, const uint32_t *p, int32_t n, Counters *dcnt)
{
    if (n) k_check_stars<<<grid_for((size_t)n, 256, 1024), 256, 0, s>>>(p, n, dcnt);
}

void launch_check_roots(hipStream_t s, const uint32_t *p, const uint32_t *q, int32_t n,
                        Counters *dcnt)
{
    if (n) k_check_roots<<<grid_for((size_t)n, 256, 1024), 256, 0, s>>>(p, q, n, dcnt);
}

}  // namespace msf
