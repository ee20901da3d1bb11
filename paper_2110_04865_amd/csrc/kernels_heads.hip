// Head sweep: the multilinear projection evaluated over key-sorted runs.
//
// For a star root k the projection of section 3.2 keeps the smallest key
// over stored entries i->j with p_i == k != p_j; the multilinear function of
// section 3.1 gives the empty key when p_i == p_j.  Trees only merge, so an
// entry found with p_i == p_j (internal) stays internal for the rest of the
// solve.  When a row's entries are in ascending key order, the row's
// smallest outgoing key is the key of its first entry that is not internal,
// and every internal entry in front of it can be passed over for good.
//
// Layout.  Once per solve, every 64-entry chunk of the adjacency (entries
// [64c, 64c + 64)) is ordered by (row, key): rows keep their places and each
// row's part of the chunk (a run, at most 64 entries) is in ascending key
// order.  The entries themselves do not move: the order is a permutation,
// one byte per entry, perm[64c + j] = the chunk offset of the entry at
// sorted position j (so the adjacency is only read and can belong to a kept
// graph).  A run is described by {cur, end, row, hcol, hkey} in sorted
// positions: cur is its head (first entry not yet known to be internal),
// hcol and hkey the head's column and key (hkey = UINT64_MAX once the run
// is exhausted).  A sweep
// visits runs, not entries:
//   phase A, one lane per run: gathers p[hcol]; an outgoing head gives the
//     run's minimum; an internal one makes the lane probe the next
//     HEAD_PROBE entries with independent loads; a run still internal after
//     that is queued;
//   phase B, one wave per queued run: the rest of the run at once, first
//     outgoing entry by ballot.
// Both phases move the head past the internal entries they saw and fold
// their minima into r[root] (a read, then a 64-bit atomicMin only when it
// improves), after a wave-wide segmented minimum over lanes of the same
// root.  Phase A first compares the head's key with r[root]: runs hold
// ascending keys and r only falls during a sweep, so a head no smaller than
// r[root] is passed over without a gather (with ~97K live roots on R-MAT
// s22 this still pays: 0.56 -> 0.47 ms over the solve's head sweeps).  A
// round reads 16 bytes and gathers one parent per live run plus the entries
// that became internal, instead of every entry; the result equals the full
// sweep's, element by element of r.
#include "msf_internal.hpp"
#include "wave.hpp"

namespace msf {

namespace {

#ifndef HEAD_PROBE_ENTRIES
#define HEAD_PROBE_ENTRIES 4
#endif
constexpr int HEAD_PROBE = HEAD_PROBE_ENTRIES;

// Runs of rows longer than LONG_ROW entries carry RUN_LONG in their row
// word (rows are below 2^31).  A sweep visits them first: their heads are
// the smallest keys of 64-entry pieces of hub rows, so their roots' minima
// fall early and prune more of the short rows' heads after them.
#ifndef HEAD_LONG_ROW
#define HEAD_LONG_ROW 2048
#endif
constexpr uint32_t LONG_ROW = HEAD_LONG_ROW;
constexpr uint32_t RUN_LONG = 0x80000000u;


// v from lane (lane ^ J): DPP quad permutations for 1 and 2, swizzles
// within 32 lanes for 4..16, a permute for 32.  The sort below is bound by
// vector issue and the LDS crossbar together: swizzles for 1 and 2 (0.58 ->
// 0.61 ms), a DPP row rotation for 8 (even), two DPP moves for 4 or the
// permlane16/32 swaps for 16 and 32 (0.71-0.79 ms) all measured no better.
template <int J>
__device__ __forceinline__ uint32_t xor_move(uint32_t v)
{
    // quad permutations give every lane a source: no old value needed
    if constexpr (J == 1)
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);  // [1,0,3,2]
    else if constexpr (J == 2)
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);  // [2,3,0,1]
    else if constexpr (J <= 16)
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (J << 10));
    else
        return (uint32_t)__builtin_amdgcn_ds_bpermute((int)((__lane_id() ^ (uint32_t)J) << 2),
                                                      (int)v);
}

template <int J>
__device__ __forceinline__ uint64_t xor_move64(uint64_t v)
{
    return ((uint64_t)xor_move<J>((uint32_t)(v >> 32)) << 32) | xor_move<J>((uint32_t)v);
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

#ifndef BITONIC_SGPR_SELECT
#define BITONIC_SGPR_SELECT 1
#endif

// Lanes l of a wave for which bit log2(KK) of l equals bit log2(J): in a
// bitonic step they keep the smaller element of their pair.
constexpr uint64_t keep_min_lanes(int KK, int J)
{
    uint64_t m = 0;
    for (int l = 0; l < 64; ++l)
        if (((l / KK) & 1) == ((l / J) & 1)) m |= 1ull << l;
    return m;
}

// Per lane: mask bit set ? if_set : if_clear (one v_cndmask on a scalar
// lane mask; register operands only).
__device__ __forceinline__ uint32_t select_lanes(uint64_t mask, uint32_t if_set, uint32_t if_clear)
{
    uint32_t r;
    asm volatile("v_cndmask_b32 %0, %1, %2, %3" : "=v"(r) : "v"(if_clear), "v"(if_set), "s"(mask));
    return r;
}

// One compare-exchange step of the bitonic network over 64 lanes (block
// size KK, partner distance J): the lower lane of an ascending pair keeps
// the smaller element.  Elements are (pi, k, payload); with PACKED the run
// index is folded into k and pi is unused.  lb[t] is bit t of the lane id
// (computed once: the direction of a step is then lane-mask arithmetic).
template <bool PACKED, int KK, int J>
__device__ __forceinline__ void bitonic_step(const bool (&lb)[7], uint32_t &pi, uint64_t &k,
                                             uint32_t &pl)
{
    const uint64_t ok = xor_move64<J>(k);
    const uint32_t opl = xor_move<J>(pl);
    bool other_less;
    uint32_t opi = 0;
    if constexpr (PACKED) {
        other_less = ok < k;
    } else {
        opi = xor_move<J>(pi);
        other_less = (opi < pi) | ((opi == pi) & (ok < k));
    }
#if BITONIC_SGPR_SELECT
    (void)lb;
    // the lanes that keep the smaller element are a fixed pattern; the
    // selection mask is then scalar arithmetic on the comparison's lane mask
    constexpr uint64_t KEEP_MIN = keep_min_lanes(KK, J);
    const uint64_t take = ~(__ballot(other_less) ^ KEEP_MIN);
    k = ((uint64_t)select_lanes(take, (uint32_t)(ok >> 32), (uint32_t)(k >> 32)) << 32) |
        select_lanes(take, (uint32_t)ok, (uint32_t)k);
    pl = select_lanes(take, opl, pl);
    if constexpr (!PACKED) pi = select_lanes(take, opi, pi);
#else
    const bool keep_min = lb[ilog2(KK)] == lb[ilog2(J)];
    const bool take = keep_min == other_less;
    k = take ? ok : k;
    pl = take ? opl : pl;
    if constexpr (!PACKED) pi = take ? opi : pi;
#endif
}

template <bool PACKED, int KK, int J>
__device__ __forceinline__ void bitonic_merge(const bool (&lb)[7], uint32_t &pi, uint64_t &k,
                                              uint32_t &pl)
{
    bitonic_step<PACKED, KK, J>(lb, pi, k, pl);
    if constexpr (J > 1) bitonic_merge<PACKED, KK, J / 2>(lb, pi, k, pl);
}

template <bool PACKED, int KK>
__device__ __forceinline__ void bitonic_sort(const bool (&lb)[7], uint32_t &pi, uint64_t &k,
                                             uint32_t &pl)
{
    bitonic_merge<PACKED, KK, KK / 2>(lb, pi, k, pl);
    if constexpr (KK < 64) bitonic_sort<PACKED, KK * 2>(lb, pi, k, pl);
}

// The same network over one distinct 32-bit word per lane: one lane move,
// one compare and one select per step instead of three of each.
template <int KK, int J>
__device__ __forceinline__ void bitonic_merge32(uint32_t &w)
{
    const uint32_t ow = xor_move<J>(w);
    constexpr uint64_t KEEP_MIN = keep_min_lanes(KK, J);
    const uint64_t take = ~(__ballot(ow < w) ^ KEEP_MIN);
    w = select_lanes(take, ow, w);
    if constexpr (J > 1) bitonic_merge32<KK, J / 2>(w);
}

template <int KK>
__device__ __forceinline__ void bitonic_sort32(uint32_t &w)
{
    bitonic_merge32<KK, KK / 2>(w);
    if constexpr (KK < 64) bitonic_sort32<KK * 2>(w);
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, uint32_t src)
{
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, (int)src, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), (int)src, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Wave-wide minimum per run of consecutive lanes holding the same root; the
// last lane of each run folds it into r (lanes without a root hold NONE32).
__device__ __forceinline__ void flush_by_root(uint64_t *r, uint32_t root, uint64_t v)
{
    const uint32_t lane = __lane_id();
    const uint32_t prev = __shfl_up(root, 1);
    bool head = lane == 0 || prev != root;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t ov = __shfl_up(v, d);
        const bool oh = __shfl_up(head ? 1 : 0, d) != 0;
        if (lane >= (uint32_t)d && !head) {
            v = ov < v ? ov : v;
            head = oh;
        }
    }
    const uint32_t next = __shfl_down(root, 1);
    const bool last = lane == 63 || next != root;
    if (!last || root == NONE32 || v == KEY_INF) return;
    min_into(r, root, v);
}

}  // namespace

// Runs per row (a row's entries cut at multiples of 64).  One lane per row.
__global__ __launch_bounds__(256) void k_runs_count(const uint32_t *__restrict__ row_ptr,
                                                    int32_t n, uint32_t *__restrict__ rc)
{
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= (uint32_t)n) return;
    const uint32_t s = row_ptr[r], e = row_ptr[r + 1];
    rc[r] = e > s ? ((e - 1u) >> 6) - (s >> 6) + 1u : 0u;
}

// Run descriptors {cur, end, row} in entry order (run roff[r] + t is row r's
// t-th run) and the first run of every chunk.  Rows with few runs are
// written by their lane, longer ones by the whole wave.
__global__ __launch_bounds__(256) void k_runs_write(const uint32_t *__restrict__ row_ptr,
                                                    int32_t n, const uint32_t *__restrict__ roff,
                                                    uint32_t *__restrict__ cur,
                                                    uint32_t *__restrict__ end,
                                                    uint32_t *__restrict__ row,
                                                    uint32_t *__restrict__ cfirst)
{
    const uint32_t lane = __lane_id();
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t s = 0, e = 0, o = 0;
    if (r < (uint32_t)n) {
        s = row_ptr[r];
        e = row_ptr[r + 1];
    }
    const uint32_t nk = e > s ? ((e - 1u) >> 6) - (s >> 6) + 1u : 0u;
    if (nk) o = roff[r];
    auto put = [&](uint32_t rs, uint32_t re, uint32_t rr, uint32_t ro, uint32_t t) {
        const uint32_t c0 = rs >> 6;
        const uint32_t q = t == 0 ? rs : (c0 + t) << 6;
        const uint32_t qe = (c0 + t + 1u) << 6 < re ? (c0 + t + 1u) << 6 : re;
        cur[ro + t] = q;
        end[ro + t] = qe;
        row[ro + t] = rr | (((re - rs) > LONG_ROW) ? RUN_LONG : 0u);
        if ((q & 63u) == 0) cfirst[q >> 6] = ro + t;
    };
    constexpr uint32_t LANE_RUNS = 8;
    if (nk && nk <= LANE_RUNS)
        for (uint32_t t = 0; t < nk; ++t) put(s, e, r, o, t);
    uint64_t lm = __ballot(nk > LANE_RUNS);
    while (lm) {
        const int src = __ffsll((unsigned long long)lm) - 1;
        lm &= lm - 1;
        const uint32_t ls = __shfl(s, src), le = __shfl(e, src), lo = __shfl(o, src);
        const uint32_t lr = __shfl(r, src), lk = __shfl(nk, src);
        for (uint32_t t = lane; t < lk; t += 64) put(ls, le, lr, lo, t);
    }
}

// Order every 64-entry chunk by (run, key) with a bitonic network over the
// lanes (one wave per chunk; keys are distinct within a row, and runs keep
// their places) carrying each entry's chunk offset, write the order to
// perm and store each run's head (its smallest key and its column) into its
// descriptor.  Reads the keys and columns (12 bytes per entry) and writes one
// byte per entry.  The chunk's runs are cfirst[c] .. cfirst[c + 1] - 1 (the
// last chunk ends at *nruns); their starts are flagged in the wave's LDS
// bytes (before: ORed across the lanes, 0.509 -> 0.481 ms on R-MAT s22).
// The network first orders one 32-bit word per entry (run index, the top
// bits of the weight key below the bits all the chunk's keys share, lane):
// a step then moves one register instead of three (0.563 -> 0.537 ms at
// seven chunks per wave).  Entries of one run with equal words are put in
// key order by a few transposition steps, or, past three such pairs, the
// chunk is ordered again by the 64-bit network.  With PACKED (edge ids of
// at most 26 bits) that network's key is one 64-bit word: run index inside
// the chunk, weight key, edge id.
// Chunks one wave orders: their loads (keys, columns, first runs, then the
// runs' starts) are all issued before the first network runs, so the chains
// of dependent loads of different chunks overlap; a run head's column then
// comes from the lane that loaded it, not from a load after the network.
// Five chunks (55-57 VGPRs, nine waves per SIMD) beat seven (67, seven
// waves) once the network was lighter: 0.513 vs 0.537 ms; 2 / 3 / 4 / 10 /
// 14 chunks gave 0.570 / 0.535 / 0.519 / 0.640 / 0.745 ms.
#ifndef SORT_CHUNKS_PER_WAVE
#define SORT_CHUNKS_PER_WAVE 5
#endif
#ifndef SORT_WORD32
#define SORT_WORD32 1
#endif
#ifndef SORT_START_LDS
#define SORT_START_LDS 1
#endif
constexpr int SORT_CH = SORT_CHUNKS_PER_WAVE;

template <bool PACKED>
__global__ __launch_bounds__(256) void k_sort_chunks(const uint32_t *__restrict__ col,
                                                     const uint64_t *__restrict__ key,
                                                     uint8_t *__restrict__ perm,
                                                     const uint32_t *__restrict__ d_nnz,
                                                     const uint32_t *__restrict__ cfirst,
                                                     const uint32_t *__restrict__ nruns,
                                                     const uint32_t *__restrict__ run_cur, int eb,
                                                     uint32_t *__restrict__ hcol,
                                                     uint64_t *__restrict__ hkey)
{
    const uint32_t lane = __lane_id();
    const uint32_t nnz = *d_nnz;  // the grid covers an upper bound
    const uint32_t nch = (nnz + 63u) / 64u;
    const uint32_t c0 = (blockIdx.x * 4u + (threadIdx.x >> 6)) * (uint32_t)SORT_CH;
    if (c0 >= nch) return;  // whole waves
    const uint32_t total = *nruns;
    uint64_t kk[SORT_CH];
    uint32_t cl[SORT_CH], r0[SORT_CH], r1[SORT_CH], rc[SORT_CH];
#pragma unroll
    for (int t = 0; t < SORT_CH; ++t) {
        const uint32_t c = c0 + (uint32_t)t;
        const uint32_t pos = c * 64u + lane;
        kk[t] = c < nch && pos < nnz ? key[pos] : KEY_INF;
        cl[t] = c < nch && pos < nnz ? col[pos] : 0u;
        r0[t] = c < nch ? cfirst[c] : 0u;
        r1[t] = c + 1u < nch ? cfirst[c + 1u] : total;
    }
    // run starts of each chunk, from the run descriptors (OR over the lanes)
#pragma unroll
    for (int t = 0; t < SORT_CH; ++t)
        rc[t] = c0 + (uint32_t)t < nch && r0[t] + lane < r1[t] ? run_cur[r0[t] + lane] : NONE32;
    bool lb[7];
#pragma unroll
    for (int b = 0; b < 7; ++b) lb[b] = (lane >> b) & 1u;
#if SORT_START_LDS
    __shared__ uint8_t flags[4][64];
    const uint32_t wv = threadIdx.x >> 6;
#endif
    const uint64_t emask = (1ull << eb) - 1ull;
#pragma unroll
    for (int t = 0; t < SORT_CH; ++t) {
        const uint32_t c = c0 + (uint32_t)t;
        if (c >= nch) break;  // uniform
        const uint32_t pos = c * 64u + lane;
        const bool valid = pos < nnz;
        uint64_t k = kk[t];
        uint32_t pl = lane;  // carried through the network: the entry's chunk offset
#if SORT_START_LDS
        // one flag byte per chunk offset in the wave's own LDS bytes: the
        // wave's LDS instructions run in order, so no barrier is needed
        flags[wv][lane] = 0;
        if (rc[t] != NONE32) flags[wv][rc[t] & 63u] = 1;
        __builtin_amdgcn_wave_barrier();
        const uint64_t sm = __ballot(flags[wv][lane] != 0);
        __builtin_amdgcn_wave_barrier();
#else
        uint64_t sm = rc[t] != NONE32 ? 1ull << (rc[t] & 63u) : 0ull;
        sm |= xor_move64<1>(sm);
        sm |= xor_move64<2>(sm);
        sm |= xor_move64<4>(sm);
        sm |= xor_move64<8>(sm);
        sm |= xor_move64<16>(sm);
        sm |= xor_move64<32>(sm);
#endif
        const uint64_t vmask = nnz - c * 64u >= 64u ? ~0ull : (1ull << (nnz - c * 64u)) - 1ull;
        const uint64_t starts = sm & vmask;
        const uint32_t below = (uint32_t)__popcll(starts & lanemask_lt());
        const bool is_start = (starts >> lane) & 1ull;
        uint32_t pi = valid ? below + (is_start ? 1u : 0u) - 1u : 63u;  // run inside the chunk
        bool full = true;
#if SORT_WORD32
        {
            // One 32-bit word per entry: run index (pb bits), the bits of the
            // weight key below the highest bit in which the chunk's keys
            // differ (shifted to fit 26 - pb bits: order-preserving, but it
            // may merge keys), and the lane.  Words are distinct, so the
            // network orders the entries by (run, word bits); where two
            // neighbours of one run have equal bits their order is settled
            // on the full keys below.
            const uint32_t nv = nnz - c * 64u >= 64u ? 64u : nnz - c * 64u;
            const uint32_t nr = (uint32_t)__popcll(starts);
            const uint32_t wk = (uint32_t)(k >> 32);
            const uint32_t ref = __builtin_amdgcn_readfirstlane(wk);  // lane 0 is valid
            uint32_t x = valid ? wk ^ ref : 0u;
            x |= xor_move<1>(x);
            x |= xor_move<2>(x);
            x |= xor_move<4>(x);
            x |= xor_move<8>(x);
            x |= xor_move<16>(x);
            x |= xor_move<32>(x);
            x = __builtin_amdgcn_readfirstlane(x);
            const uint32_t hb = x ? 32u - (uint32_t)__clz((int)x) : 0u;
            const uint32_t pb = nr > 1u ? 32u - (uint32_t)__clz((int)(nr - 1u)) : 0u;
            const uint32_t vb = 26u - pb;
            const uint32_t sh = hb > vb ? hb - vb : 0u;
            const uint32_t lowm = hb >= 32u ? ~0u : (1u << hb) - 1u;
            const uint32_t v = (wk & lowm) >> sh;
            uint32_t w = valid ? (pb ? pi << (32u - pb) : 0u) | (v << 6) | lane
                               : 0xFFFFFFC0u | lane;  // after every valid word
            bitonic_sort32<2>(w);
            const uint32_t wp = __shfl_up(w, 1);
            const bool tie = lane > 0 && lane < nv && (wp >> 6) == (w >> 6);
            const uint64_t tm = __ballot(tie);
            const int nt = __popcll(tm);
            // more than three tied pairs: the 64-bit network instead
            if (nt <= 3) {
                full = false;
                pl = w & 63u;
                k = shfl_u64(kk[t], pl);
                if (nt) {
                    // groups of at most four: four odd-even transposition
                    // phases on the full keys, within tied neighbours only
#pragma unroll
                    for (int ph = 0; ph < 4; ++ph) {
                        const uint32_t q = (ph & 1) ? ((lane & 1u) ? lane + 1u : lane - 1u)
                                                    : lane ^ 1u;
                        const uint32_t pq = q < 64u ? q : lane;
                        const uint32_t ow = (uint32_t)__shfl((int)w, (int)pq, 64);
                        const uint64_t ok = shfl_u64(k, pq);
                        const bool pair = pq != lane && lane < nv && pq < nv &&
                                          (ow >> 6) == (w >> 6);
                        const bool swap = pair && (lane < pq ? ok < k : k < ok);
                        if (swap) {
                            w = ow;
                            k = ok;
                        }
                    }
                    pl = w & 63u;
                }
            }
        }
#endif
        if (full) {
            if constexpr (PACKED)
                k = valid ? ((uint64_t)pi << 58) | ((k >> 32) << eb) | (k & emask) : ~0ull;
            bitonic_sort<PACKED, 2>(lb, pi, k, pl);
            if constexpr (PACKED) k = (((k >> eb) & 0xFFFFFFFFull) << 32) | (k & emask);
        }
        // the column of the entry now at this lane, from the lane that
        // loaded it (every lane takes part; pl < 64)
        const uint32_t hc = (uint32_t)__shfl((int)cl[t], (int)pl, 64);
        if (valid) {
            perm[pos] = (uint8_t)pl;
            if (is_start) {
                const uint32_t ri = r0[t] + below;
                hcol[ri] = hc;
                hkey[ri] = k;
            }
        }
    }
}

// Phase A (see the top of the file).  Queued runs go to queue[*qn ...].
__global__ __launch_bounds__(256) void k_heads(const uint32_t *__restrict__ run_row,
                                               uint32_t *__restrict__ run_cur,
                                               const uint32_t *__restrict__ run_end,
                                               uint32_t *__restrict__ run_hcol,
                                               uint64_t *__restrict__ run_hkey, uint32_t nruns,
                                               const uint32_t *__restrict__ col,
                                               const uint64_t *__restrict__ key,
                                               const uint8_t *__restrict__ perm,
                                               const uint32_t *__restrict__ p,
                                               uint64_t *__restrict__ r,
                                               uint32_t *__restrict__ queue, uint32_t *qn,
                                               uint32_t want_long)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t hk = i < nruns ? run_hkey[i] : KEY_INF;
    uint32_t rw = 0;
    if (hk != KEY_INF) {
        rw = run_row[i];
        if ((rw & RUN_LONG) != want_long) hk = KEY_INF;  // the other launch's run
    }
    uint32_t root = NONE32;
    uint64_t cand = KEY_INF;
    bool push = false;
    if (hk != KEY_INF) {
        const uint32_t hc = run_hcol[i];
        root = p[rw & ~RUN_LONG];
        // a run whose head is no smaller than the root's current minimum
        // cannot lower it (its keys only grow and r only falls): it is
        // passed over without a gather
        if (hk >= load_relaxed_u64(r + root)) {
            root = NONE32;
        } else if (p[hc] != root) {
            cand = hk;
        } else {
            // the head is internal: probe the next entries together
            const uint32_t cur = run_cur[i], end = run_end[i];
            const uint32_t b = cur + 1u;
            uint32_t cc[HEAD_PROBE], pc[HEAD_PROBE], ce[HEAD_PROBE];
#pragma unroll
            for (int t = 0; t < HEAD_PROBE; ++t) {
                const uint32_t q = b + (uint32_t)t < end ? b + (uint32_t)t : end - 1u;
                ce[t] = (q & ~63u) | perm[q];
            }
#pragma unroll
            for (int t = 0; t < HEAD_PROBE; ++t) cc[t] = col[ce[t]];
#pragma unroll
            for (int t = 0; t < HEAD_PROBE; ++t) pc[t] = p[cc[t]];
            uint32_t f = (uint32_t)HEAD_PROBE, fc = 0, fe = 0;
#pragma unroll
            for (int t = HEAD_PROBE - 1; t >= 0; --t)
                if (b + (uint32_t)t < end && pc[t] != root) {
                    f = (uint32_t)t;
                    fc = cc[t];
                    fe = ce[t];
                }
            if (f < (uint32_t)HEAD_PROBE) {
                const uint32_t nc = b + f;
                cand = key[fe];
                run_cur[i] = nc;
                run_hcol[i] = fc;
                run_hkey[i] = cand;
            } else {
                const uint32_t nc = b + (uint32_t)HEAD_PROBE < end ? b + (uint32_t)HEAD_PROBE : end;
                run_cur[i] = nc;
                push = nc < end;
                if (!push) run_hkey[i] = KEY_INF;
            }
        }
    }
    const uint64_t bal = __ballot(push);
    if (bal) {
        uint32_t base = 0;
        if (__lane_id() == 0) base = atomicAdd(qn, (uint32_t)__popcll(bal));
        base = __shfl(base, 0);
        if (push) queue[base + (uint32_t)__popcll(bal & lanemask_lt())] = i;
    }
    flush_by_root(r, root, cand);
}

// Phase B: one wave per queued run (at most 64 - 1 - HEAD_PROBE entries
// remain).  The grid is fixed; each wave strides over the queue and stops at
// its length.  Also clears the other queue counter for the next round.
__global__ __launch_bounds__(256) void k_heads_rest(
    const uint32_t *__restrict__ queue, const uint32_t *qn, uint32_t *qn_next, uint32_t nruns,
    const uint32_t *__restrict__ run_row, uint32_t *__restrict__ run_cur,
    const uint32_t *__restrict__ run_end, uint32_t *__restrict__ run_hcol,
    uint64_t *__restrict__ run_hkey, const uint32_t *__restrict__ col,
    const uint64_t *__restrict__ key, const uint8_t *__restrict__ perm,
    const uint32_t *__restrict__ p, uint64_t *__restrict__ r)
{
    const uint32_t lane = __lane_id();
    uint32_t n = load_relaxed_u32(qn);
    n = n < nruns ? n : nruns;  // every run is queued at most once
    if (blockIdx.x == 0 && threadIdx.x == 0) *qn_next = 0u;
    const uint32_t nw = gridDim.x * (blockDim.x / 64u);
    for (uint32_t w = blockIdx.x * (blockDim.x / 64u) + (threadIdx.x >> 6); w < n; w += nw) {
        const uint32_t i = queue[w];
        const uint32_t cur = run_cur[i], end = run_end[i];
        const uint32_t root = p[run_row[i] & ~RUN_LONG];
        const uint32_t q = cur + lane;
        uint32_t c = 0, qe = 0;
        bool ext = false;
        if (q < end) {
            qe = (q & ~63u) | perm[q];
            c = col[qe];
            ext = p[c] != root;
        }
        const uint64_t b = __ballot(ext);
        if (b) {
            if (lane == (uint32_t)__ffsll((unsigned long long)b) - 1u) {
                const uint64_t kq = key[qe];
                run_cur[i] = q;
                run_hcol[i] = c;
                run_hkey[i] = kq;
                min_into(r, root, kq);
            }
        } else if (lane == 0) {
            run_cur[i] = end;
            run_hkey[i] = KEY_INF;
        }
    }
}

// ------------------------------------------------------------------ host --

size_t heads_runs_cap(size_t nnz_cap, int32_t n)
{
    return (nnz_cap + 63) / 64 + (size_t)(n > 0 ? n : 0) + 1;
}

msf_status build_runs(Ctx *c, const Runs &R, const uint32_t *row_ptr, int32_t n,
                      const uint32_t *col, const uint64_t *key, uint32_t nnz_max, int eb)
{
    hipStream_t s = c->stream;
    const uint32_t nch = (nnz_max + 63u) / 64u;
    if (nch == 0 || n <= 0) {
        launch_fill_u32(s, &c->dcnt->nruns, 0u, 1);
        return MSF_OK;
    }
    const unsigned gr = (unsigned)(((uint32_t)n + 255u) / 256u);
    k_runs_count<<<gr, 256, 0, s>>>(row_ptr, n, R.rc);
    MSF_TRY(scan_u32(c, R.rc, R.roff, (int64_t)n, &c->dcnt->nruns));
    k_runs_write<<<gr, 256, 0, s>>>(row_ptr, n, R.roff, R.cur, R.end, R.row, R.cfirst);
    const unsigned gs = (nch + 4u * SORT_CH - 1u) / (4u * SORT_CH);
    const uint32_t *total = R.roff + n;  // the scan's total: the number of runs
    MSF_HIP(hipEventRecord(c->kev[2], s));
    const uint32_t *d_nnz = row_ptr + n;  // one slice: the stored entry count
    if (eb <= 26)
        k_sort_chunks<true><<<gs, 256, 0, s>>>(col, key, R.perm, d_nnz, R.cfirst, total, R.cur,
                                               eb, R.hcol, R.hkey);
    else
        k_sort_chunks<false><<<gs, 256, 0, s>>>(col, key, R.perm, d_nnz, R.cfirst, total, R.cur,
                                                eb, R.hcol, R.hkey);
    MSF_HIP(hipEventRecord(c->kev[3], s));
    c->pass_done |= 2u;
    MSF_HIP(hipGetLastError());
    return MSF_OK;
}

// Blocks of the phase-B grid (4 waves each).
constexpr uint32_t HEADS_REST_BLOCKS = 1024;

void launch_heads(hipStream_t s, const Runs &R, uint32_t nruns, const uint32_t *col,
                  const uint64_t *key, const uint32_t *p, uint64_t *r, Counters *dcnt, int parity)
{
    if (nruns == 0) return;
    uint32_t *qn = &dcnt->qn[parity & 1], *qn_next = &dcnt->qn[(parity & 1) ^ 1];
    for (uint32_t want_long : {RUN_LONG, 0u})
        k_heads<<<(nruns + 255u) / 256u, 256, 0, s>>>(R.row, R.cur, R.end, R.hcol, R.hkey, nruns,
                                                      col, key, R.perm, p, r, R.queue, qn,
                                                      want_long);
    k_heads_rest<<<HEADS_REST_BLOCKS, 256, 0, s>>>(R.queue, qn, qn_next, nruns, R.row, R.cur,
                                                   R.end, R.hcol, R.hkey, col, key, R.perm, p, r);
}

}  // namespace msf
