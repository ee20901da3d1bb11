// The multilinear kernel of section 3.1 fused with the projection of
// Algorithm 2, evaluated all-at-once: for every stored
// direction i->j with key k,
//     f(p_i, a_ij, p_j) = k if p_i != p_j, else the empty key,
// reduced with MinWeight (unsigned min of packed keys) over each run of
// entries whose row shares the same root p_i, and written with one 64-bit
// atomicMin per run into r[p_i].  The per-vertex minimum q_i of the paper
// is never materialised: it lives in registers, as in the all-at-once
// formulation that writes n values instead of nnz (section 4.1).
//
// Work split: the nnz stored entries are cut into chunks of SWEEP_CHUNK
// (one workgroup each), independent of row lengths, so skewed degree
// distributions (R-MAT) stay balanced.  Each lane owns SWEEP_E consecutive
// entries (16-byte vector loads of col, two of key); runs that cross lanes
// are merged with a wave-wide segmented scan; the first and last run of a
// wave may be partial and are combined through the atomic.
//
// COMPACT variant (intra-component edge filtering): entries with
// p_i == p_j can never become outgoing again (trees only merge), so the
// sweep also writes the surviving entries, in order, to a second CSR.  The
// chunk's output offset comes from a decoupled look-back over chunk
// survivor counts; row_ptr of the output is written by the lane holding each
// row's first entry.
#include "msf_internal.hpp"
#include "wave.hpp"

namespace msf {

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

struct RunAgg {
    uint32_t first_root, last_root;
    uint32_t hib;  // a run boundary lies inside the span
    uint64_t lrm;  // min over the span's last run
};

__device__ __forceinline__ RunAgg combine(const RunAgg &a, const RunAgg &b)
{
    RunAgg r;
    const bool boundary = a.last_root != b.first_root;
    r.first_root = a.first_root;
    r.last_root = b.last_root;
    r.hib = a.hib | b.hib | (boundary ? 1u : 0u);
    r.lrm = (b.hib || boundary) ? b.lrm : (a.lrm < b.lrm ? a.lrm : b.lrm);
    return r;
}

// One step of the wave-wide segmented scan: every field moved by the same
// DPP control; lanes whose source exists combine it in front of their own.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void scan_step(RunAgg &agg, bool recv)
{
    RunAgg o;
    o.first_root = dpp_u32<CTRL, ROW_MASK>(agg.first_root);
    o.last_root = dpp_u32<CTRL, ROW_MASK>(agg.last_root);
    o.hib = dpp_u32<CTRL, ROW_MASK>(agg.hib);
    o.lrm = dpp_u64<CTRL, ROW_MASK>(agg.lrm);
    if (recv) agg = combine(o, agg);
}

}  // namespace

// Lazy gathers: entries per lane and root whose column parent is gathered
// up front (the smallest keys); the rest only if all of those are internal.
#ifndef SWEEP_LAZY
#define SWEEP_LAZY 1
#endif
// Gathers and row-window loads issued only by the lanes that need them (1;
// measured 2.7% faster on R-MAT s22 with the parents after round 1) or by
// every lane with a clamped index (0).
#ifndef SWEEP_MASKED_GATHER
#define SWEEP_MASKED_GATHER 1
#endif
#ifndef SWEEP_MASKED_WINDOW
#define SWEEP_MASKED_WINDOW 1
#endif
// Lazy sweep with the read filter on (few live roots): read r of each
// lane's roots before gathering, and gather only for entries whose key is
// below it (1).  r only decreases during a sweep, so an entry with a key at
// or above a value read earlier cannot lower it.  With many live roots the
// values read are still mostly empty and the reads would not pay.
#ifndef SWEEP_PRUNE
#define SWEEP_PRUNE 1
#endif
// Bits of k_sweep's filter argument: read r before an atomic and skip
// the ones that cannot lower it (FILTER_READ; with SWEEP_PRUNE also before
// the gathers), and, where r was read before the gathers, go straight to the
// atomic instead of reading r again (FILTER_KNOWN: pays on graphs where
// long rows put many waves on one root, whose slot they would all read
// twice; with many small roots the second read skips more atomics than it
// costs).
constexpr int FILTER_READ = 1, FILTER_KNOWN = 2;

// Rows of a chunk staged in LDS (two per lane); a chunk that spans more
// rows (long runs of rows without entries in its slice) searches row_ptr in
// global memory instead.
constexpr int SWEEP_WIN = 2 * SWEEP_BLOCK;

// Chunk k of slice q covers entries [cb + k*CHUNK, cb + (k+1)*CHUNK) with
// cb = sstart[q] rounded down to 4 entries (16-byte aligned loads); entries
// outside [sstart[q], sstart[q+1]) belong to neighbouring slices and are
// ignored.  Geometry of global chunk c for this lane:
struct ChunkGeom {
    uint32_t q;       // slice
    uint32_t lo, hi;  // first and last row the chunk touches
    uint32_t base;    // first entry of this lane
    int kb, ke;       // this lane's valid entries: [base + kb, base + ke)
};

__device__ __forceinline__ ChunkGeom chunk_geom(const SliceInfo &sl,
                                                const uint32_t *__restrict__ chunk_row, uint32_t c)
{
    ChunkGeom g;
    uint32_t q = 0;
    while (q + 1 < (uint32_t)sl.S && c >= sl.cbase[q + 1]) ++q;
    const uint32_t k = c - sl.cbase[q];
    const uint32_t s_lo = sl.sstart[q], s_hi = sl.sstart[q + 1];
    const uint32_t base = (s_lo & ~3u) + k * (uint32_t)SWEEP_CHUNK + threadIdx.x * SWEEP_E;
    g.q = q;
    g.base = base;
    g.kb = base >= s_lo ? 0 : (int)(s_lo - base < (uint32_t)SWEEP_E ? s_lo - base : SWEEP_E);
    g.ke = base >= s_hi ? 0 : (s_hi - base >= (uint32_t)SWEEP_E ? SWEEP_E : (int)(s_hi - base));
    const uint32_t *crow = chunk_row + sl.cbase[q] + q;
    g.lo = crow[k];
    g.hi = crow[k + 1];
    return g;
}

// Streamed entry loads (non-temporal: each entry is read once per sweep).
// The lane's whole group of entries is always loaded (the arrays are padded),
// so the number of loads does not depend on the chunk; entries outside
// [kb, ke) are masked to column 0 / the empty key.
__device__ __forceinline__ void load_entries(const uint32_t *__restrict__ col,
                                             const uint64_t *__restrict__ key, const ChunkGeom &g,
                                             uint32_t (&cl)[SWEEP_E], uint64_t (&ky)[SWEEP_E])
{
    uint32_t cv[SWEEP_E];
    uint64_t kv[SWEEP_E];
#pragma unroll
    for (int h = 0; h < SWEEP_E / 4; ++h) {
        const uint32_t b = g.base + 4 * h;
        const u32x4 c4 = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(col + b));
        const u64x2 k01 = __builtin_nontemporal_load(reinterpret_cast<const u64x2 *>(key + b));
        const u64x2 k23 =
            __builtin_nontemporal_load(reinterpret_cast<const u64x2 *>(key + b + 2));
        cv[4 * h] = c4.x;
        cv[4 * h + 1] = c4.y;
        cv[4 * h + 2] = c4.z;
        cv[4 * h + 3] = c4.w;
        kv[4 * h] = k01.x;
        kv[4 * h + 1] = k01.y;
        kv[4 * h + 2] = k23.x;
        kv[4 * h + 3] = k23.y;
    }
#pragma unroll
    for (int e = 0; e < SWEEP_E; ++e) {
        const bool v = e >= g.kb && e < g.ke;
        cl[e] = v ? cv[e] : 0u;
        ky[e] = v ? kv[e] : KEY_INF;
    }
}

// Root of the row of each of this lane's valid entries: rows are found by
// binary search over row_ptr values rp_at(lo..hi+1) (one search for the
// first entry, further ones only where a row ends); FIRST: the root is the
// row itself, otherwise p_row(row).
template <bool FIRST, typename RpAt, typename PRow>
__device__ __forceinline__ void entry_roots(RpAt rp_at, PRow p_row, uint32_t lo, uint32_t hi,
                                            uint32_t base, int kb, int ke,
                                            uint32_t (&root)[SWEEP_E])
{
    auto search = [&](uint32_t a, uint32_t b, uint32_t idx) -> uint32_t {
        while (a < b) {
            const uint32_t mid = a + ((b - a + 1) >> 1);
            if (rp_at(mid) <= idx) a = mid;
            else b = mid - 1;
        }
        return a;
    };
    uint32_t row = search(lo, hi, base + kb);
    uint32_t nx = rp_at(row + 1);
    uint32_t prow = FIRST ? row : p_row(row);
#pragma unroll
    for (int e = 0; e < SWEEP_E; ++e) {
        const uint32_t idx = base + e;
        if (e >= kb && e < ke) {
            if (idx >= nx) {
                row = search(row + 1, hi, idx);
                nx = rp_at(row + 1);
                prow = FIRST ? row : p_row(row);
            }
            root[e] = prow;
        }
    }
}

// The same from global memory, for chunks whose rows exceed the LDS window.
// Kept out of line: merged with the LDS variant, the compiler would select
// between an LDS and a global pointer and load through the generic address
// space.
struct LaneRoots {
    uint32_t v[SWEEP_E];
};

template <bool FIRST>
__device__ __attribute__((noinline)) LaneRoots entry_roots_global(const uint32_t *__restrict__ rp,
                                                                  const uint32_t *__restrict__ p,
                                                                  uint32_t lo, uint32_t hi,
                                                                  uint32_t base, int kb, int ke)
{
    LaneRoots out;
#pragma unroll
    for (int e = 0; e < SWEEP_E; ++e) out.v[e] = NONE32;
    entry_roots<FIRST>([&](uint32_t rw) { return rp[rw]; }, [&](uint32_t rw) { return p[rw]; },
                       lo, hi, base, kb, ke, out.v);
    return out;
}

// FIRST: the parent vector is the identity (round 1), so every stored entry
// is outgoing, runs are rows, and no parent is read at all; with a single
// slice a row that lies wholly inside one wave has a single writer and is
// stored without an atomic.
//
// PAIR: the second pass of the pairwise formulation; col then holds each
// stored entry's column parent p_j, written by k_pair_attach, so no parent
// is gathered.
//
// One chunk per workgroup.  Plain sweep: workgroup b serves chunk b / S of
// slice b % S (workgroups are dealt to the XCDs round-robin, so a slice's
// parents stay in one XCD's L2).  Compacting sweep: chunks are taken by
// ticket in increasing order, so every chunk an earlier one waits on in the
// look-back is held by a running workgroup.
template <bool COMPACT, bool FIRST, bool PAIR = false>
__global__ __launch_bounds__(SWEEP_BLOCK) void k_sweep(
    const uint32_t *__restrict__ row_ptr, const uint32_t *__restrict__ col,
    const uint64_t *__restrict__ key, const uint32_t *__restrict__ chunk_row, SliceInfo sl,
    int32_t n, const uint32_t *__restrict__ p, uint64_t *__restrict__ r,
    uint32_t *__restrict__ chunk_wpre, uint32_t *__restrict__ chunk_mask,
    uint32_t *__restrict__ col_out, uint64_t *__restrict__ key_out, uint64_t *status,
    Counters *cnt, uint32_t *__restrict__ wave_live, int read_filter)
{
    static_assert(!(PAIR && (COMPACT || FIRST)), "pairs: the plain sweep of a parent vector");
    constexpr int E = SWEEP_E;
    __shared__ uint32_t s_ticket;
    __shared__ uint32_t s_lds[SWEEP_BLOCK / 64 + 1];
    __shared__ uint64_t s_prefix;
    __shared__ uint32_t s_rp[SWEEP_WIN + 1];
    __shared__ uint32_t s_p[FIRST ? 1 : SWEEP_WIN];

    if (cnt->gdone) return;  // rounds driven on the device: the solve is done
    const uint32_t lane = __lane_id();
    const uint32_t S = (uint32_t)sl.S;
    const uint32_t total = sl.cbase[S];
    uint32_t c;
    if (COMPACT) {
        if (threadIdx.x == 0) s_ticket = atomicAdd(&cnt->ticket, 1u);
        __syncthreads();
        c = s_ticket;
    } else {
        // the sum k_reduce_live adds into, cleared before any workgroup leaves
        if (wave_live && blockIdx.x == 0 && threadIdx.x == 0) cnt->live = 0;
        const uint32_t q = blockIdx.x % S, k = blockIdx.x / S;
        if (k >= sl.cbase[q + 1] - sl.cbase[q]) return;  // slice q has fewer chunks
        c = sl.cbase[q] + k;
    }

    // 1. entries, row window and column parents.  Every load is issued
    //    unconditionally (indices clamped in bounds), so the compiler's count
    //    of outstanding loads stays exact and no wait covers more than the
    //    loads it needs.
    const ChunkGeom g = chunk_geom(sl, chunk_row, c);
    uint32_t cl[E];
    uint64_t ky[E];
    load_entries(col, key, g, cl, ky);
    const uint32_t *__restrict__ rp = row_ptr + (size_t)g.q * ((size_t)n + 1);
    const uint32_t lo = g.lo, hi = g.hi;
    const uint32_t nrows = hi - lo + 1;
    const bool win = nrows <= (uint32_t)SWEEP_WIN;
    const int kb = g.kb, ke = g.ke;
    const uint32_t base = g.base;
    const uint32_t t0 = threadIdx.x, t1 = threadIdx.x + SWEEP_BLOCK;
    uint32_t wr0 = 0, wr1 = 0, wr2 = 0, wp0 = 0, wp1 = 0;
    if (SWEEP_MASKED_WINDOW) {
        if (t0 <= nrows) wr0 = rp[lo + t0];
        if (t1 <= nrows) wr1 = rp[lo + t1];
        if (t0 == 0) wr2 = rp[lo + min((uint32_t)SWEEP_WIN, nrows)];
        if (!FIRST && t0 < nrows) wp0 = p[lo + t0];
        if (!FIRST && t1 < nrows) wp1 = p[lo + t1];
    } else {
        wr0 = rp[lo + min(t0, nrows)];
        wr1 = rp[lo + min(t1, nrows)];
        wr2 = rp[lo + min((uint32_t)SWEEP_WIN, nrows)];
        if (!FIRST) {
            wp0 = p[lo + min(t0, nrows - 1)];
            wp1 = p[lo + min(t1, nrows - 1)];
        }
    }
    // eager variants gather every column parent now, overlapping the
    // window loads; the lazy plain sweep gathers after the row search
    constexpr bool LAZY = !COMPACT && !FIRST && !PAIR;
    uint32_t pc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) pc[e] = PAIR ? cl[e] : (FIRST || LAZY) ? 0u : p[cl[e]];

    // 2. stage the window
    if (win) {
        if (t0 <= nrows) s_rp[t0] = wr0;
        if (t1 <= nrows) s_rp[t1] = wr1;
        if (t0 == 0 && nrows == (uint32_t)SWEEP_WIN) s_rp[SWEEP_WIN] = wr2;
        if (!FIRST) {
            if (t0 < nrows) s_p[t0] = wp0;
            if (t1 < nrows) s_p[t1] = wp1;
        }
    }
    __syncthreads();

    // 3. the root of every entry's row, then runs
    uint32_t root[E];
    uint64_t cand[E];
    bool live[E];
#pragma unroll
    for (int e = 0; e < E; ++e) root[e] = NONE32;
    if (ke > kb) {
        if (win) {
            entry_roots<FIRST>([&](uint32_t rw) { return s_rp[rw - lo]; },
                               [&](uint32_t rw) { return s_p[rw - lo]; }, lo, hi, base, kb, ke,
                               root);
        } else {
            const LaneRoots v = entry_roots_global<FIRST>(rp, p, lo, hi, base, kb, ke);
#pragma unroll
            for (int e = 0; e < E; ++e) root[e] = v.v[e];
        }
    }
    uint32_t dead_found = 0;  // lazy: gathered entries found internal
    // r of each entry's root read before the gathers (pruned lazy sweep)
    uint64_t rv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) rv[e] = KEY_INF;
    const bool pruned = LAZY && SWEEP_PRUNE && (read_filter & FILTER_READ);
    if (LAZY) {
        // Lazy gathers: only the smallest entry of the lane for each root
        // can be the lane's contribution to that root, so its column parent
        // is gathered first; the other entries of a root are gathered only
        // if that entry is internal (p_i == p_j).  Skipped entries have
        // larger keys than a live one of the same root, so the minima are
        // exact.  Loads are unconditional: lanes with nothing to gather read
        // p[lo], a line the whole wave shares.
        // ok: the entry can still lower r of its root (with SWEEP_PRUNE, its
        // key is below the value of r read now: one read per run of equal
        // roots in the lane; the reads of a wave's shared root coalesce)
        bool ok[E];
#pragma unroll
        for (int e = 0; e < E; ++e) ok[e] = e >= kb && e < ke;
        if (pruned) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const bool fresh = ok[e] && (e == kb || root[e] != root[e > 0 ? e - 1 : 0]);
                rv[e] = fresh ? load_relaxed_u64(r + root[e]) : KEY_INF;
            }
#pragma unroll
            for (int e = 1; e < E; ++e)
                if (ok[e] && e > kb && root[e] == root[e - 1]) rv[e] = rv[e - 1];
#pragma unroll
            for (int e = 0; e < E; ++e) ok[e] = ok[e] && ky[e] < rv[e];
        }
        // am: among the SWEEP_LAZY smallest such entries of its root in
        // this lane
        bool am[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            int below = 0;
#pragma unroll
            for (int f = 0; f < E; ++f)
                if (f != e && ok[f] && root[f] == root[e] &&
                    (ky[f] < ky[e] || (ky[f] == ky[e] && f < e)))
                    ++below;
            am[e] = ok[e] && below < SWEEP_LAZY;
        }
        uint32_t pa[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (SWEEP_MASKED_GATHER) pa[e] = am[e] ? p[cl[e]] : 0u;
            else pa[e] = p[am[e] ? cl[e] : lo];
        }
        bool need[E];
        bool any = false;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            live[e] = am[e] && root[e] != pa[e];
            dead_found += (am[e] && root[e] == pa[e]) ? 1u : 0u;
        }
        // a root needs its other entries only if every gathered one is internal
#pragma unroll
        for (int e = 0; e < E; ++e) {
            bool has_live = false;
#pragma unroll
            for (int f = 0; f < E; ++f)
                if (live[f] && root[f] == root[e]) has_live = true;
            need[e] = !has_live && !am[e] && ok[e];
            any |= need[e];
        }
        if (__ballot(any)) {
            uint32_t pb[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (SWEEP_MASKED_GATHER) pb[e] = need[e] ? p[cl[e]] : 0u;
                else pb[e] = p[need[e] ? cl[e] : lo];
            }
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (need[e]) {
                    live[e] = root[e] != pb[e];
                    dead_found += live[e] ? 0u : 1u;
                }
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) cand[e] = live[e] ? ky[e] : KEY_INF;
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            live[e] = e >= kb && e < ke && (FIRST || root[e] != pc[e]);
            cand[e] = live[e] ? ky[e] : KEY_INF;
        }
    }

    // flush one run's minimum: in round 1 with one slice, a row wholly
    // inside this wave's entries (known from the staged window) has no
    // other writer; everything else goes through the atomic
    const uint32_t wave_lo = base - lane * E;
    const uint32_t wave_hi = wave_lo + 64 * E;  // exclusive
    auto flush = [&](uint32_t rt, uint64_t v, uint64_t known) {
        if (v == KEY_INF) return;
        if (FIRST && S == 1 && win && s_rp[rt - lo] >= wave_lo && s_rp[rt + 1 - lo] <= wave_hi)
            r[rt] = v;
        else if (pruned && (read_filter & FILTER_KNOWN)) {
            if (v < known)
                __hip_atomic_fetch_min(r + rt, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (read_filter & FILTER_READ)
            min_into(r, rt, v);
        else  // many live roots: few runs share one, so the read would not pay
            __hip_atomic_fetch_min(r + rt, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };

    // lane-local runs by root; interior runs are complete and flushed now
    uint32_t froot = NONE32, lroot = NONE32;
    uint64_t fmin = KEY_INF, lmin = KEY_INF, frv = KEY_INF, lrv = KEY_INF;
    bool single = true, started = false;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (e < kb || e >= ke) continue;
        if (!started) {
            froot = lroot = root[e];
            frv = lrv = rv[e];
            fmin = cand[e];
            started = true;
        } else if (root[e] == lroot) {
            if (single) fmin = fmin < cand[e] ? fmin : cand[e];
            else lmin = lmin < cand[e] ? lmin : cand[e];
        } else {
            if (!single) flush(lroot, lmin, lrv);
            single = false;
            lroot = root[e];
            lrv = rv[e];
            lmin = cand[e];
        }
    }

    // wave-wide segmented scan of lane aggregates
    RunAgg agg;
    agg.first_root = froot;
    agg.last_root = lroot;
    agg.hib = single ? 0u : 1u;
    agg.lrm = single ? fmin : lmin;
    // DPP steps (VALU lane moves, no LDS): within rows of 16, then the row
    // aggregates carried across rows; a lane combines only when its source
    // lane exists
    scan_step<DPP_ROW_SHR1, 0xF>(agg, (lane & 15u) >= 1u);
    scan_step<DPP_ROW_SHR2, 0xF>(agg, (lane & 15u) >= 2u);
    scan_step<DPP_ROW_SHR4, 0xF>(agg, (lane & 15u) >= 4u);
    scan_step<DPP_ROW_SHR8, 0xF>(agg, (lane & 15u) >= 8u);
    scan_step<DPP_ROW_BCAST15, 0xA>(agg, ((lane >> 4) & 1u) != 0u);
    scan_step<DPP_ROW_BCAST31, 0xC>(agg, (lane >> 4) >= 2u);
    const uint32_t prev_last = dpp_u32<DPP_WAVE_SHR1>(agg.last_root);
    const uint64_t prev_lrm = dpp_u64<DPP_WAVE_SHR1>(agg.lrm);
    const uint32_t next_first = dpp_u32<DPP_WAVE_SHL1>(froot, NONE32);  // lane 63: none
    if (started) {
        uint64_t ffull = fmin;
        if (lane > 0 && prev_last == froot) ffull = ffull < prev_lrm ? ffull : prev_lrm;
        if (single) {
            if (next_first != froot) flush(froot, ffull, frv);
        } else {
            flush(froot, ffull, frv);
            if (next_first != lroot) flush(lroot, lmin, lrv);
        }
    }

    // live entries: exact in the eager variants; the lazy sweep counts
    // every entry not found internal (an upper bound, for the filtering
    // policy only)
    uint32_t lcnt = 0;
    if (LAZY) {
        lcnt = (uint32_t)(ke > kb ? ke - kb : 0) - dead_found;
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) lcnt += live[e] ? 1u : 0u;
    }

    if (!COMPACT) {
        // live entries of this sweep (filtering policy): one count per wave,
        // summed by k_reduce_live (atomics on one counter would serialise)
        if (wave_live) {
            const uint32_t ws = wave_sum(lcnt);
            if (lane == 0) wave_live[(size_t)c * (SWEEP_BLOCK / 64) + threadIdx.x / 64] = ws;
        }
        return;
    }

    // ---- filtering: order-preserving compaction of live entries ----
    uint32_t btot;
    const uint32_t lex = block_excl_sum<SWEEP_BLOCK>(lcnt, s_lds, &btot);
    if (threadIdx.x < 64) {
        const uint64_t ex = lookback(status, c, (uint64_t)btot);
        if (threadIdx.x == 0) s_prefix = ex;
    }
    __syncthreads();
    const uint64_t P = s_prefix;
    uint32_t pos = (uint32_t)P + lex;
    // survivor bitmask and per-32-entry prefix of this chunk: the output row
    // pointers are derived from them by k_rowptr_compact
    uint32_t nib = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) nib |= (live[e] ? 1u : 0u) << e;
    constexpr uint32_t LPW = 32 / E;  // lanes per 32-entry mask word
    uint32_t word = nib << ((lane % LPW) * E);
#pragma unroll
    for (uint32_t d = 1; d < LPW; d <<= 1) word |= __shfl_xor(word, (int)d, 64);
    if (lane % LPW == 0) {
        const size_t wi = (size_t)c * (SWEEP_CHUNK / 32) + threadIdx.x / LPW;
        chunk_mask[wi] = word;
        chunk_wpre[wi] = pos;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (live[e]) {
            col_out[pos] = cl[e];
            key_out[pos] = ky[e];
            ++pos;
        }
    }
    if (c == total - 1 && threadIdx.x == 0) cnt->nnz_out = (uint32_t)(P + btot);
}

// Output row pointers of a compaction: rp'_q[i] = survivors stored before
// old position rp_q[i] (all survivors when that position is the end).
__global__ void k_rowptr_compact(const uint32_t *__restrict__ row_ptr, int32_t n, SliceInfo sl,
                                 const uint32_t *__restrict__ chunk_wpre,
                                 const uint32_t *__restrict__ chunk_mask, const Counters *cnt,
                                 uint32_t *__restrict__ row_ptr_out)
{
    const uint32_t total = cnt->nnz_out;
    const uint32_t nnz = sl.sstart[sl.S];
    const int64_t count = (int64_t)sl.S * ((int64_t)n + 1);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count; j += stride) {
        const uint32_t x = row_ptr[j];
        uint32_t v = total;
        if (x < nnz) {
            int q = 0;
            while (q + 1 < sl.S && x >= sl.sstart[q + 1]) ++q;
            const uint32_t rel = x - (sl.sstart[q] & ~3u);
            const size_t w = (size_t)(sl.cbase[q] + rel / SWEEP_CHUNK) * (SWEEP_CHUNK / 32) +
                             (rel % SWEEP_CHUNK) / 32;
            v = chunk_wpre[w] + __popc(chunk_mask[w] & ((1u << (rel & 31u)) - 1u));
        }
        row_ptr_out[j] = v;
    }
}

// Sum of the per-wave live counts into cnt->live (cleared by the sweep).
__global__ void k_reduce_live(const uint32_t *__restrict__ wave_live, size_t count,
                              Counters *cnt)
{
    __shared__ uint64_t s_lds[256 / 64 + 1];
    uint64_t v = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (size_t)gridDim.x * blockDim.x)
        v += wave_live[i];
    v = block_sum<256>(v, s_lds);
    if (threadIdx.x == 0 && v) atomicAdd((unsigned long long *)&cnt->live, (unsigned long long)v);
}

void launch_sweep(hipStream_t s, const Adj &a, const uint32_t *p, uint64_t *r, Counters *dcnt,
                  bool first, uint32_t *wave_live, bool read_filter, bool known_flush)
{
    const int filt = (read_filter ? FILTER_READ : 0) | (read_filter && known_flush ? FILTER_KNOWN : 0);
    if (a.nnz == 0) return;
    const unsigned grid = a.sl.maxch * (unsigned)a.sl.S;  // slice = workgroup % S
    if (first)
        k_sweep<false, true><<<grid, SWEEP_BLOCK, 0, s>>>(
            a.row_ptr, a.col, a.key, a.chunk_row, a.sl, a.n, p, r, nullptr, nullptr, nullptr,
            nullptr, nullptr, dcnt, wave_live, filt);
    else
        k_sweep<false, false><<<grid, SWEEP_BLOCK, 0, s>>>(
            a.row_ptr, a.col, a.key, a.chunk_row, a.sl, a.n, p, r, nullptr, nullptr, nullptr,
            nullptr, nullptr, dcnt, wave_live, filt);
    if (wave_live) {
        const size_t count = (size_t)a.nchunks * (SWEEP_BLOCK / 64);
        k_reduce_live<<<64, 256, 0, s>>>(wave_live, count, dcnt);
    }
}

void launch_sweep_compact(hipStream_t s, const Adj &a, const uint32_t *p, uint64_t *r,
                          uint32_t *row_ptr_out, uint32_t *col_out, uint64_t *key_out,
                          uint32_t *chunk_info, uint64_t *status, Counters *dcnt,
                          bool read_filter)
{
    if (a.nnz == 0) return;
    uint32_t *wpre = chunk_info;
    uint32_t *mask = chunk_info + (size_t)a.nchunks * (SWEEP_CHUNK / 32);
    launch_zero_lookback(s, status, a.nchunks, &dcnt->ticket, 1, nullptr, 0);
    k_sweep<true, false><<<a.nchunks, SWEEP_BLOCK, 0, s>>>(
        a.row_ptr, a.col, a.key, a.chunk_row, a.sl, a.n, p, r, wpre, mask, col_out, key_out,
        status, dcnt, nullptr, read_filter ? 1 : 0);
    size_t g = ((size_t)a.sl.S * ((size_t)a.n + 1) + 255) / 256;
    if (g > 8192) g = 8192;
    k_rowptr_compact<<<(unsigned)g, 256, 0, s>>>(a.row_ptr, a.n, a.sl, wpre, mask, dcnt,
                                                 row_ptr_out);
}

// First pass of the pairwise formulation (section 4.1): the pair
// (a_ij, p_j) of every stored entry, kept as p_j beside the entry's key.
// Covers the whole padded extent of the column array; slots outside the
// stored entries hold no column, so the gather index is clamped (their
// values are never used).
// Four entries per 16-byte load and store, two groups per thread and step
// (eight gathers in flight); the last extent % 4 entries one by one.
__device__ __forceinline__ u32x4 pair_gather(u32x4 c, const uint32_t *__restrict__ p, uint32_t n)
{
    u32x4 o;
    o.x = p[c.x < n ? c.x : 0u];
    o.y = p[c.y < n ? c.y : 0u];
    o.z = p[c.z < n ? c.z : 0u];
    o.w = p[c.w < n ? c.w : 0u];
    return o;
}

__global__ __launch_bounds__(256) void k_pair_attach(const uint32_t *__restrict__ col,
                                                     size_t extent, int32_t n,
                                                     const uint32_t *__restrict__ p,
                                                     uint32_t *__restrict__ pj)
{
    const size_t nv = extent / 4;
    const u32x4 *__restrict__ c4 = reinterpret_cast<const u32x4 *>(col);
    u32x4 *__restrict__ o4 = reinterpret_cast<u32x4 *>(pj);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t v = t0; v < nv; v += 2 * stride) {
        const size_t v1 = v + stride < nv ? v + stride : v;
        const u32x4 a = __builtin_nontemporal_load(c4 + v);
        const u32x4 b = __builtin_nontemporal_load(c4 + v1);
        const u32x4 oa = pair_gather(a, p, (uint32_t)n);
        const u32x4 ob = pair_gather(b, p, (uint32_t)n);
        o4[v] = oa;
        if (v + stride < nv) o4[v1] = ob;
    }
    for (size_t t = nv * 4 + t0; t < extent; t += stride) {
        const uint32_t j = col[t];
        pj[t] = p[j < (uint32_t)n ? j : 0u];
    }
}

void launch_sweep_pairwise(hipStream_t s, const Adj &a, const uint32_t *p, uint64_t *r,
                           uint32_t *pj, size_t extent, Counters *dcnt)
{
    if (a.nnz == 0) return;
    size_t g = (extent / 8 + 255) / 256;  // one thread per two groups of four
    if (g < 1) g = 1;
    if (g > 16384) g = 16384;
    k_pair_attach<<<(unsigned)g, 256, 0, s>>>(a.col, extent, a.n, p, pj);
    const unsigned grid = a.sl.maxch * (unsigned)a.sl.S;
    k_sweep<false, false, true><<<grid, SWEEP_BLOCK, 0, s>>>(
        a.row_ptr, pj, a.key, a.chunk_row, a.sl, a.n, p, r, nullptr, nullptr, nullptr, nullptr,
        nullptr, dcnt, nullptr, 0);
}

size_t chunk_info_words(uint32_t nchunks) { return 2 * (size_t)nchunks * (SWEEP_CHUNK / 32); }

}  // namespace msf
