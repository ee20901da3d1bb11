// Internal declarations of the gfx950 MSF library (not part of the C ABI).
//
// Device data layout (all arrays in HBM, 256-byte aligned):
//   adjacency  CSR over all n vertices, both directions of every non-loop
//              edge stored (the symmetric adjacency matrix A of section 2):
//                row_ptr u32[n+1], col u32[nnz], key u64[nnz]  (SoA)
//              key = (u64)wkey(w_e) << 32 | e, identical in both directions.
//   chunk_row  u32[nchunks+1]: row holding the first entry of each sweep chunk
//   p          u32[n]  parent vector (a star forest at every round start)
//   r          u64[n]  per-root minimum outgoing key (UINT64_MAX = none)
//   h          u32[n]  hook targets, then roots after shortcutting
//   hedge      u32[n]  edge id each root hooked with
//   R, F       u32[n]  compacted lists: live roots, roots that hooked
//   in_forest  u8[m]   forest flags
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <string>

#include "msf.h"

namespace msf {

constexpr uint64_t KEY_INF = ~0ull;
constexpr int MAX_SLICES = 8;
constexpr uint32_t NONE32 = 0xFFFFFFFFu;

// Sweep geometry: a workgroup of SWEEP_BLOCK lanes handles SWEEP_E
// consecutive entries per lane (one chunk of SWEEP_BLOCK*SWEEP_E entries).
#ifndef SWEEP_BLOCK_LANES
#define SWEEP_BLOCK_LANES 256
#endif
#ifndef SWEEP_LANE_ENTRIES
#define SWEEP_LANE_ENTRIES 4
#endif
constexpr int SWEEP_BLOCK = SWEEP_BLOCK_LANES;
constexpr int SWEEP_E = SWEEP_LANE_ENTRIES;
static_assert(SWEEP_E == 4 || SWEEP_E == 8, "a lane owns one or two 16-byte column loads");
constexpr int SWEEP_CHUNK = SWEEP_BLOCK * SWEEP_E;
// Column/key arrays are allocated SWEEP_PAD entries beyond their capacity:
// the sweep loads whole lane groups past the last stored entry (without
// a branch, so the compiler can count outstanding loads exactly).
constexpr size_t SWEEP_PAD = SWEEP_CHUNK;

// Device error flags raised by validation kernels.
enum : uint32_t {
    ERR_ENDPOINT = 1u,
    ERR_NAN = 2u,
    ERR_PARENT = 4u,
    ERR_CYCLE = 8u,
    ERR_STAR = 16u  // round check: a tree that is not a star after shortcutting
};

// ---------------------------------------------------------------- device --

// Order-preserving unsigned key of a float32 weight: -0.0 is +0.0;
// negative values have every bit flipped, non-negative ones gain the sign
// bit, so unsigned comparison of keys follows float comparison.
__device__ __forceinline__ uint32_t wkey_f32_bits(uint32_t b)
{
    if (b == 0x80000000u) b = 0u;
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ uint64_t load_relaxed_u64(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_relaxed_u32(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_relaxed_u32(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// r[slot] <- min(r[slot], v), skipping the atomic when a plain read already
// shows a value <= v (r only decreases within a sweep, so a stale read can
// only cause an unnecessary atomic, never a missed one).
__device__ __forceinline__ void min_into(uint64_t *r, uint32_t slot, uint64_t v)
{
    if (v == KEY_INF) return;
    uint64_t cur = load_relaxed_u64(r + slot);
    if (v < cur) __hip_atomic_fetch_min(r + slot, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ host --

struct DevBuf {
    void *ptr = nullptr;
    size_t cap = 0;
};

// Workspace slots cached per context (grow-only).
enum Slot {
    WS_EDGES, WS_W, WS_SLOT, WS_DEG, WS_ROWPTR, WS_COL, WS_KEY, WS_CHUNKROW,
    WS_ROWPTR2, WS_COL2, WS_KEY2, WS_CHUNKROW2, WS_HWK,
    WS_P, WS_R, WS_H, WS_HEDGE, WS_RL, WS_RL2, WS_FL, WS_FLAGS, WS_IDS,
    WS_STATUS, WS_WLIVE, WS_PART, WS_Q, WS_Q2,
    WS_BATCH0, WS_BATCH1, WS_BATCH2, WS_BATCH3,
    WS_BH, WS_BHOFF, WS_BRLO, WS_BCOL, WS_BKEY, WS_CHUNKINFO,
    WS_TL1, WS_TL2, WS_TLSUB, WS_TLORDER, WS_TLPLAN, WS_T2, WS_T2OFF, WS_FSTART,
    WS_RUNCHUNK, WS_RUNROW, WS_RUNS, WS_RUNPERM, WS_PAIR,
    WS_PORDER, WS_PCTL, WS_PSCRATCH, WS_SCAN,
    WS_COUNT
};

// Small device-side counters, mirrored to pinned host memory per round.
struct Counters {
    uint32_t err;         // ERR_* flags
    uint32_t nR;          // live roots for the next round
    uint32_t nF;          // roots that hooked this round
    uint32_t hooks;       // hooks kept after tie breaking
    uint32_t max_chase;   // longest shortcut chase
    uint32_t ticket;      // tile ticket for look-back scans
    uint32_t nnz_out;     // survivors of a compaction
    uint32_t count;       // generic output count
    uint32_t inf_pos;     // +inf forest weights
    uint32_t inf_neg;     // -inf forest weights
    uint64_t total_u64;   // forest weight (uint32 weights)
    int64_t acc[10];      // exact float accumulator: signed 32-bit digits
    double total_f64;     // finalised forest weight
    uint64_t live;        // live entries counted by the last plain sweep
    uint32_t rows;        // rows with stored entries (counted by update)
    uint32_t segs;        // non-empty (row, slice) segments of an adjacency
    uint32_t sstart[MAX_SLICES + 1];  // slice boundaries of an adjacency
    uint32_t nruns;       // key-sorted runs of the adjacency (head sweep)
    uint32_t qn[2];       // head sweep queue lengths (alternating rounds)
    uint64_t rf;          // tie break: slots taken, roots << 31 | hooks
    uint32_t tdone;       // tie break: workgroups done
    uint32_t roots;       // round check: vertices with p[v] == v at round start
    // rounds driven on the device (graph rounds): set once a round kept no
    // hook (every later kernel of the round sequence returns at once), the
    // kept hooks of the current round, the rounds run and their hooks
    uint32_t gdone;
    uint32_t ghooks;
    uint32_t grounds;
    uint32_t gpad;
    uint32_t ghist[64];
    uint64_t long_entries;  // stored entries in rows of at least WAVE_ROW entries
};

// Key-sorted runs for the head sweep: every 64-entry chunk of the
// adjacency sorted by (row, key); a run is one row's part of one chunk.
struct Runs {
    uint32_t *cfirst = nullptr;  // per chunk: index of its first run
    uint32_t *rc = nullptr;      // per row: runs
    uint32_t *roff = nullptr;    // per row: exclusive prefix of rc (n + 1 entries)
    uint32_t *cur = nullptr;     // per run: its head (first entry not known internal)
    uint32_t *end = nullptr;     // per run: one past its last entry
    uint32_t *row = nullptr;     // per run: its row (bit 31: a long row, swept first)
    uint32_t *hcol = nullptr;    // per run: column of the head
    uint64_t *hkey = nullptr;    // per run: key of the head (UINT64_MAX: run exhausted)
    uint32_t *queue = nullptr;   // runs left to phase B of a sweep
    uint8_t *perm = nullptr;     // per entry: chunk offset of the entry at this sorted position
};

struct SolveBufs {
    uint32_t *rp[2], *col[2], *crow[2], *p, *h, *hedge, *hwk, *R[2], *F, *wlive, *cinfo;
    uint64_t *key[2], *r, *status;
    uint8_t *flags;
    void *part;
};

// Column slices: the stored entries are grouped by the slice of their
// column (S contiguous vertex ranges of slice_w vertices), and inside a
// slice by row.  Sweep workgroup b serves slice b % S, and workgroups are
// dealt to the 8 XCDs round-robin by index, so each XCD gathers parents
// from one slice only and keeps that slice of p in its own L2.

struct SliceInfo {
    int S = 1;
    uint32_t slice_w = 0;                // vertices per slice (multiple of 32)
    uint32_t sstart[MAX_SLICES + 1] = {};  // slice s holds entries [sstart[s], sstart[s+1])
    uint32_t cbase[MAX_SLICES + 1] = {};   // first sweep chunk of slice s
    uint32_t maxch = 0;                  // most chunks in one slice
};

// Device view of an adjacency structure.
struct Adj {
    int32_t n = 0;
    int64_t m = 0;
    uint32_t nnz = 0;
    SliceInfo sl;
    uint32_t *row_ptr = nullptr;    // S*(n+1): slice s at row_ptr + s*(n+1), global positions
    uint32_t *col = nullptr;
    uint64_t *key = nullptr;
    uint32_t *chunk_row = nullptr;  // slice s: chunks of s + 1 entries from cbase[s] + s
    uint32_t nchunks = 0;           // all slices
    uint32_t segs = 0;              // non-empty (row, slice) segments
    const int32_t *edges = nullptr; // endpoint pairs, for hook decoding
    const void *w = nullptr;        // weights, for totals
    msf_wtype wtype = MSF_W_U32;
};

// Slice count for n vertices (columns sliced once p outgrows one L2).
int choose_slices(int32_t n, int64_t m, int forced);
// Fill the chunk layout of a from sl.sstart (host values).
void set_chunks(Adj *a);

struct SolveState {
    int phase = 0;  // 0 idle, 1 build, 2 roots, 3 round, 4 output, 5 done,
                    // 6 device-driven rounds, 7 build and runs (head sweep)
    int32_t n = 0;
    int64_t m = 0;
    const int32_t *edges = nullptr;
    const void *w = nullptr;
    msf_wtype wt = MSF_W_U32;
    int32_t *ids = nullptr;
    SolveBufs b{};
    Adj a;
    uint32_t nR = 0, rows = 0;
    bool rows_pending = false, compact = false;
    bool first_done = false;  // the build wrote round 1's minima into r
    bool heads = false;       // rounds use the head sweep over key-sorted runs
    bool graph = false;       // rounds driven on the device, GRAPH_K at a time
    // rounds on a kept graph's adjacency (connected components): no build,
    // and the final parent vector goes to labels (through perm, if set)
    // instead of the forest output
    bool kept = false;
    uint32_t *labels = nullptr;
    const uint32_t *perm = nullptr;
    Runs runs;
    uint32_t nruns = 0;
    int ri = 0, ai = 0, rounds = 0;
    int sweep_events = 0;     // rounds whose sweep start/end events were recorded
    double live_frac = 1.0;
    msf_stats st{};
};

struct Ctx {
    int device = 0;
    bool async_alloc = false;   // stream-ordered workspace (server slots)
    hipStream_t stream = nullptr;
    DevBuf ws[WS_COUNT];
    Counters *dcnt = nullptr;   // device
    Counters *hcnt = nullptr;   // pinned host mirror
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t sev[2 * 64] = {};  // sweep start/end events, per round
    // one-launch passes (placement, run sort, level-2 and level-1
    // partitions): start/end events, which ran, record bytes per level
    hipEvent_t kev[8] = {};
    unsigned pass_done = 0;
    int rec1 = 0, rec2 = 0;
    int sub2 = 2;  // bytes of the separate row-in-bucket array per level-2 entry
    msf_stats stats{};
    // msf_multilinear recorded sev[0..1] around its sweep; msf_get_stats
    // turns them into sweep_ms[0] once they have completed
    bool ml_pending = false;
    int filter_mode = 1;        // 0 never, 1 adaptive, 2 every round
    double filter_threshold = 0.30;
    bool check_rounds = false;  // read back error flags after every shortcut
    // round 1: 0 generic sweep, 1 identity-parent sweep, 2 row minima
    // written by the adjacency build (falls back to 1 where it cannot)
    int first_round = 2;
    // adjacency build: 0 device-atomic, 1 two-level bucketed where it
    // applies (one slice), 2 one-level bucketed
    int bucketed_build = 1;
    int slices = 0;                  // column slices: 0 automatic, else forced (1..8)
    // rounds after the first on one-slice adjacencies: head sweep over
    // key-sorted runs (1 from a size and an average degree on, 2 always) or
    // full sweep with the filtering policy (0)
    int heads = 1;
    // batched solve: 1 persistent kernel (graphs up to its size limits;
    // larger ones solved one by one), 0 the disjoint union through the
    // round loop
    int batch_mode = 1;
    // msf_solve of graphs with at most this many edges (and state that fits
    // LDS) by one workgroup of the persistent kernel; 0 turns it off
    int64_t small_m = (int64_t)1 << 17;
    // kept graphs (msf_graph_create) store their vertices by decreasing
    // degree class (1) or in the caller's order (0)
    int graph_order = 1;
    // rounds of the full sweep driven on the device, several per host round
    // trip, for graphs of at most graph_rounds_max_n vertices: 0 off, 1 as
    // direct launches, 2 replays of a HIP graph captured once per solve.
    // Their kernels cover all n vertices every round; measured, that pays
    // up to about a million vertices (grid 64^3 1.09 -> 0.91 ms, ER with
    // 10^5 vertices 0.89 -> 0.74 ms) and not at 2^21 (grid 128^3: 2.15 ms
    // host-stepped over compacted root lists, 2.28 ms on the device).
    int graph_rounds = 2;
    int64_t graph_rounds_max_n = (int64_t)1 << 20;
    // two-level build: each level-2 entry's row inside its fine bucket in
    // the high bits of its column word when column bits + L2 <= 32 (1), or
    // in a separate 2-byte array (0)
    int tl_row_in_col = 1;
    // failure-path test hook (MSF_TEST_FAIL_ALLOC_AFTER): after this many
    // workspace allocations the next one is refused once, without calling
    // the allocator (-1: never)
    int64_t fail_alloc_after = -1;
    hipStream_t cap_stream = nullptr;  // private stream the graph is captured on
    hipGraphExec_t gexec = nullptr;    // the captured rounds, for gkey
    uint64_t gkey[16] = {};
    SolveState ss;
};


// Error reporting (thread-local message).
void set_error(const char *fmt, ...);
msf_status hip_fail(hipError_t e, const char *what);

#define MSF_HIP(call)                                              \
    do {                                                           \
        hipError_t _e = (call);                                    \
        if (_e != hipSuccess) return msf::hip_fail(_e, #call);     \
    } while (0)

#define MSF_TRY(call)                                              \
    do {                                                           \
        msf_status _s = (call);                                    \
        if (_s != MSF_OK) return _s;                               \
    } while (0)

// Workspace: returns a device buffer of at least `bytes` for slot s.
msf_status ws_get(Ctx *c, Slot s, size_t bytes, void **out);

// Sync the context stream and copy the counters to the host mirror.
msf_status read_counters(Ctx *c);

// ---- kernels (launch wrappers), all ordered on c->stream -----------------

// Two-level bucketed build (one column slice): coarse buckets of 2^L1 rows
// (NC of them), each cut into nsub fine buckets of 2^L2 rows.
struct TwoLevel {
    int L1 = 0, L2 = 0, nsub = 1, NC = 1;
};
bool two_level_params(int32_t n, int64_t m, TwoLevel *tl);
msf_status build_two_level(Ctx *c, int32_t n, int64_t m, const int32_t *d_edges, const void *d_w,
                           msf_wtype wt, const TwoLevel &tl, uint32_t *row_ptr, uint32_t *col,
                           uint64_t *key, uint64_t *r_first);
// Coarse histogram of the bucketed builds: per block of epb edges, counts
// of the stored directions per bucket (slice of column, row >> lb), written
// bucket-major into bh[nb * nblk]; validates endpoints and weights.
msf_status launch_bucket_hist(Ctx *c, const int32_t *d_edges, const void *d_w, int64_t m,
                              int32_t n, int lb, int nb, uint32_t slice_w, uint32_t nbr,
                              int64_t epb, uint32_t nblk, msf_wtype wt, uint32_t *bh,
                              bool check_w = true);

// Adjacency build (section 2 adjacency matrix, both directions).
// Fills row_ptr[n+1], col/key[nnz] (capacity 2m) and *a; the number of
// stored entries lands in dcnt->count and validation flags in dcnt->err.
// With r_first, the build may also store every row's smallest key into
// r_first[n] (round 1 of the sweep); *first_done says whether it did.
msf_status build_adjacency(Ctx *c, int32_t n, int64_t m, const int32_t *d_edges, const void *d_w,
                           msf_wtype wt, int S, Adj *a, uint32_t *row_ptr, uint32_t *col,
                           uint64_t *key, uint32_t *chunk_row, uint64_t *r_first = nullptr,
                           bool *first_done = nullptr);
uint32_t sweep_nchunks(uint32_t nnz);
// Chunk-row tables of every slice of a (needs a->sl and a->row_ptr).
void launch_chunk_rows_sliced(hipStream_t s, const Adj &a);
// Slice boundaries (rp_s[0], rp_{S-1}[n]) and non-empty segments into dcnt.
void launch_slice_info(hipStream_t s, const Adj &a, Counters *dcnt);
// Rows at least one wave of the sweep long (64 lanes of SWEEP_E entries).
constexpr uint32_t WAVE_ROW = 64 * SWEEP_LANE_ENTRIES;
// dcnt->long_entries = stored entries in rows of at least WAVE_ROW entries
// (one-slice row_ptr of n rows).
void launch_long_entries(hipStream_t s, const uint32_t *row_ptr, int32_t n, Counters *dcnt);
// Exclusive scan of u32 in[0..N) -> out[0..N]; out[N] (and *total_out,
// nullable, device) receive the total.
msf_status scan_u32(Ctx *c, const uint32_t *in, uint32_t *out, int64_t N, uint32_t *total_out);
void launch_chunk_rows(hipStream_t s, const uint32_t *row_ptr, int32_t n, uint32_t nnz,
                       uint32_t *chunk_row, uint32_t nchunks);

// Multilinear sweep (+ optional compaction into out_*).
void launch_fill_u64(hipStream_t s, uint64_t *p, uint64_t v, size_t n);
void launch_fill_u32(hipStream_t s, uint32_t *p, uint32_t v, size_t n);
void launch_iota_u32(hipStream_t s, uint32_t *p, size_t n);
// p = h = identity over n vertices, r = empty when non-null, `words`
// words of flags cleared, in one launch.
void launch_round_state(hipStream_t s, uint32_t *p, uint32_t *h, uint64_t *r, size_t n,
                        uint32_t *flags, size_t words);
// status[0..tiles) = 0, z1[0..n1) = 0, z2[0..n2) = 0 in one launch (n1, n2
// at most a few hundred)
void launch_zero_lookback(hipStream_t s, uint64_t *status, uint32_t tiles, uint32_t *z1,
                          uint32_t n1, uint32_t *z2, uint32_t n2);
// With wave_live (SWEEP_BLOCK/64 u32 per chunk), dcnt->live receives the
// number of live entries (p_i != p_j).
// read_filter: read r before each atomic and skip non-improving updates
// (needed when many runs share a root); otherwise atomics go straight out.
// known_flush (with read_filter): where r was read before the gathers, the
// atomic follows without a second read (for graphs with many long rows).
void launch_sweep(hipStream_t s, const Adj &a, const uint32_t *p, uint64_t *r, Counters *dcnt,
                  bool first = false, uint32_t *wave_live = nullptr, bool read_filter = true,
                  bool known_flush = false);
// The same minima by the pairwise formulation: k_pair_attach writes every
// stored entry's column parent to pj (extent entries: the padded length of
// a.col), then the sweep reads those instead of gathering.
void launch_sweep_pairwise(hipStream_t s, const Adj &a, const uint32_t *p, uint64_t *r,
                           uint32_t *pj, size_t extent, Counters *dcnt);
// Sweep that also writes the surviving entries (p_i != p_j) in order to
// col_out/key_out and their row pointers to row_ptr_out; chunk_info holds
// chunk_info_words(a.nchunks) u32 of per-chunk survivor masks and prefixes.
void launch_sweep_compact(hipStream_t s, const Adj &a, const uint32_t *p, uint64_t *r,
                          uint32_t *row_ptr_out, uint32_t *col_out, uint64_t *key_out,
                          uint32_t *chunk_info, uint64_t *status, Counters *dcnt,
                          bool read_filter = true);
size_t chunk_info_words(uint32_t nchunks);

// Round kernels.  `status` is a look-back status array (>= tiles entries;
// the root list uses tiles + 1 entries as scratch for its per-tile counts);
// `part` holds per-block partials (>= 4096 u32, chase_part_bytes() or
// output_part_bytes(m)).
uint32_t compaction_tiles(uint64_t n);
msf_status launch_init_roots(Ctx *c, const uint32_t *row_ptr, int32_t n, int S, uint32_t *R,
                             uint64_t *status);
// hwk[i]: the weight key (high word of the edge key) of root i's hook;
// identity: p is the identity (round 1), so endpoints need no lookup; with
// row_ptr, col and run_perm (a one-slice adjacency whose 64-entry chunks
// the head sweep ordered by (row, key)) a row inside one chunk gives its
// target directly: the column of its first entry in that order.
void launch_hook(hipStream_t s, const uint32_t *R, uint32_t nR, uint64_t *r, const uint32_t *p,
                 const int32_t *edges, uint32_t *h, uint32_t *hedge, uint32_t *hwk,
                 bool identity = false, const uint32_t *row_ptr = nullptr,
                 const uint32_t *col = nullptr, const uint8_t *run_perm = nullptr,
                 Counters *tb_cnt = nullptr);
// Counts into dcnt->nR, nF; they (and the slot counts) start at zero: the
// hook launched just before with tb_cnt clears them (counts_cleared), else
// this call does.
void launch_tiebreak(hipStream_t s, const uint32_t *R, uint32_t nR, uint32_t *h,
                     const uint32_t *hedge, uint8_t *in_forest, uint32_t *Rnext, uint32_t *F,
                     uint64_t *status, Counters *dcnt, bool counts_cleared = false);
// Also adds the weights of the kept hooks F (from hwk) exactly to dcnt's
// forest-weight sums.
void launch_chase(hipStream_t s, const uint32_t *F, uint32_t nF, uint32_t *h,
                  const uint32_t *hwk, msf_wtype wt, uint32_t *part, Counters *dcnt);
// S > 1: every vertex is updated (stale parents of vertices without
// entries are never read); S == 1: only rows that still have entries.
// all: every vertex (as with S > 1), so p stays exact for every vertex.
// A parent is written only where it changes.
void launch_update_parents(hipStream_t s, const uint32_t *row_ptr, int32_t n, int S, uint32_t *p,
                           const uint32_t *h, uint32_t *part, Counters *dcnt, bool all = false);
int64_t output_tiles(int64_t m);
size_t output_part_bytes(int64_t m);
// bytes `part` needs for launch_chase
size_t chase_part_bytes();
// Fold nb per-block chase partials held in `part` (the layout launch_chase
// uses) into dcnt; returns at once when dcnt->gdone is set.
void launch_chase_fold(hipStream_t s, const uint32_t *part, uint32_t nb, Counters *dcnt);
constexpr unsigned CHASE_MAX_BLOCKS = 2048;

// Head sweep (kernels_heads.hip).  heads_runs_cap: runs of an adjacency of
// at most nnz_cap entries over n rows.  build_runs derives the runs of a
// one-slice adjacency from row_ptr, orders every 64-entry chunk of col/key
// by (row, key) into R.perm (the entries stay where they are) and fills the
// run arrays (keys' edge ids take eb bits); the run count lands in
// dcnt->nruns.  The entry count is read on the device (row_ptr[n]);
// nnz_max, an upper bound of it, sizes the launches.  launch_heads runs one sweep (queue counter
// dcnt->qn[parity], clearing the other one).
size_t heads_runs_cap(size_t nnz_cap, int32_t n);
msf_status build_runs(Ctx *c, const Runs &R, const uint32_t *row_ptr, int32_t n,
                      const uint32_t *col, const uint64_t *key, uint32_t nnz_max, int eb);
void launch_heads(hipStream_t s, const Runs &R, uint32_t nruns, const uint32_t *col,
                  const uint64_t *key, const uint32_t *p, uint64_t *r, Counters *dcnt, int parity);
msf_status launch_output(Ctx *c, const uint8_t *in_forest, int64_t m, const void *w,
                         msf_wtype wt, int32_t *ids, void *part);

// Shortcut of an arbitrary parent vector (msf_shortcut).
void launch_check_parents(hipStream_t s, const uint32_t *p, int32_t n, Counters *dcnt);
void launch_jump_init(hipStream_t s, const uint32_t *q, int32_t n, uint32_t *F, uint64_t *status,
                      Counters *dcnt);
void launch_jump_pass(hipStream_t s, const uint32_t *Fin, uint32_t nF, uint32_t *q,
                      uint32_t *Fout, uint64_t *status, Counters *dcnt);
// Rounds driven on the device (kernels_graphround.hip): one round of
// Algorithm 2 over every vertex with fixed launch sizes, each kernel
// returning at once when dcnt->gdone is set; sweep = false skips the
// multilinear sweep (round 1 minima from the build).  Enqueued K rounds at
// a time, directly or as a captured graph, without host round trips.
struct GraphRound {
    Adj a;
    uint32_t *p, *h, *hedge, *hwk;
    uint64_t *r;
    uint8_t *flags;
    uint32_t *part;
    msf_wtype wt;
};
void enqueue_graph_round(hipStream_t s, const GraphRound &g, Counters *dcnt, bool sweep);
// Round checks (MSF_CHECK_ROUNDS): dcnt->roots = #{v : p[v] == v} (the
// caller clears it), and ERR_STAR if some p[p[v]] != p[v].
void launch_count_roots(hipStream_t s, const uint32_t *p, int32_t n, Counters *dcnt);
void launch_check_stars(hipStream_t s, const uint32_t *p, int32_t n, Counters *dcnt);
void launch_check_roots(hipStream_t s, const uint32_t *p, const uint32_t *q, int32_t n,
                        Counters *dcnt);
// One full pointer-jumping pass over all n vertices; adds the vertices left
// unfinished into dcnt->nR.
void launch_jump_full(hipStream_t s, uint32_t *q, int32_t n, Counters *dcnt);
// Connected components: hooks of the star roots along the edges of r (h,
// hooked roots added into dcnt->nR), then their application to p.
// With star non-null only star roots hook (original AS rounds); in_forest
// (nullable) gets the hooking edges marked.
void launch_cc_hook(hipStream_t s, const uint32_t *p, const uint64_t *r, const int32_t *edges,
                    int32_t n, uint32_t *h, Counters *dcnt, const uint32_t *star = nullptr,
                    uint8_t *in_forest = nullptr);
// Original AS rounds: star flags of p, and one synchronous shortcut step
// (changes added into dcnt->nR).
void launch_star_check(hipStream_t s, const uint32_t *p, int32_t n, uint32_t *star);
void launch_jump_once(hipStream_t s, const uint32_t *src, int32_t n, uint32_t *dst,
                      Counters *dcnt);
void launch_cc_apply(hipStream_t s, const uint32_t *h, int32_t n, uint32_t *p);

void zero_counters(Ctx *c);
msf_status ctx_init(Ctx *c, int device, hipStream_t stream, bool async_alloc);
// Vertex order of a kept graph by decreasing degree class (relabel.hip),
// from its one-slice adjacency built in the caller's order (rp0, col0,
// key0): perm[new] = old, inv[old] = new, and the adjacency renumbered into
// rp (n + 1 words), col, key.  deg holds 2n words, tab
// relabel_table_words(n), seg 2n + 1, seg_row relabel_segments_cap(n, nnz).
msf_status relabel_csr_by_degree(Ctx *c, int32_t n, const uint32_t *rp0, const uint32_t *col0,
                                 const uint64_t *key0, uint32_t *deg, uint32_t *tab,
                                 uint32_t *perm, uint32_t *inv, uint32_t *seg,
                                 uint32_t *seg_row, uint32_t *rp, uint32_t *col, uint64_t *key);
size_t relabel_table_words(int32_t n);
size_t relabel_segments_cap(int32_t n, int64_t nnz);
// edges[e] <- (inv[u], inv[v]) in place
void launch_relabel_edges(hipStream_t s, int32_t *edges, int64_t m, const uint32_t *inv);
// q[i] = p[perm[i]] (a caller's parent vector in the graph's order)
void launch_relabel_gather(hipStream_t s, const uint32_t *p, const uint32_t *perm, int32_t n,
                           uint32_t *q);
// labels[perm[i]] = perm[q[i]] (labels in the graph's order back to caller ids)
void launch_relabel_labels(hipStream_t s, const uint32_t *q, const uint32_t *perm, int32_t n,
                           uint32_t *labels);
// Device address of the static scratch array of msf_solve_batched_noalloc
// on `device` (taken once per device; the device must be current).
msf_status noalloc_init(int device);
void ctx_release_workspace(Ctx *c);
void ctx_release(Ctx *c);
msf_status decode_err(uint32_t err);

// ---- resumable solve (one per context) -----------------------------------
// solve_start enqueues the adjacency build; every later step is enqueued by
// solve_advance once the previous step's counters have reached the host
// (solve_ready polls an event without blocking).  Each step ends with an
// asynchronous copy of the counters to pinned memory, so a driver can keep
// many contexts (each with its own stream) in flight at once.
msf_status solve_start(Ctx *c, int32_t n, int64_t m, const int32_t *d_edges, const void *d_w,
                       msf_wtype wt, int32_t *d_ids);
// The same rounds on a kept graph's adjacency a (connected components,
// section 2.4): the head sweep where a qualifies (kept_heads_eligible, the
// same rule as msf_solve; the run order goes to the workspace), else the
// full sweep without filtering; a itself is only read.  At the end the
// parent vector, every vertex at its tree's root, goes to labels (device
// uint32[n], through perm when the graph has one).
bool kept_heads_eligible(const Ctx *c, const Adj &a);
msf_status solve_start_kept(Ctx *c, const Adj &a, const uint32_t *perm, uint32_t *labels);
bool solve_ready(Ctx *c);
msf_status solve_advance(Ctx *c);
bool solve_done(const Ctx *c);
void solve_result(const Ctx *c, int64_t *count, msf_total *total);

// Whole-graph solve on device inputs (blocking driver of the above); writes
// ids (device) and fills count/total.
msf_status solve_device(Ctx *c, int32_t n, int64_t m, const int32_t *d_edges, const void *d_w,
                        msf_wtype wt, int32_t *d_ids, int64_t *count, msf_total *total);

}  // namespace msf

struct msf_ctx {
    msf::Ctx c;
};

struct msf_graph {
    msf_ctx *ctx = nullptr;
    msf::Adj a;
    // at least a quarter of the stored entries lie in rows of WAVE_ROW or
    // more entries (the multilinear kernel then skips second reads of r)
    bool long_rows = false;
    void *bufs[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    // vertex order of the stored adjacency: perm[internal] = caller id
    // (null: the caller's order)
    uint32_t *perm = nullptr;
};
