// Two-level bucketed adjacency build (one column slice): the symmetric
// adjacency matrix A of section 2, both directions of every non-loop edge,
// each carrying the edge's key.
//
// The entries are partitioned by row in two levels and then placed in LDS,
// so that every pass writes whole runs of consecutive addresses instead of
// scattering single entries (which leaves partly written cache lines):
//   A1. per block of edges, an LDS histogram of the coarse buckets (rows
//       [c << L1, (c+1) << L1)), written bucket-major; one scan gives every
//       (bucket, block) its offset (shared with the one-level build);
//   B1. the same blocks expand each edge into its two stored directions,
//       sort LDS tiles of them by coarse bucket and write each bucket's run
//       of the tile contiguously, and beside it each entry's fine bucket
//       within its coarse bucket as one byte;
//   P.  a plan: per coarse bucket, how many level-2 workgroups (TL_E2
//       entries each) cover it, and their prefix;
//   A2. each level-2 workgroup counts its entries per fine bucket (rows
//       [f << L2, (f+1) << L2)) from those bytes; the counts are laid out
//       so one scan makes each fine bucket contiguous, in row order;
//   B2. the level-2 workgroups sort LDS tiles by fine bucket and write runs;
//   C.  one workgroup per fine bucket counts its rows, scans them into
//       row_ptr, places the entries in LDS by row and writes the bucket out
//       in one coalesced sweep (buckets larger than LDS scatter directly).
//       In the solve it also keeps each row's smallest key: round 1 of the
//       multilinear sweep, where the parent vector is the identity.
// Every atomic is an LDS atomic.  Between the passes an entry is one
// 16-byte record (row, column, key): one vector load or store per entry, and
// one run per bucket in flight instead of three.
#include <type_traits>

#include "msf_internal.hpp"
#include "wave.hpp"

namespace msf {

namespace {

#ifndef TL_PART_THREADS
#define TL_PART_THREADS 512
#endif
constexpr int TL_NT = TL_PART_THREADS;  // partition workgroup
#ifndef TL_TILE_ENTRIES
#define TL_TILE_ENTRIES 4096
#endif
constexpr int TL_TILE = TL_TILE_ENTRIES;  // entries per LDS tile
#ifndef TL_E2_ENTRIES
#define TL_E2_ENTRIES 8192
#endif
constexpr int TL_E2 = TL_E2_ENTRIES;  // level-1 entries per level-2 workgroup
#ifndef TL_PLACE_THREADS
#define TL_PLACE_THREADS 512
#endif
constexpr int TC_NT = TL_PLACE_THREADS;  // placement workgroup
#ifndef TL_PLACE_PER_THREAD
#define TL_PLACE_PER_THREAD 8
#endif
constexpr int TC_PT = TL_PLACE_PER_THREAD;  // entries per thread per pass of a placement
constexpr int TC_CAP = TC_NT * TC_PT;        // entries of a one-pass placement
// Copies of each row's placement counter (and minimum): lane l uses copy
// l % C, so lanes of one wave that hold entries of the same row rarely hit
// the same LDS word; at most TC_SLOTS (row, copy) counters per bucket.
#ifndef TL_PLACE_COPIES
#define TL_PLACE_COPIES 2
#endif
static_assert((TL_PLACE_COPIES & (TL_PLACE_COPIES - 1)) == 0, "copies: a power of two");
constexpr uint32_t TC_SLOTS = 512;
__host__ __device__ inline uint32_t tc_copies(int L2)
{
    const uint32_t R = 1u << L2;
    uint32_t c = R >= TC_SLOTS ? 1u : TC_SLOTS / R;
    return c < (uint32_t)TL_PLACE_COPIES ? c : (uint32_t)TL_PLACE_COPIES;
}
// average entries per fine bucket the levels are sized for (at most this
// many, at least half)
#ifndef TL_FINE_ENTRIES
#define TL_FINE_ENTRIES 2048
#endif
constexpr int TL_MAX_NC = 1024;    // coarse buckets
constexpr int TL_MAX_NSUB = 256;   // fine buckets per coarse bucket
constexpr int TL_MAX_L2 = 10;      // log2 rows per fine bucket
// Copies of each bucket's tile counter in the partition passes: lane l
// counts in copy l % TP_C, so fewer lanes of a wave hit the same LDS word;
// a bucket's entries fill its copies' segments in order.
#ifndef TL_PART_COPIES
#define TL_PART_COPIES 2
#endif
constexpr uint32_t TP_C = TL_PART_COPIES;
// packed 12-byte records between the passes when the bits allow: bit 0 for
// the level-1 records, bit 1 for the level-2 ones
#ifndef TL_PACK
#define TL_PACK 1
#endif
// level-2 entries as two arrays, columns (4 bytes) and keys (8 bytes), with
// the row inside the fine bucket from the 2-byte array the level-2 pass
// writes anyway (1), instead of 16-byte records that repeat the row (0)
#ifndef TL_L2_SOA
#define TL_L2_SOA 1
#endif
// copies of the fine histogram's counters (a power of two)
#ifndef TL_HIST2_COPIES
#define TL_HIST2_COPIES 8
#endif
static_assert((TP_C & (TP_C - 1)) == 0, "copies: a power of two");
static_assert(TL_TILE % (2 * TL_NT) == 0, "a tile: whole edges per partition thread");

// In-place exclusive scan of a[0..N) in LDS by an NT-thread workgroup;
// returns the total.  Every thread must call it.
template <int NT>
__device__ uint32_t lds_excl_scan(uint32_t *a, int N, uint32_t *scr)
{
    const int per = (N + NT - 1) / NT;
    const int i0 = (int)threadIdx.x * per;
    uint32_t run = 0;
    for (int j = 0; j < per; ++j)
        if (i0 + j < N) run += a[i0 + j];
    uint32_t tot;
    const uint32_t ex = block_excl_sum<NT>(run, scr, &tot);
    uint32_t acc = ex;
    for (int j = 0; j < per; ++j) {
        if (i0 + j < N) {
            const uint32_t c = a[i0 + j];
            a[i0 + j] = acc;
            acc += c;
        }
    }
    __syncthreads();
    return tot;
}

// Level-2 workgroup b -> coarse bucket c and its index j inside c
// (P[c] <= b < P[c+1]); returns false past the last workgroup.
__device__ __forceinline__ bool l2_block(const uint32_t *__restrict__ P, int NC, uint32_t b,
                                         uint32_t *c, uint32_t *j)
{
    if (b >= P[NC]) return false;
    int lo = 0, hi = NC - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    *c = (uint32_t)lo;
    *j = b - P[lo];
    return true;
}

// Index of (coarse c, fine sub, level-2 workgroup j) in the level-2 count
// table: coarse-major, then fine bucket, then workgroup.
__device__ __forceinline__ size_t t2_index(const uint32_t *__restrict__ P,
                                           const uint32_t *__restrict__ nb2, int nsub, uint32_t c,
                                           uint32_t sub, uint32_t j)
{
    return (size_t)nsub * P[c] + (size_t)sub * nb2[c] + j;
}

// An entry between the passes: x = row, y = column, (z, w) = key.
__device__ __forceinline__ uint4 make_ent(uint32_t row, uint32_t col, uint64_t key)
{
    return make_uint4(row, col, (uint32_t)key, (uint32_t)(key >> 32));
}
__device__ __forceinline__ uint64_t ent_key(const uint4 &x)
{
    return ((uint64_t)x.w << 32) | x.z;
}

// In HBM an entry is either that 16-byte record or, when the bits allow
// (edge id bits + column bits + rb <= 64), a packed 12-byte one:
// x = weight key, (y, z) = edge id << (cb + rb) | column << rb | the row's
// low rb bits; the row's high bits are its bucket, known to the reader.
template <bool PK>
using RecT = typename std::conditional<PK, uint3, uint4>::type;

template <bool PK>
__device__ __forceinline__ RecT<PK> rec_pack(const uint4 &x, uint32_t rb, uint32_t cb)
{
    if constexpr (PK) {
        const uint64_t v = ((uint64_t)x.z << (cb + rb)) | ((uint64_t)x.y << rb) |
                           (uint64_t)(x.x & ((1u << rb) - 1u));
        return make_uint3(x.w, (uint32_t)v, (uint32_t)(v >> 32));
    } else {
        (void)rb;
        (void)cb;
        return x;
    }
}

// rowhi: the bucket's first row (its low rb bits are zero)
template <bool PK>
__device__ __forceinline__ uint4 rec_unpack(const RecT<PK> &p, uint32_t rowhi, uint32_t rb,
                                            uint32_t cb)
{
    if constexpr (PK) {
        const uint64_t v = ((uint64_t)p.z << 32) | p.y;
        const uint32_t row = rowhi | (uint32_t)(v & ((1ull << rb) - 1ull));
        const uint32_t col = (uint32_t)((v >> rb) & ((1ull << cb) - 1ull));
        return make_uint4(row, col, (uint32_t)(v >> (rb + cb)), p.x);
    } else {
        (void)rowhi;
        (void)rb;
        (void)cb;
        return p;
    }
}

}  // namespace

// B1: edges -> coarse buckets, LDS-sorted tiles, runs written contiguously.
// A tile is TL_TILE/2 edges; each thread loads its TL_EP edges into
// registers once (all loads in flight together), then counts, ranks and
// places them through LDS.
constexpr int TL_EP = TL_TILE / 2 / TL_NT;  // edges per thread per tile

template <int WT, bool PK1>
__global__ __launch_bounds__(TL_NT) void k_part_edges(
    const int32_t *__restrict__ edges, const void *__restrict__ w, int64_t m, int32_t n, int L1,
    int NC, int64_t epb, uint32_t nblk, const uint32_t *__restrict__ bo1, int L2, uint32_t cb,
    RecT<PK1> *__restrict__ o1, uint8_t *__restrict__ sub1, Counters *ctr)
{
    const uint32_t smask = (1u << (L1 - L2)) - 1u;
    bool nan = false;  // a NaN weight among the block's edges
    __shared__ uint4 s_ent[TL_TILE];
    __shared__ uint32_t s_run[TL_MAX_NC], s_pos[TL_MAX_NC * TP_C];  // s_pos: [bucket][copy]
    __shared__ uint32_t s_scr[TL_NT / 64 + 1];
    const uint32_t cp = threadIdx.x & (TP_C - 1);
    const int NCC = NC * (int)TP_C;
    for (int c = threadIdx.x; c < NC; c += TL_NT) s_run[c] = bo1[(size_t)c * nblk + blockIdx.x];
    const int64_t e0 = (int64_t)blockIdx.x * epb;
    const int64_t e1 = e0 + epb < m ? e0 + epb : m;
    // the next tile's edges are loaded while the current one is ranked and
    // written (the barriers below wait for LDS only); indices are clamped to
    // the block's last edge so the loads are unconditional (two 4-byte loads
    // per edge: the edge array is only guaranteed 4-byte aligned)
    const int64_t elast = e1 - 1;
    int32_t pu[TL_EP], pv[TL_EP];
    uint32_t pw[TL_EP];
#pragma unroll
    for (int k = 0; k < TL_EP; ++k) {
        int64_t e = e0 + threadIdx.x + (int64_t)k * TL_NT;
        e = e < elast ? e : elast;
        pu[k] = edges[2 * e];
        pv[k] = edges[2 * e + 1];
        pw[k] = ((const uint32_t *)w)[e];
    }
    for (int64_t t0 = e0; t0 < e1; t0 += TL_TILE / 2) {
        int32_t eu[TL_EP], ev[TL_EP];
        uint32_t ew[TL_EP];
        bool ok[TL_EP];
#pragma unroll
        for (int k = 0; k < TL_EP; ++k) {
            const int64_t e = t0 + threadIdx.x + (int64_t)k * TL_NT;
            const bool in = e < e1;
            eu[k] = in ? pu[k] : 0;
            ev[k] = in ? pv[k] : 0;
            ew[k] = in ? pw[k] : 0u;
            ok[k] = in && (uint32_t)eu[k] < (uint32_t)n && (uint32_t)ev[k] < (uint32_t)n &&
                    eu[k] != ev[k];
            if (WT == MSF_W_F32) nan |= in && (ew[k] & 0x7FFFFFFFu) > 0x7F800000u;
        }
#pragma unroll
        for (int k = 0; k < TL_EP; ++k) {
            int64_t e = t0 + TL_TILE / 2 + threadIdx.x + (int64_t)k * TL_NT;
            e = e < elast ? e : elast;
            pu[k] = edges[2 * e];
            pv[k] = edges[2 * e + 1];
            pw[k] = ((const uint32_t *)w)[e];
        }
        for (int c = threadIdx.x; c < NCC; c += TL_NT) s_pos[c] = 0;
        __syncthreads();
        // one LDS atomic per entry: its return value is the entry's rank in
        // its bucket within the tile
        uint32_t ru[TL_EP], rv[TL_EP];
#pragma unroll
        for (int k = 0; k < TL_EP; ++k) {
            ru[k] = rv[k] = 0;
            if (!ok[k]) continue;
            ru[k] = atomicAdd(&s_pos[((uint32_t)eu[k] >> L1) * TP_C + cp], 1u);
            rv[k] = atomicAdd(&s_pos[((uint32_t)ev[k] >> L1) * TP_C + cp], 1u);
        }
        __syncthreads();
        const uint32_t cnt = lds_excl_scan<TL_NT>(s_pos, NCC, s_scr);  // s_pos: starts
#pragma unroll
        for (int k = 0; k < TL_EP; ++k) {
            if (!ok[k]) continue;
            const int64_t e = t0 + threadIdx.x + (int64_t)k * TL_NT;
            uint32_t wk = ew[k];
            if (WT == MSF_W_F32) wk = wkey_f32_bits(wk);
            const uint64_t key = ((uint64_t)wk << 32) | (uint64_t)(uint32_t)e;
            const uint32_t u = (uint32_t)eu[k], v = (uint32_t)ev[k];
            s_ent[s_pos[(u >> L1) * TP_C + cp] + ru[k]] = make_ent(u, v, key);
            s_ent[s_pos[(v >> L1) * TP_C + cp] + rv[k]] = make_ent(v, u, key);
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < cnt; i += TL_NT) {
            const uint4 x = s_ent[i];
            const uint32_t c = x.x >> L1;
            const uint32_t pos = s_run[c] + (i - s_pos[c * TP_C]);
            o1[pos] = rec_pack<PK1>(x, (uint32_t)L1, cb);
            sub1[pos] = (uint8_t)((x.x >> L2) & smask);
        }
        __syncthreads();
        for (int c = threadIdx.x; c < NC; c += TL_NT) {
            const uint32_t end = c + 1 < NC ? s_pos[(c + 1) * TP_C] : cnt;
            s_run[c] += end - s_pos[c * TP_C];
        }
        __syncthreads();
    }
    if (WT == MSF_W_F32 && __ballot(nan) && __lane_id() == 0) atomicOr(&ctr->err, ERR_NAN);
}

// P: coarse bucket starts cs[0..NC] (cs[NC] = total), level-2 workgroups
// per coarse bucket nb2[c] and their prefix P[0..NC].  One workgroup.
__global__ __launch_bounds__(1024) void k_tl_plan(const uint32_t *__restrict__ bo1, uint32_t nblk,
                                                  int NC, uint32_t *__restrict__ cs,
                                                  uint32_t *__restrict__ nb2,
                                                  uint32_t *__restrict__ P)
{
    __shared__ uint32_t s[TL_MAX_NC];
    __shared__ uint32_t scr[1024 / 64 + 1];
    const uint32_t total = bo1[(size_t)NC * nblk];
    for (int c = threadIdx.x; c < NC; c += 1024) {
        const uint32_t a = bo1[(size_t)c * nblk];
        const uint32_t b = c + 1 < NC ? bo1[(size_t)(c + 1) * nblk] : total;
        const uint32_t k = (b - a + TL_E2 - 1) / TL_E2;
        cs[c] = a;
        nb2[c] = k;
        s[c] = k;
    }
    __syncthreads();
    const uint32_t tot = lds_excl_scan<1024>(s, NC, scr);
    for (int c = threadIdx.x; c < NC; c += 1024) P[c] = s[c];
    if (threadIdx.x == 0) {
        P[NC] = tot;
        cs[NC] = total;
    }
}

// A2: per level-2 workgroup, its entries per fine bucket, read from the
// fine-bucket bytes four at a time (the byte array is padded to whole words).
__global__ __launch_bounds__(256) void k_tl_hist2(const uint8_t *__restrict__ sub1,
                                                  int nsub, int NC, const uint32_t *__restrict__ cs,
                                                  const uint32_t *__restrict__ nb2,
                                                  const uint32_t *__restrict__ P,
                                                  uint32_t *__restrict__ t2)
{
    // TH_C copies of every counter, [fine][copy]; summed at the end
    constexpr uint32_t TH_C = TL_HIST2_COPIES;
    __shared__ uint32_t s_h[TL_MAX_NSUB * TH_C];
    const uint32_t cp = threadIdx.x & (TH_C - 1);
    uint32_t c, j;
    if (!l2_block(P, NC, blockIdx.x, &c, &j)) return;
    const uint32_t a = cs[c] + j * (uint32_t)TL_E2;
    // 64-bit: a + TL_E2 can pass 2^32 near the largest adjacencies
    const uint32_t e = (uint64_t)a + TL_E2 < (uint64_t)cs[c + 1] ? a + TL_E2 : cs[c + 1];
    for (int s = threadIdx.x; s < nsub * (int)TH_C; s += 256) s_h[s] = 0;
    __syncthreads();
    const uint32_t *sw = reinterpret_cast<const uint32_t *>(sub1);
    const uint32_t w0 = a >> 2, w1 = (uint32_t)(((uint64_t)e + 3) >> 2);
    for (uint64_t b = w0; b < w1; b += 256 * 4) {
        uint32_t ww[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint64_t i = b + threadIdx.x + 256u * k;
            ww[k] = i < w1 ? sw[i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint64_t i = b + threadIdx.x + 256u * k;
            if (i >= w1) continue;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint64_t pos = 4 * i + t;
                if (pos >= a && pos < e)
                    atomicAdd(&s_h[((ww[k] >> (8 * t)) & 0xFFu) * TH_C + cp], 1u);
            }
        }
    }
    __syncthreads();
    for (int s = threadIdx.x; s < nsub; s += 256) {
        uint32_t t = 0;
        for (uint32_t q = 0; q < TH_C; ++q) t += s_h[s * TH_C + q];
        t2[t2_index(P, nb2, nsub, c, s, j)] = t;
    }
}

// B2: coarse-bucket entries -> fine buckets, LDS-sorted tiles, runs
// written contiguously at the scanned offsets o2.  Each thread loads its
// TL_SP entries of a tile into registers once.
constexpr int TL_SP = TL_TILE / TL_NT;  // entries per thread per tile

template <bool PK1, bool PK2, bool SOA, bool SUBC>
__global__ __launch_bounds__(TL_NT) void k_part_sub(
    const RecT<PK1> *__restrict__ e1, int L2, int nsub, int NC, const uint32_t *__restrict__ cs,
    const uint32_t *__restrict__ nb2, const uint32_t *__restrict__ P,
    const uint32_t *__restrict__ o2, uint32_t cb, RecT<PK2> *__restrict__ e2,
    uint32_t *__restrict__ c2, uint64_t *__restrict__ k2, uint16_t *__restrict__ sub2)
{
    __shared__ uint4 s_ent[TL_TILE];
    __shared__ uint32_t s_run[TL_MAX_NSUB], s_pos[TL_MAX_NSUB * TP_C];  // s_pos: [fine][copy]
    __shared__ uint32_t s_scr[TL_NT / 64 + 1];
    uint32_t c, j;
    if (!l2_block(P, NC, blockIdx.x, &c, &j)) return;
    const uint32_t a = cs[c] + j * (uint32_t)TL_E2;
    // 64-bit: a + TL_E2 can pass 2^32 near the largest adjacencies
    const uint32_t e = (uint64_t)a + TL_E2 < (uint64_t)cs[c + 1] ? a + TL_E2 : cs[c + 1];
    const uint32_t mask = (uint32_t)nsub - 1u;
    for (int s = threadIdx.x; s < nsub; s += TL_NT) s_run[s] = o2[t2_index(P, nb2, nsub, c, s, j)];
    const uint32_t cp = threadIdx.x & (TP_C - 1);
    const int nsc = nsub * (int)TP_C;
    int lg = 0;
    while ((1 << lg) < nsub) ++lg;
    const uint32_t L1 = (uint32_t)(L2 + lg), rowhi = c << L1;
    // the next tile's records are loaded while the current one is ranked and
    // written (the barriers below wait for LDS only, so the loads stay in
    // flight across them)
    // (indices clamped to the last entry: unconditional loads keep the
    // compiler from waiting for each one in its own branch)
    RecT<PK1> raw[TL_SP];
    const uint64_t last = (uint64_t)e - 1u;
#pragma unroll
    for (int k = 0; k < TL_SP; ++k) {
        const uint64_t i = (uint64_t)a + threadIdx.x + (uint32_t)k * TL_NT;
        raw[k] = e1[i < last ? i : last];
    }
    for (uint64_t t0 = a; t0 < e; t0 += TL_TILE) {
        uint4 xx[TL_SP];
#pragma unroll
        for (int k = 0; k < TL_SP; ++k) {
            const uint64_t i = t0 + threadIdx.x + (uint32_t)k * TL_NT;
            xx[k] = i < e ? rec_unpack<PK1>(raw[k], rowhi, L1, cb) : make_uint4(NONE32, 0u, 0u, 0u);
        }
#pragma unroll
        for (int k = 0; k < TL_SP; ++k) {
            const uint64_t i = t0 + TL_TILE + threadIdx.x + (uint32_t)k * TL_NT;
            raw[k] = e1[i < last ? i : last];
        }
        for (int s = threadIdx.x; s < nsc; s += TL_NT) s_pos[s] = 0;
        __syncthreads();
        uint32_t rk[TL_SP];  // rank in the fine bucket's copy within the tile
#pragma unroll
        for (int k = 0; k < TL_SP; ++k)
            rk[k] = xx[k].x != NONE32
                        ? atomicAdd(&s_pos[((xx[k].x >> L2) & mask) * TP_C + cp], 1u)
                        : 0u;
        __syncthreads();
        const uint32_t cnt = lds_excl_scan<TL_NT>(s_pos, nsc, s_scr);  // s_pos: starts
#pragma unroll
        for (int k = 0; k < TL_SP; ++k)
            if (xx[k].x != NONE32)
                s_ent[s_pos[((xx[k].x >> L2) & mask) * TP_C + cp] + rk[k]] = xx[k];
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < cnt; i += TL_NT) {
            const uint4 x = s_ent[i];
            const uint32_t s = (x.x >> L2) & mask;
            const uint32_t q = s_run[s] + (i - s_pos[s * TP_C]);
            const uint32_t rf = x.x & ((1u << L2) - 1u);  // row inside the fine bucket
            if constexpr (SOA) {
                c2[q] = SUBC ? x.y | (rf << cb) : x.y;
                k2[q] = ent_key(x);
            } else {
                e2[q] = rec_pack<PK2>(x, (uint32_t)L2, cb);
            }
            if constexpr (!SUBC) sub2[q] = (uint16_t)rf;
        }
        __syncthreads();
        for (int s = threadIdx.x; s < nsub; s += TL_NT) {
            const uint32_t end = s + 1 < nsub ? s_pos[(s + 1) * TP_C] : cnt;
            s_run[s] += end - s_pos[s * TP_C];
        }
        __syncthreads();
    }
}

// Start of every fine bucket in the final adjacency: fstart[f] for
// f = c * nsub + sub, and fstart[NC * nsub] = total.
__global__ void k_tl_fstart(const uint32_t *__restrict__ o2, const uint32_t *__restrict__ nb2,
                            const uint32_t *__restrict__ P, int nsub, int NC,
                            uint32_t *__restrict__ fstart)
{
    const uint32_t nf = (uint32_t)NC * (uint32_t)nsub;
    for (uint32_t f = blockIdx.x * blockDim.x + threadIdx.x; f <= nf;
         f += gridDim.x * blockDim.x) {
        const uint32_t c = f < nf ? f / (uint32_t)nsub : (uint32_t)NC;
        const uint32_t sub = f < nf ? f % (uint32_t)nsub : 0u;
        fstart[f] = f < nf ? o2[t2_index(P, nb2, nsub, c, sub, 0)] : o2[(size_t)nsub * P[NC]];
    }
}

// Order of the placement workgroups: fine buckets above the one-pass
// capacity first (from the front, ascending), the rest after them (from the
// back).  A bucket with a hub row can hold 10^5 entries and keeps one
// workgroup busy for a long time; started first, it overlaps the many small
// buckets instead of running alone at the end.
constexpr int TO_NT = 256, TO_IT = 16, TO_TILE = TO_NT * TO_IT;

__global__ __launch_bounds__(TO_NT) void k_tl_order(const uint32_t *__restrict__ fstart,
                                                    uint32_t nf, uint32_t cap,
                                                    uint32_t *__restrict__ order,
                                                    uint64_t *status, uint32_t *ticket)
{
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_lds[TO_NT / 64 + 1];
    __shared__ uint64_t s_pre;
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t base = tile * TO_TILE + threadIdx.x * TO_IT;
    uint32_t big = 0, ca = 0, cb = 0;
#pragma unroll
    for (int k = 0; k < TO_IT; ++k) {
        const uint32_t f = base + k;
        if (f < nf) {
            if (fstart[f + 1] - fstart[f] > cap) {
                big |= 1u << k;
                ++ca;
            } else {
                ++cb;
            }
        }
    }
    uint32_t oa, ob;
    uint64_t tot;
    tile_offsets2<TO_NT>(tile, ca, cb, status, s_lds, &s_pre, &oa, &ob, &tot);
#pragma unroll
    for (int k = 0; k < TO_IT; ++k) {
        const uint32_t f = base + k;
        if (f >= nf) continue;
        if (big & (1u << k)) order[oa++] = f;
        else order[nf - 1 - ob++] = f;
    }
}

// C: one workgroup per fine bucket f (rows [f << L2, (f+1) << L2)): count,
// scan into row_ptr, place by row.  A bucket's output span is small (tens of
// KB), so its scattered stores merge in L2 before they reach HBM.  MIN:
// also store each row's smallest key into r (round 1 of the sweep).
template <bool MIN, bool PK2, bool SOA, bool SUBC>
__global__ __launch_bounds__(TC_NT) void k_tl_place(
    const RecT<PK2> *__restrict__ e2, int32_t n, int L2, uint32_t cb,
    const uint32_t *__restrict__ fstart,
    const uint32_t *__restrict__ order, uint32_t *__restrict__ row_ptr,
    uint32_t *__restrict__ col, uint64_t *__restrict__ key, uint64_t *__restrict__ r,
    const uint16_t *__restrict__ sub2, const uint32_t *__restrict__ c2,
    const uint64_t *__restrict__ k2)
{
    extern __shared__ uint64_t tc_lds[];
    const uint32_t R = 1u << L2;
    const uint32_t C = tc_copies(L2), RC = R * C;  // counters are [row][copy]
    const uint32_t cmask = SUBC ? (cb >= 32 ? ~0u : (1u << cb) - 1u) : ~0u;
    uint64_t *s_min = tc_lds;                                             // RC (MIN)
    uint32_t *s_cnt = reinterpret_cast<uint32_t *>(tc_lds + (MIN ? RC : 0));  // RC
    const uint32_t cp = threadIdx.x & (C - 1);  // this lane's copy
    __shared__ uint32_t s_scr[TC_NT / 64 + 1];
    const uint32_t f = order[blockIdx.x];
    const int64_t row0 = (int64_t)f << L2;
    if (row0 >= n) return;
    const uint32_t rows = (uint32_t)((int64_t)n - row0 < (int64_t)R ? (int64_t)n - row0 : R);
    const uint32_t fs = fstart[f], fe = fstart[f + 1];
    for (uint32_t i = threadIdx.x; i < RC; i += TC_NT) {
        s_cnt[i] = 0;
        if (MIN) s_min[i] = KEY_INF;
    }
    __syncthreads();
    // a row's entries take the segments of its copies in copy order; the
    // row starts where its copy 0 does
    if (fe - fs <= (uint32_t)TC_CAP) {
        // one batch: the counting atomic's return value is the entry's rank
        // in its row, so every entry takes a single LDS atomic
        uint32_t rl[TC_PT], cc[TC_PT], rk[TC_PT];
        uint64_t kk[TC_PT];
#pragma unroll
        for (int k = 0; k < TC_PT; ++k) {
            const uint64_t i = (uint64_t)fs + threadIdx.x + (uint32_t)k * TC_NT;
            if constexpr (SOA && SUBC) {
                const uint32_t w = i < fe ? c2[i] : 0u;
                rl[k] = i < fe ? w >> cb : NONE32;
                cc[k] = w & cmask;
                kk[k] = i < fe ? k2[i] : KEY_INF;
            } else if constexpr (SOA) {
                rl[k] = i < fe ? (uint32_t)sub2[i] : NONE32;
                cc[k] = i < fe ? c2[i] : 0u;
                kk[k] = i < fe ? k2[i] : KEY_INF;
            } else {
                const uint4 x = i < fe ? rec_unpack<PK2>(e2[i], (uint32_t)row0, (uint32_t)L2, cb)
                                       : make_uint4(NONE32, 0u, 0u, 0u);
                rl[k] = x.x != NONE32 ? x.x - (uint32_t)row0 : NONE32;
                cc[k] = x.y;
                kk[k] = ent_key(x);
            }
        }
#pragma unroll
        for (int k = 0; k < TC_PT; ++k) {
            rk[k] = 0;
            if (rl[k] == NONE32) continue;
            rk[k] = atomicAdd(&s_cnt[rl[k] * C + cp], 1u);
            if (MIN)
                atomicMin((unsigned long long *)&s_min[rl[k] * C + cp], (unsigned long long)kk[k]);
        }
        __syncthreads();
        lds_excl_scan<TC_NT>(s_cnt, (int)RC, s_scr);
        for (uint32_t i = threadIdx.x; i < rows; i += TC_NT) row_ptr[row0 + i] = fs + s_cnt[i * C];
        if (row0 + rows == (int64_t)n && threadIdx.x == 0) row_ptr[n] = fe;
#pragma unroll
        for (int k = 0; k < TC_PT; ++k) {
            if (rl[k] == NONE32) continue;
            const uint32_t p = s_cnt[rl[k] * C + cp] + rk[k];
            col[fs + p] = cc[k];
            key[fs + p] = kk[k];
        }
    } else {
        for (uint64_t b = fs; b < fe; b += TC_NT * TC_PT) {
            uint32_t rl[TC_PT];
#pragma unroll
            for (int k = 0; k < TC_PT; ++k) {
                const uint64_t i = b + threadIdx.x + (uint32_t)k * TC_NT;
                if constexpr (SOA && SUBC) rl[k] = i < fe ? c2[i] >> cb : NONE32;
                else rl[k] = i < fe ? (uint32_t)sub2[i] : NONE32;
            }
#pragma unroll
            for (int k = 0; k < TC_PT; ++k)
                if (rl[k] != NONE32) atomicAdd(&s_cnt[rl[k] * C + cp], 1u);
        }
        __syncthreads();
        lds_excl_scan<TC_NT>(s_cnt, (int)RC, s_scr);
        for (uint32_t i = threadIdx.x; i < rows; i += TC_NT) row_ptr[row0 + i] = fs + s_cnt[i * C];
        if (row0 + rows == (int64_t)n && threadIdx.x == 0) row_ptr[n] = fe;
        __syncthreads();
        for (uint64_t b = fs; b < fe; b += TC_NT * TC_PT) {
            uint32_t rl[TC_PT], cc[TC_PT];
            uint64_t kk[TC_PT];
#pragma unroll
            for (int k = 0; k < TC_PT; ++k) {
                const uint64_t i = b + threadIdx.x + (uint32_t)k * TC_NT;
                if constexpr (SOA && SUBC) {
                    const uint32_t w = i < fe ? c2[i] : 0u;
                    rl[k] = i < fe ? w >> cb : NONE32;
                    cc[k] = w & cmask;
                    kk[k] = i < fe ? k2[i] : KEY_INF;
                } else if constexpr (SOA) {
                    rl[k] = i < fe ? (uint32_t)sub2[i] : NONE32;
                    cc[k] = i < fe ? c2[i] : 0u;
                    kk[k] = i < fe ? k2[i] : KEY_INF;
                } else {
                    const uint4 x = i < fe ? rec_unpack<PK2>(e2[i], (uint32_t)row0, (uint32_t)L2,
                                                             cb)
                                           : make_uint4(NONE32, 0u, 0u, 0u);
                    rl[k] = x.x != NONE32 ? x.x - (uint32_t)row0 : NONE32;
                    cc[k] = x.y;
                    kk[k] = ent_key(x);
                }
            }
#pragma unroll
            for (int k = 0; k < TC_PT; ++k) {
                if (rl[k] == NONE32) continue;
                const uint32_t p = atomicAdd(&s_cnt[rl[k] * C + cp], 1u);
                col[fs + p] = cc[k];
                key[fs + p] = kk[k];
                if (MIN)
                    atomicMin((unsigned long long *)&s_min[rl[k] * C + cp],
                              (unsigned long long)kk[k]);
            }
        }
    }
    if (MIN) {
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < rows; i += TC_NT) {
            uint64_t v = s_min[i * C];
            for (uint32_t c = 1; c < C; ++c) v = v < s_min[i * C + c] ? v : s_min[i * C + c];
            r[row0 + i] = v;
        }
    }
}

// ------------------------------------------------------------------ host --

namespace {

int ceil_log2(uint64_t x)
{
    int k = 0;
    while ((1ull << k) < x) ++k;
    return k;
}

}  // namespace

bool two_level_params(int32_t n, int64_t m, TwoLevel *tl)
{
    if (n <= 0 || m <= 0) return false;
    const double avg = (2.0 * (double)m) / (double)n;  // stored entries per row (bound)
    int L2 = 0;
    while (L2 < TL_MAX_L2 && avg * (double)(1u << (L2 + 1)) <= (double)TL_FINE_ENTRIES) ++L2;
    for (;;) {
        const uint64_t F = ((uint64_t)n + (1ull << L2) - 1) >> L2;
        int lg = (ceil_log2(F) + 1) / 2;
        if (lg > 8) lg = 8;
        int L1 = L2 + lg;
        uint64_t NC = ((uint64_t)n + (1ull << L1) - 1) >> L1;
        while (NC > (uint64_t)TL_MAX_NC && lg < 8) {
            ++lg;
            ++L1;
            NC = ((uint64_t)n + (1ull << L1) - 1) >> L1;
        }
        if (NC <= (uint64_t)TL_MAX_NC) {
            tl->L1 = L1;
            tl->L2 = L2;
            tl->nsub = 1 << lg;
            tl->NC = (int)NC;
            return true;
        }
        if (++L2 > TL_MAX_L2) return false;
    }
}

namespace {

int bits_for(uint64_t max_value)
{
    int b = 1;
    while (b < 64 && (max_value >> b)) ++b;
    return b;
}

// Everything of the build after the coarse histogram, for one pair of
// record formats (level 1, level 2).
struct TLBufs {
    const uint32_t *bo;
    uint32_t *cs, *nb2, *P, *t2, *o2, *fst, *order;
    uint64_t *ostat;
    void *e1, *e2;
    uint8_t *sub1;
};

template <bool PK1, bool PK2, bool SOA, bool SUBC>
msf_status two_level_passes(Ctx *c, int32_t n, int64_t m, const int32_t *d_edges,
                            const void *d_w, msf_wtype wt, const TwoLevel &tl, int64_t epb,
                            uint32_t nblk, size_t g2max, size_t nt2, uint32_t otiles,
                            uint32_t cb, const TLBufs &B, uint32_t *row_ptr, uint32_t *col,
                            uint64_t *key, uint64_t *r_first)
{
    hipStream_t s = c->stream;
    const int NC = tl.NC;
    auto *e1 = (RecT<PK1> *)B.e1;
    auto *e2 = (RecT<PK2> *)B.e2;
    // level-2 columns, then keys (8-byte aligned), in the same buffer
    const size_t cap = 2 * (size_t)m;
    uint32_t *c2 = (uint32_t *)B.e2;
    uint64_t *k2 = reinterpret_cast<uint64_t *>(((uintptr_t)(c2 + cap) + 7) & ~(uintptr_t)7);
    // B1
    MSF_HIP(hipEventRecord(c->kev[6], s));
    if (wt == MSF_W_F32)
        k_part_edges<MSF_W_F32, PK1><<<nblk, TL_NT, 0, s>>>(
            d_edges, d_w, m, n, tl.L1, NC, epb, nblk, B.bo, tl.L2, cb, e1, B.sub1, c->dcnt);
    else
        k_part_edges<MSF_W_U32, PK1><<<nblk, TL_NT, 0, s>>>(
            d_edges, d_w, m, n, tl.L1, NC, epb, nblk, B.bo, tl.L2, cb, e1, B.sub1, c->dcnt);
    MSF_HIP(hipEventRecord(c->kev[7], s));
    // P, A2, scan, B2
    k_tl_plan<<<1, 1024, 0, s>>>(B.bo, nblk, NC, B.cs, B.nb2, B.P);
    launch_fill_u32(s, B.t2, 0u, nt2);
    k_tl_hist2<<<(unsigned)g2max, 256, 0, s>>>(B.sub1, tl.nsub, NC, B.cs, B.nb2, B.P, B.t2);
    MSF_TRY(scan_u32(c, B.t2, B.o2, (int64_t)nt2, nullptr));
    // the level-1 bytes are dead once the fine histogram has read them:
    // their buffer takes each level-2 entry's row inside its fine bucket
    uint16_t *sub2 = reinterpret_cast<uint16_t *>(B.sub1);
    MSF_HIP(hipEventRecord(c->kev[4], s));
    k_part_sub<PK1, PK2, SOA, SUBC><<<(unsigned)g2max, TL_NT, 0, s>>>(
        e1, tl.L2, tl.nsub, NC, B.cs, B.nb2, B.P, B.o2, cb, e2, c2, k2, sub2);
    MSF_HIP(hipEventRecord(c->kev[5], s));
    // C
    const unsigned nf = (unsigned)NC * (unsigned)tl.nsub;
    k_tl_fstart<<<(nf + 256) / 256, 256, 0, s>>>(B.o2, B.nb2, B.P, tl.nsub, NC, B.fst);
    launch_zero_lookback(s, B.ostat, otiles, &c->dcnt->ticket, 1, nullptr, 0);
    k_tl_order<<<otiles, TO_NT, 0, s>>>(B.fst, nf, (uint32_t)TC_CAP, B.order, B.ostat,
                                       &c->dcnt->ticket);
    const size_t RC = ((size_t)1 << tl.L2) * tc_copies(tl.L2);
    MSF_HIP(hipEventRecord(c->kev[0], s));
    if (r_first)
        k_tl_place<true, PK2, SOA, SUBC><<<nf, TC_NT, 12 * RC, s>>>(
            e2, n, tl.L2, cb, B.fst, B.order, row_ptr, col, key, r_first, sub2, c2, k2);
    else
        k_tl_place<false, PK2, SOA, SUBC><<<nf, TC_NT, 4 * RC, s>>>(
            e2, n, tl.L2, cb, B.fst, B.order, row_ptr, col, key, nullptr, sub2, c2, k2);
    MSF_HIP(hipEventRecord(c->kev[1], s));
    c->pass_done |= 1u | 4u | 8u;
    c->rec1 = PK1 ? 12 : 16;
    c->rec2 = SOA ? 12 : PK2 ? 12 : 16;
    c->sub2 = SUBC ? 0 : 2;
    MSF_HIP(hipGetLastError());
    return MSF_OK;
}

}  // namespace

msf_status build_two_level(Ctx *c, int32_t n, int64_t m, const int32_t *d_edges, const void *d_w,
                           msf_wtype wt, const TwoLevel &tl, uint32_t *row_ptr, uint32_t *col,
                           uint64_t *key, uint64_t *r_first)
{
    const int NC = tl.NC;
    int64_t epb = (m + 2047) / 2048;
    if (epb < 32768) epb = 32768;
    epb = (epb + 255) & ~(int64_t)255;
    const uint32_t nblk = (uint32_t)((m + epb - 1) / epb);
    const size_t nh = (size_t)NC * nblk;
    const size_t cap = 2 * (size_t)m;  // stored entries, at most
    const size_t g2max = (cap + TL_E2 - 1) / TL_E2 + (size_t)NC;
    const size_t nt2 = (size_t)tl.nsub * g2max;
    // packed 12-byte records where edge id, column and the row's low bits
    // fit in 64 bits
    const uint32_t cb = (uint32_t)bits_for((uint64_t)(n > 1 ? n - 1 : 1));
    const int eb = bits_for((uint64_t)(m > 1 ? m - 1 : 1));
    const bool pk1 = (TL_PACK & 1) && eb + (int)cb + tl.L1 <= 64;
    const bool pk2 = !TL_L2_SOA && (TL_PACK & 2) && eb + (int)cb + tl.L2 <= 64;
    void *vbh, *vbo, *ve1, *ve2, *vsub, *vplan, *vt2, *vo2;
    MSF_TRY(ws_get(c, WS_BH, 4 * nh, &vbh));
    MSF_TRY(ws_get(c, WS_BHOFF, 4 * (nh + 1), &vbo));
    MSF_TRY(ws_get(c, WS_TL1, (pk1 ? 12 : 16) * cap, &ve1));
    MSF_TRY(ws_get(c, WS_TL2, (TL_L2_SOA ? 12 * cap + 8 : (pk2 ? 12 : 16) * cap), &ve2));
    MSF_TRY(ws_get(c, WS_TLSUB, 2 * cap + 8, &vsub));  // level-1 u8, then level-2 u16
    MSF_TRY(ws_get(c, WS_TLPLAN, 4 * (3 * (size_t)NC + 3), &vplan));
    MSF_TRY(ws_get(c, WS_T2, 4 * nt2, &vt2));
    MSF_TRY(ws_get(c, WS_T2OFF, 4 * (nt2 + 1), &vo2));
    void *vfs;
    const size_t nfine = (size_t)NC * (size_t)tl.nsub;
    MSF_TRY(ws_get(c, WS_FSTART, 4 * (nfine + 1), &vfs));
    // placement order (nfine u32) and its look-back status (one u64 per tile)
    const uint32_t otiles = (uint32_t)((nfine + TO_TILE - 1) / TO_TILE);
    void *vord;
    MSF_TRY(ws_get(c, WS_TLORDER, 4 * nfine + 8 * (size_t)otiles + 8, &vord));
    TLBufs B;
    B.order = (uint32_t *)vord;
    B.ostat = (uint64_t *)(((uintptr_t)(B.order + nfine) + 7) & ~(uintptr_t)7);
    B.fst = (uint32_t *)vfs;
    uint32_t *bh = (uint32_t *)vbh;
    B.bo = (const uint32_t *)vbo;
    B.cs = (uint32_t *)vplan;
    B.nb2 = B.cs + NC + 1;
    B.P = B.nb2 + NC;
    B.t2 = (uint32_t *)vt2;
    B.o2 = (uint32_t *)vo2;
    B.e1 = ve1;
    B.e2 = ve2;
    B.sub1 = (uint8_t *)vsub;

    // A1 (coarse histogram; also validates endpoints; the weights are
    // validated by B1, which reads them anyway) + scan
    MSF_TRY(launch_bucket_hist(c, d_edges, d_w, m, n, tl.L1, NC, (uint32_t)n, (uint32_t)NC, epb,
                               nblk, wt, bh, false));
    MSF_TRY(scan_u32(c, bh, (uint32_t *)vbo, (int64_t)nh, &c->dcnt->count));
    constexpr bool SOA = TL_L2_SOA != 0;
    // the row inside the fine bucket rides in the level-2 column word
    const bool subc = SOA && c->tl_row_in_col && (int)cb + tl.L2 <= 32;
#define TL_PASSES(P1, P2, SC)                                                                  \
    two_level_passes<P1, P2, SOA, SC>(c, n, m, d_edges, d_w, wt, tl, epb, nblk, g2max, nt2,    \
                                      otiles, cb, B, row_ptr, col, key, r_first)
    if (SOA) {  // level-2 records are not used: their packing does not apply
        if (subc) return pk1 ? TL_PASSES(true, false, true) : TL_PASSES(false, false, true);
        return pk1 ? TL_PASSES(true, false, false) : TL_PASSES(false, false, false);
    }
    if (pk1 && pk2) return TL_PASSES(true, true, false);
    if (pk2) return TL_PASSES(false, true, false);
    if (pk1) return TL_PASSES(true, false, false);
    return TL_PASSES(false, false, false);
#undef TL_PASSES
}

}  // namespace msf
