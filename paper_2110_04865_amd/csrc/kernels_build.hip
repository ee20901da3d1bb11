// Adjacency build: the symmetric adjacency matrix A of the paper's section 2
// (a_ij = w(i,j); both stored directions carry the edge's key, as the
// tracking remark of section 3.2 suggests carrying (a_ij, i, j) in A).
//
// Three streaming passes over the edge list, no sort:
//   1. degree: per non-loop edge, one returning atomicAdd per endpoint gives
//      the entry's slot inside its row; endpoints and NaN weights validated.
//   2. exclusive scan of degrees -> row_ptr (single pass, decoupled look-back).
//   3. scatter (col, key) of both directions to row_ptr[row] + slot.
#include "msf_internal.hpp"
#include "wave.hpp"

namespace msf {

// --------------------------------------------------------------- fills ---

__global__ void k_fill_u64(uint64_t *p, uint64_t v, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}
__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}
// Look-back preparation in one launch: status[0..tiles) and two short runs
// of u32 counters (z1[0..n1), z2[0..n2)) set to zero.
__global__ void k_zero_lookback(uint64_t *status, uint32_t tiles, uint32_t *z1, uint32_t n1,
                                uint32_t *z2, uint32_t n2)
{
    const uint32_t i0 = blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t i = i0; i < tiles; i += gridDim.x * blockDim.x) status[i] = 0;
    if (i0 < n1) z1[i0] = 0;
    if (i0 < n2) z2[i0] = 0;
}
__global__ void k_iota_u32(uint32_t *p, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = (uint32_t)i;
}

static unsigned grid_for(size_t n, unsigned block = 256, unsigned cap = 8192)
{
    size_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

void launch_fill_u64(hipStream_t s, uint64_t *p, uint64_t v, size_t n)
{
    if (n) k_fill_u64<<<grid_for(n), 256, 0, s>>>(p, v, n);
}
void launch_fill_u32(hipStream_t s, uint32_t *p, uint32_t v, size_t n)
{
    if (n) k_fill_u32<<<grid_for(n), 256, 0, s>>>(p, v, n);
}
void launch_zero_lookback(hipStream_t s, uint64_t *status, uint32_t tiles, uint32_t *z1,
                          uint32_t n1, uint32_t *z2, uint32_t n2)
{
    const uint32_t need = tiles > n1 ? (tiles > n2 ? tiles : n2) : (n1 > n2 ? n1 : n2);
    k_zero_lookback<<<grid_for(need > 0 ? need : 1), 256, 0, s>>>(status, tiles, z1, n1, z2, n2);
}
void launch_iota_u32(hipStream_t s, uint32_t *p, size_t n)
{
    if (n) k_iota_u32<<<grid_for(n), 256, 0, s>>>(p, n);
}

// -------------------------------------------------------------- degree ---

template <int WT>
__global__ void k_degree(const int32_t *__restrict__ edges, const void *__restrict__ w, int64_t m,
                         int32_t n, uint32_t *__restrict__ deg, uint2 *__restrict__ slot,
                         Counters *cnt)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t err = 0;
    for (; e < m; e += stride) {
        const int32_t u = edges[2 * e], v = edges[2 * e + 1];
        if (WT == MSF_W_F32) {
            const uint32_t b = ((const uint32_t *)w)[e];
            if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu)) err |= ERR_NAN;
        }
        if ((uint32_t)u >= (uint32_t)n || (uint32_t)v >= (uint32_t)n) {
            err |= ERR_ENDPOINT;
            slot[e] = make_uint2(NONE32, NONE32);
            continue;
        }
        if (u == v) {
            slot[e] = make_uint2(NONE32, NONE32);  // self-loop: never stored
            continue;
        }
        const uint32_t su = atomicAdd(deg + u, 1u);
        const uint32_t sv = atomicAdd(deg + v, 1u);
        slot[e] = make_uint2(su, sv);
    }
    if (__ballot(err != 0)) {
        // one atomic per wave
        uint32_t any = err;
        for (int d = 32; d >= 1; d >>= 1) any |= __shfl_xor(any, d, 64);
        if (__lane_id() == 0) atomicOr(&cnt->err, any);
    }
}

// ------------------------------------------------------------- scan -----
// Exclusive prefix of u32 values in[0..N) into out[0..N], out[N] = total.
// Tile = SCAN_NT threads x SCAN_IT items.
//
// Up to SCAN3_TILES tiles the scan takes three launches: the tiles' sums,
// one workgroup scanning those sums, then every tile from its offset.  A
// launch of that size has all its tiles resident at once, and one pass with
// a ticket and a decoupled look-back then costs a serial chain of
// device-wide atomics and status reads (measured: 50-54 us for 2048 tiles,
// against a few us of data).  Beyond that, tiles run in waves and the one
// pass reads each item once.
constexpr int SCAN_NT = 256;
constexpr int SCAN_IT = 8;
constexpr int SCAN_TILE = SCAN_NT * SCAN_IT;
constexpr int SCAN_SUMS_NT = 1024;
constexpr int64_t SCAN3_TILES = 16384;

__global__ __launch_bounds__(SCAN_NT) void k_scan_u32(const uint32_t *__restrict__ in,
                                                      uint32_t *__restrict__ out, int64_t N,
                                                      uint64_t *status, Counters *cnt,
                                                      uint32_t *total_out)
{
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_lds[SCAN_NT / 64 + 1];
    __shared__ uint64_t s_excl;
    if (threadIdx.x == 0) s_tile = atomicAdd(&cnt->ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t base = (int64_t)tile * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IT;
    uint32_t v[SCAN_IT];
    uint64_t sum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_IT; ++k) {
        v[k] = (base + k < N) ? in[base + k] : 0u;
        sum += v[k];
    }
    uint64_t tot;
    uint64_t ex = block_excl_sum<SCAN_NT>(sum, s_lds, &tot);
    if (threadIdx.x < 64) {
        uint64_t e = lookback(status, tile, tot);
        if (threadIdx.x == 0) s_excl = e;
    }
    __syncthreads();
    uint64_t run = s_excl + ex;
#pragma unroll
    for (int k = 0; k < SCAN_IT; ++k) {
        if (base + k < N) out[base + k] = (uint32_t)run;
        run += v[k];
    }
    const int64_t ntiles = (N + SCAN_TILE - 1) / SCAN_TILE;
    if ((int64_t)tile == ntiles - 1 && threadIdx.x == SCAN_NT - 1) {
        out[N] = (uint32_t)(s_excl + tot);
        if (total_out) *total_out = (uint32_t)(s_excl + tot);
    }
}

// Three-launch scan, step 1: each tile's sum.
__global__ __launch_bounds__(SCAN_NT) void k_scan_tile_sums(const uint32_t *__restrict__ in,
                                                            int64_t N,
                                                            uint32_t *__restrict__ sums)
{
    __shared__ uint32_t s_lds[SCAN_NT / 64 + 1];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IT;
    uint32_t v[SCAN_IT];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_IT; ++k) v[k] = (base + k < N) ? in[base + k] : 0u;
#pragma unroll
    for (int k = 0; k < SCAN_IT; ++k) sum += v[k];
    const uint32_t tot = block_sum<SCAN_NT>(sum, s_lds);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Step 2, one workgroup: sums[0..T) replaced by their exclusive prefix,
// sums[T] = the total.  Each thread takes a run of consecutive tiles.
__global__ __launch_bounds__(SCAN_SUMS_NT) void k_scan_sums(uint32_t *__restrict__ sums,
                                                            uint32_t T)
{
    __shared__ uint32_t s_lds[SCAN_SUMS_NT / 64 + 1];
    const uint32_t per = (T + SCAN_SUMS_NT - 1) / SCAN_SUMS_NT;
    const uint32_t i0 = threadIdx.x * per;
    uint32_t run = 0;
    for (uint32_t j = 0; j < per; ++j)
        if (i0 + j < T) run += sums[i0 + j];
    uint32_t tot;
    uint32_t acc = block_excl_sum<SCAN_SUMS_NT>(run, s_lds, &tot);
    for (uint32_t j = 0; j < per; ++j) {
        if (i0 + j < T) {
            const uint32_t x = sums[i0 + j];
            sums[i0 + j] = acc;
            acc += x;
        }
    }
    if (threadIdx.x == 0) sums[T] = tot;
}

// Step 3: every tile from its offset; the last tile writes the total.
__global__ __launch_bounds__(SCAN_NT) void k_scan_apply(const uint32_t *__restrict__ in,
                                                        uint32_t *__restrict__ out, int64_t N,
                                                        const uint32_t *__restrict__ offs,
                                                        uint32_t *total_out)
{
    __shared__ uint32_t s_lds[SCAN_NT / 64 + 1];
    const uint32_t tile = blockIdx.x;
    const int64_t base = (int64_t)tile * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IT;
    uint32_t v[SCAN_IT];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_IT; ++k) v[k] = (base + k < N) ? in[base + k] : 0u;
#pragma unroll
    for (int k = 0; k < SCAN_IT; ++k) sum += v[k];
    uint32_t tot;
    uint32_t run = offs[tile] + block_excl_sum<SCAN_NT>(sum, s_lds, &tot);
#pragma unroll
    for (int k = 0; k < SCAN_IT; ++k) {
        if (base + k < N) out[base + k] = run;
        run += v[k];
    }
    if (tile == gridDim.x - 1 && threadIdx.x == 0) {
        const uint32_t total = offs[gridDim.x];
        out[N] = total;
        if (total_out) *total_out = total;
    }
}

msf_status scan_u32(Ctx *c, const uint32_t *in, uint32_t *out, int64_t N, uint32_t *total_out)
{
    const int64_t ntiles = (N + SCAN_TILE - 1) / SCAN_TILE;
    if (ntiles == 0) {
        launch_fill_u32(c->stream, out, 0u, 1);
        if (total_out) launch_fill_u32(c->stream, total_out, 0u, 1);
        return MSF_OK;
    }
    if (ntiles <= SCAN3_TILES) {
        void *vs;
        msf_status rc = ws_get(c, WS_SCAN, 4 * ((size_t)ntiles + 1), &vs);
        if (rc) return rc;
        uint32_t *sums = (uint32_t *)vs;
        k_scan_tile_sums<<<(unsigned)ntiles, SCAN_NT, 0, c->stream>>>(in, N, sums);
        k_scan_sums<<<1, SCAN_SUMS_NT, 0, c->stream>>>(sums, (uint32_t)ntiles);
        k_scan_apply<<<(unsigned)ntiles, SCAN_NT, 0, c->stream>>>(in, out, N, sums, total_out);
        return MSF_OK;
    }
    void *st;
    msf_status rc = ws_get(c, WS_STATUS, sizeof(uint64_t) * (size_t)ntiles, &st);
    if (rc) return rc;
    launch_zero_lookback(c->stream, (uint64_t *)st, (uint32_t)ntiles, &c->dcnt->ticket, 1,
                         nullptr, 0);
    k_scan_u32<<<(unsigned)ntiles, SCAN_NT, 0, c->stream>>>(in, out, N, (uint64_t *)st, c->dcnt,
                                                          total_out);
    return MSF_OK;
}

// ------------------------------------------------------------- scatter ---

template <int WT>
__global__ void k_scatter(const int32_t *__restrict__ edges, const void *__restrict__ w, int64_t m,
                          const uint2 *__restrict__ slot, const uint32_t *__restrict__ row_ptr,
                          uint32_t *__restrict__ col, uint64_t *__restrict__ key)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; e < m; e += stride) {
        const uint2 s = slot[e];
        if (s.x == NONE32) continue;
        const int32_t u = edges[2 * e], v = edges[2 * e + 1];
        uint32_t wk = ((const uint32_t *)w)[e];
        if (WT == MSF_W_F32) wk = wkey_f32_bits(wk);
        const uint64_t k = ((uint64_t)wk << 32) | (uint64_t)(uint32_t)e;
        const uint32_t pu = row_ptr[u] + s.x;
        const uint32_t pv = row_ptr[v] + s.y;
        col[pu] = (uint32_t)v;
        key[pu] = k;
        col[pv] = (uint32_t)u;
        key[pv] = k;
    }
}

// --------------------------------------------------------- chunk rows ---
// For chunk k of slice s: the row holding entry sstart[s] + min(k*CHUNK,
// len_s - 1), i.e. the largest r with rp_s[r] <= that position.

uint32_t sweep_nchunks(uint32_t nnz) { return (nnz + SWEEP_CHUNK - 1) / SWEEP_CHUNK; }

int choose_slices(int32_t n, int64_t m, int forced)
{
    if (forced >= 1) return forced > MAX_SLICES ? MAX_SLICES : forced;
    // Slices keep each XCD's p[col] gathers inside its own L2, which pays
    // when every entry is gathered.  The plain sweep gathers lazily (about
    // one entry per lane), and then one slice is faster: no per-slice row
    // pointers and longer row segments.  Slices stay available on request.
    (void)n;
    (void)m;
    return 1;
}

void set_chunks(Adj *a)
{
    SliceInfo &sl = a->sl;
    uint32_t tot = 0, mx = 0;
    for (int q = 0; q < sl.S; ++q) {
        sl.cbase[q] = tot;
        // chunks of a slice start at its first entry rounded down to 4
        const uint32_t len = sl.sstart[q + 1] - sl.sstart[q];
        const uint32_t ch = len ? sweep_nchunks(sl.sstart[q + 1] - (sl.sstart[q] & ~3u)) : 0u;
        tot += ch;
        mx = ch > mx ? ch : mx;
    }
    sl.cbase[sl.S] = tot;
    sl.maxch = mx;
    a->nchunks = tot;
    a->nnz = sl.sstart[sl.S] - sl.sstart[0];
}

__global__ void k_chunk_rows(const uint32_t *__restrict__ row_ptr, int32_t n, SliceInfo sl,
                             uint32_t *__restrict__ chunk_row)
{
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= sl.cbase[sl.S] + (uint32_t)sl.S) return;
    int q = 0;
    while (q + 1 < sl.S && j >= sl.cbase[q + 1] + (uint32_t)(q + 1)) ++q;
    const uint32_t k = j - (sl.cbase[q] + (uint32_t)q);
    const uint32_t len = sl.sstart[q + 1] - sl.sstart[q];
    if (len == 0) {
        chunk_row[j] = 0;
        return;
    }
    uint64_t pos = (uint64_t)(sl.sstart[q] & ~3u) + (uint64_t)k * SWEEP_CHUNK;
    if (pos < sl.sstart[q]) pos = sl.sstart[q];
    if (pos > sl.sstart[q + 1] - 1) pos = sl.sstart[q + 1] - 1;
    const uint32_t *rp = row_ptr + (size_t)q * ((size_t)n + 1);
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo + 1) / 2;
        if (rp[mid] <= pos) lo = mid;
        else hi = mid - 1;
    }
    chunk_row[j] = (uint32_t)lo;
}

void launch_chunk_rows_sliced(hipStream_t s, const Adj &a)
{
    const uint32_t items = a.sl.cbase[a.sl.S] + (uint32_t)a.sl.S;
    k_chunk_rows<<<(items + 255) / 256, 256, 0, s>>>(a.row_ptr, a.n, a.sl, a.chunk_row);
}

// Slice boundaries and the number of non-empty (row, slice) segments.
// Each thread counts SI_ROWS consecutive rows of a slice (their pointers
// loaded together); one atomic per workgroup, on a grid of at most
// SI_BLOCKS workgroups (same-address atomics from thousands of workgroups
// serialise: 30 us on 4.2M rows with 2048 workgroups of one row per thread).
constexpr int SI_ROWS = 16;
constexpr size_t SI_BLOCKS = 256;

__global__ __launch_bounds__(256) void k_slice_info(const uint32_t *__restrict__ row_ptr,
                                                    int32_t n, int S, Counters *cnt)
{
    __shared__ uint32_t s_lds[256 / 64 + 1];
    const size_t stride = (size_t)n + 1;
    if (blockIdx.x == 0 && threadIdx.x <= (unsigned)S)
        cnt->sstart[threadIdx.x] = threadIdx.x < (unsigned)S
                                       ? row_ptr[(size_t)threadIdx.x * stride]
                                       : row_ptr[(size_t)(S - 1) * stride + n];
    uint32_t segs = 0;
    const size_t groups = ((size_t)n + SI_ROWS - 1) / SI_ROWS;  // per slice
    const size_t total = (size_t)S * groups;
    for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < total;
         j += (size_t)gridDim.x * blockDim.x) {
        const size_t q = j / groups, i0 = (j - q * groups) * SI_ROWS;
        const uint32_t *rp = row_ptr + q * stride;
        uint32_t v[SI_ROWS + 1];
#pragma unroll
        for (int k = 0; k <= SI_ROWS; ++k) {
            const size_t i = i0 + (size_t)k;
            v[k] = rp[i < (size_t)n ? i : (size_t)n];  // clamped: past the end adds nothing
        }
#pragma unroll
        for (int k = 0; k < SI_ROWS; ++k) segs += v[k + 1] > v[k] ? 1u : 0u;
    }
    segs = block_sum<256>(segs, s_lds);
    if (threadIdx.x == 0 && segs) atomicAdd(&cnt->segs, segs);
}

void launch_slice_info(hipStream_t s, const Adj &a, Counters *dcnt)
{
    launch_fill_u32(s, &dcnt->segs, 0u, 1);
    const size_t groups = (size_t)a.sl.S * (((size_t)a.n + SI_ROWS - 1) / SI_ROWS);
    size_t g = (groups + 255) / 256;
    if (g < 1) g = 1;
    if (g > SI_BLOCKS) g = SI_BLOCKS;
    k_slice_info<<<(unsigned)g, 256, 0, s>>>(a.row_ptr, a.n, a.sl.S, dcnt);
}

// Stored entries in rows of at least min_len entries (one-slice row_ptr),
// added into cnt->long_entries.
__global__ __launch_bounds__(256) void k_long_entries(const uint32_t *__restrict__ row_ptr,
                                                      int32_t n, uint32_t min_len, Counters *cnt)
{
    unsigned long long sum = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t len = row_ptr[i + 1] - row_ptr[i];
        if (len >= min_len) sum += len;
    }
    for (int d = 32; d >= 1; d >>= 1) sum += __shfl_xor(sum, d, 64);
    if (__lane_id() == 0 && sum)
        atomicAdd(reinterpret_cast<unsigned long long *>(&cnt->long_entries), sum);
}

void launch_long_entries(hipStream_t s, const uint32_t *row_ptr, int32_t n, Counters *dcnt)
{
    launch_fill_u32(s, reinterpret_cast<uint32_t *>(&dcnt->long_entries), 0u, 2);
    if (n <= 0) return;
    const unsigned g = (unsigned)std::min<int64_t>(std::max<int64_t>(((int64_t)n + 255) / 256, 1), 2048);
    k_long_entries<<<g, 256, 0, s>>>(row_ptr, n, WAVE_ROW, dcnt);
}

// ------------------------------------------------- bucketed build ------
// The same adjacency built without any global atomic: rows are grouped in
// buckets of 2^LB consecutive ids (at most BK_MAX_NB buckets).
//   A. per block of edges, an LDS histogram of the endpoint buckets,
//      written bucket-major so one exclusive scan gives every
//      (bucket, block) its output offset and every bucket its start;
//   B. the same blocks scatter both directions of each edge into their
//      buckets (row offset in the bucket, column, key), ranked by LDS
//      atomics;
//   C. per bucket, a workgroup counts its rows in LDS, scans them into
//      row_ptr, and scatters the entries to their final positions; in the
//      solve, one workgroup takes all slices of a row block and also keeps
//      the row minima that round 1 needs.
// Every atomic is an LDS atomic, so a vertex of very high degree costs LDS
// conflicts inside one workgroup instead of serialised device atomics.

constexpr int BK_MAX_NB = 16384;  // pass A/B keep one LDS counter per bucket
constexpr int BKA_NT = 256;
// most counter copies of the coarse histogram (a power of two)
#ifndef BKA_COPIES
#define BKA_COPIES 8
#endif
constexpr int BKC_NT = 1024;
constexpr int BK_MIN_LB = 12;  // fewer, larger buckets keep pass B's writes in long runs
constexpr int BK_MAX_LB = 15;  // pass C keeps 2^LB row counters in LDS

static int bucket_bits(int32_t n, int S)
{
    int lb = BK_MIN_LB;
    while ((int64_t)S * ((((int64_t)n + (1ll << lb) - 1) >> lb)) > BK_MAX_NB) ++lb;
    return lb;
}

// bucket of stored direction row -> col: (slice of col, row >> lb)
__device__ __forceinline__ uint32_t bucket_of(uint32_t row, uint32_t col, int lb, uint32_t slice_w,
                                              uint32_t nbr)
{
    return (col / slice_w) * nbr + (row >> lb);
}

template <int WT>
__global__ __launch_bounds__(BKA_NT) void k_bucket_hist(const int32_t *__restrict__ edges,
                                                        const void *__restrict__ w, int64_t m,
                                                        int32_t n, int lb, int nb, uint32_t slice_w,
                                                        uint32_t nbr, int64_t epb, uint32_t nblk,
                                                        int C, uint32_t *__restrict__ bh,
                                                        Counters *cnt, int check_w)
{
    // C copies of every counter, [bucket][copy]: lane l counts in copy
    // l % C, so lanes of a wave with the same bucket rarely hit the same
    // LDS word; the copies are summed at the end
    extern __shared__ uint32_t hist[];
    const uint32_t cp = threadIdx.x & (uint32_t)(C - 1);
    for (int i = threadIdx.x; i < nb * C; i += BKA_NT) hist[i] = 0;
    __syncthreads();
    const int64_t e0 = (int64_t)blockIdx.x * epb;
    const int64_t e1 = e0 + epb < m ? e0 + epb : m;
    uint32_t err = 0;
    // BKA_B edges per thread per batch, all loaded before any is counted
    constexpr int BKA_B = 8;
    for (int64_t eb = e0; eb < e1; eb += (int64_t)BKA_NT * BKA_B) {
        int32_t uu[BKA_B], vv[BKA_B];
        uint32_t ww[BKA_B];
#pragma unroll
        for (int k = 0; k < BKA_B; ++k) {
            const int64_t e = eb + threadIdx.x + (int64_t)k * BKA_NT;
            const bool in = e < e1;
            uu[k] = in ? edges[2 * e] : 0;
            vv[k] = in ? edges[2 * e + 1] : 0;
            ww[k] = (in && WT == MSF_W_F32 && check_w) ? ((const uint32_t *)w)[e] : 0u;
        }
#pragma unroll
        for (int k = 0; k < BKA_B; ++k) {
            const int64_t e = eb + threadIdx.x + (int64_t)k * BKA_NT;
            if (e >= e1) continue;
            const int32_t u = uu[k], v = vv[k];
            if (WT == MSF_W_F32) {
                const uint32_t b = ww[k];
                if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu)) err |= ERR_NAN;
            }
            if ((uint32_t)u >= (uint32_t)n || (uint32_t)v >= (uint32_t)n) {
                err |= ERR_ENDPOINT;
                continue;
            }
            if (u == v) continue;
            atomicAdd(&hist[bucket_of((uint32_t)u, (uint32_t)v, lb, slice_w, nbr) * C + cp], 1u);
            atomicAdd(&hist[bucket_of((uint32_t)v, (uint32_t)u, lb, slice_w, nbr) * C + cp], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += BKA_NT) {
        uint32_t t = 0;
        for (int q = 0; q < C; ++q) t += hist[i * C + q];
        bh[(size_t)i * nblk + blockIdx.x] = t;
    }
    if (__ballot(err != 0)) {
        uint32_t any = err;
        for (int d = 32; d >= 1; d >>= 1) any |= __shfl_xor(any, d, 64);
        if (__lane_id() == 0) atomicOr(&cnt->err, any);
    }
}

template <int WT>
__global__ __launch_bounds__(BKA_NT) void k_bucket_scatter(
    const int32_t *__restrict__ edges, const void *__restrict__ w, int64_t m, int32_t n, int lb,
    int nb, uint32_t slice_w, uint32_t nbr, int64_t epb, uint32_t nblk,
    const uint32_t *__restrict__ bh_off,
    uint16_t *__restrict__ rlo, uint32_t *__restrict__ bcol, uint64_t *__restrict__ bkey)
{
    extern __shared__ uint32_t off[];
    for (int i = threadIdx.x; i < nb; i += BKA_NT) off[i] = bh_off[(size_t)i * nblk + blockIdx.x];
    __syncthreads();
    const uint32_t mask = (1u << lb) - 1u;
    const int64_t e0 = (int64_t)blockIdx.x * epb;
    const int64_t e1 = e0 + epb < m ? e0 + epb : m;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += BKA_NT) {
        const int32_t u = edges[2 * e], v = edges[2 * e + 1];
        if ((uint32_t)u >= (uint32_t)n || (uint32_t)v >= (uint32_t)n || u == v) continue;
        uint32_t wk = ((const uint32_t *)w)[e];
        if (WT == MSF_W_F32) wk = wkey_f32_bits(wk);
        const uint64_t k = ((uint64_t)wk << 32) | (uint64_t)(uint32_t)e;
        const uint32_t pu = atomicAdd(&off[bucket_of((uint32_t)u, (uint32_t)v, lb, slice_w, nbr)], 1u);
        const uint32_t pv = atomicAdd(&off[bucket_of((uint32_t)v, (uint32_t)u, lb, slice_w, nbr)], 1u);
        rlo[pu] = (uint16_t)((uint32_t)u & mask);
        bcol[pu] = (uint32_t)v;
        bkey[pu] = k;
        rlo[pv] = (uint16_t)((uint32_t)v & mask);
        bcol[pv] = (uint32_t)u;
        bkey[pv] = k;
    }
}

// Pass C.  Workgroup b serves row block rb = b % nbr and the slices
// q = b / nbr, b / nbr + G, ... (G = grid / nbr): per slice, count the
// rows in LDS, scan them into that slice's row_ptr, and place the entries.
// MIN (grid = nbr, so one workgroup sees every slice of its rows) also
// keeps each row's smallest key in LDS and stores it to r[row]: round 1 of
// the multilinear sweep, where the parent vector is the identity and every
// stored entry is outgoing, so its minima are a by-product of the build.
template <bool MIN>
__global__ __launch_bounds__(BKC_NT) void k_bucket_rows(
    const uint32_t *__restrict__ bh_off, uint32_t nblk, int32_t n, int lb, int S, uint32_t nbr,
    const uint16_t *__restrict__ rlo, const uint32_t *__restrict__ bcol,
    const uint64_t *__restrict__ bkey, uint32_t *__restrict__ row_ptr, uint32_t *__restrict__ col,
    uint64_t *__restrict__ key, uint64_t *__restrict__ r)
{
    extern __shared__ uint64_t lds64[];
    const uint32_t R = 1u << lb;
    uint64_t *smin = lds64;                                      // R keys (MIN only)
    uint32_t *cnt = reinterpret_cast<uint32_t *>(lds64 + (MIN ? R : 0));  // R counters
    uint32_t *scr = cnt + R;                                     // scan scratch
    const uint32_t rb = blockIdx.x % nbr;
    const uint32_t qstep = gridDim.x / nbr;
    const int64_t row0 = (int64_t)rb << lb;
    const uint32_t rows = (uint32_t)((int64_t)n - row0 < (int64_t)R ? (int64_t)n - row0 : R);
    if (MIN)
        for (uint32_t i = threadIdx.x; i < R; i += BKC_NT) smin[i] = KEY_INF;
    for (uint32_t q = blockIdx.x / nbr; q < (uint32_t)S; q += qstep) {
        const uint32_t b = q * nbr + rb;
        const uint32_t s = bh_off[(size_t)b * nblk];
        const uint32_t e = bh_off[(size_t)(b + 1) * nblk];
        uint32_t *rp = row_ptr + (size_t)q * ((size_t)n + 1);
        for (uint32_t i = threadIdx.x; i < R; i += BKC_NT) cnt[i] = 0;
        __syncthreads();
        for (uint32_t k = s + threadIdx.x; k < e; k += BKC_NT) atomicAdd(&cnt[rlo[k]], 1u);
        __syncthreads();
        // exclusive scan of the R counters: PER consecutive counters per thread
        const uint32_t per = R / BKC_NT > 0 ? R / BKC_NT : 1;
        const uint32_t i0 = threadIdx.x * per;
        uint32_t run = 0;
        if (i0 < R)
            for (uint32_t j = 0; j < per; ++j) run += cnt[i0 + j];
        uint32_t tot;
        const uint32_t ex = block_excl_sum<BKC_NT>(run, scr, &tot);
        if (i0 < R) {
            uint32_t acc = ex;
            for (uint32_t j = 0; j < per; ++j) {
                const uint32_t c = cnt[i0 + j];
                cnt[i0 + j] = acc;
                acc += c;
            }
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < rows; i += BKC_NT) rp[row0 + i] = s + cnt[i];
        if (rb == nbr - 1 && threadIdx.x == 0) rp[n] = e;
        __syncthreads();
        for (uint32_t k = s + threadIdx.x; k < e; k += BKC_NT) {
            const uint32_t rl = rlo[k];
            const uint64_t kk = bkey[k];
            const uint32_t pos = s + atomicAdd(&cnt[rl], 1u);
            col[pos] = bcol[k];
            key[pos] = kk;
            if (MIN) atomicMin((unsigned long long *)&smin[rl], (unsigned long long)kk);
        }
        __syncthreads();  // cnt is cleared for the next slice
    }
    if (MIN)
        for (uint32_t i = threadIdx.x; i < rows; i += BKC_NT) r[row0 + i] = smin[i];
}

// ---------------------------------------------------------------- host ---

static msf_status build_atomic(Ctx *c, int32_t n, int64_t m, const int32_t *d_edges,
                               const void *d_w, msf_wtype wt, uint32_t *row_ptr, uint32_t *col,
                               uint64_t *key)
{
    hipStream_t s = c->stream;
    void *vdeg, *vslot;
    MSF_TRY(ws_get(c, WS_DEG, 4 * (size_t)(n > 0 ? n : 1), &vdeg));
    MSF_TRY(ws_get(c, WS_SLOT, sizeof(uint2) * (size_t)(m > 0 ? m : 1), &vslot));
    uint32_t *deg = (uint32_t *)vdeg;
    uint2 *slot = (uint2 *)vslot;
    launch_fill_u32(s, deg, 0u, (size_t)n);
    const unsigned ge = grid_for((size_t)m, 256, 16384);
    if (m > 0) {
        if (wt == MSF_W_F32)
            k_degree<MSF_W_F32><<<ge, 256, 0, s>>>(d_edges, d_w, m, n, deg, slot, c->dcnt);
        else
            k_degree<MSF_W_U32><<<ge, 256, 0, s>>>(d_edges, d_w, m, n, deg, slot, c->dcnt);
    }
    MSF_TRY(scan_u32(c, deg, row_ptr, n, &c->dcnt->count));
    if (m > 0) {
        if (wt == MSF_W_F32)
            k_scatter<MSF_W_F32><<<ge, 256, 0, s>>>(d_edges, d_w, m, slot, row_ptr, col, key);
        else
            k_scatter<MSF_W_U32><<<ge, 256, 0, s>>>(d_edges, d_w, m, slot, row_ptr, col, key);
    }
    MSF_HIP(hipGetLastError());
    return MSF_OK;
}

msf_status launch_bucket_hist(Ctx *c, const int32_t *d_edges, const void *d_w, int64_t m,
                              int32_t n, int lb, int nb, uint32_t slice_w, uint32_t nbr,
                              int64_t epb, uint32_t nblk, msf_wtype wt, uint32_t *bh,
                              bool check_w)
{
    // counter copies while the histogram stays within 32 KB of LDS
    int C = 1;
    while (C < BKA_COPIES && (size_t)nb * 2 * C * 4 <= ((size_t)32 << 10)) C *= 2;
    const size_t lds_a = 4 * (size_t)nb * C;
    if (wt == MSF_W_F32)
        k_bucket_hist<MSF_W_F32><<<nblk, BKA_NT, lds_a, c->stream>>>(
            d_edges, d_w, m, n, lb, nb, slice_w, nbr, epb, nblk, C, bh, c->dcnt, check_w);
    else
        k_bucket_hist<MSF_W_U32><<<nblk, BKA_NT, lds_a, c->stream>>>(
            d_edges, d_w, m, n, lb, nb, slice_w, nbr, epb, nblk, C, bh, c->dcnt, 0);
    MSF_HIP(hipGetLastError());
    return MSF_OK;
}

static size_t rows_lds(int lb, bool with_min)
{
    const size_t R = (size_t)1 << lb;
    return (with_min ? 8 * R : 0) + 4 * R + 4 * (BKC_NT / 64 + 1);
}

template <bool MIN>
static bool rows_lds_ok(int lb);

static msf_status build_bucketed(Ctx *c, int32_t n, int64_t m, const int32_t *d_edges,
                                 const void *d_w, msf_wtype wt, int lb, int S, uint32_t slice_w,
                                 uint32_t *row_ptr, uint32_t *col, uint64_t *key, uint64_t *r_first)
{
    hipStream_t s = c->stream;
    const uint32_t nbr = (uint32_t)(((int64_t)n + (1ll << lb) - 1) >> lb);
    const int nb = (int)nbr * S;
    int64_t epb = (m + 2047) / 2048;
    if (epb < 32768) epb = 32768;
    epb = (epb + 255) & ~(int64_t)255;
    const uint32_t nblk = (uint32_t)((m + epb - 1) / epb);
    const size_t nh = (size_t)nb * nblk;
    const size_t mm = (size_t)m;
    void *vbh, *vbo, *vrlo, *vcol, *vkey;
    MSF_TRY(ws_get(c, WS_BH, 4 * nh, &vbh));
    MSF_TRY(ws_get(c, WS_BHOFF, 4 * (nh + 1), &vbo));
    MSF_TRY(ws_get(c, WS_BRLO, 2 * 2 * mm, &vrlo));
    MSF_TRY(ws_get(c, WS_BCOL, 4 * 2 * mm, &vcol));
    MSF_TRY(ws_get(c, WS_BKEY, 8 * 2 * mm, &vkey));
    uint32_t *bh = (uint32_t *)vbh, *bo = (uint32_t *)vbo;
    const size_t lds_a = 4 * (size_t)nb;
    MSF_TRY(launch_bucket_hist(c, d_edges, d_w, m, n, lb, nb, slice_w, nbr, epb, nblk, wt, bh));
    MSF_TRY(scan_u32(c, bh, bo, (int64_t)nh, &c->dcnt->count));
    if (wt == MSF_W_F32)
        k_bucket_scatter<MSF_W_F32><<<nblk, BKA_NT, lds_a, s>>>(
            d_edges, d_w, m, n, lb, nb, slice_w, nbr, epb, nblk, bo, (uint16_t *)vrlo,
            (uint32_t *)vcol, (uint64_t *)vkey);
    else
        k_bucket_scatter<MSF_W_U32><<<nblk, BKA_NT, lds_a, s>>>(
            d_edges, d_w, m, n, lb, nb, slice_w, nbr, epb, nblk, bo, (uint16_t *)vrlo,
            (uint32_t *)vcol, (uint64_t *)vkey);
    if (r_first)
        k_bucket_rows<true><<<nbr, BKC_NT, rows_lds(lb, true), s>>>(
            bo, nblk, n, lb, S, nbr, (const uint16_t *)vrlo, (const uint32_t *)vcol,
            (const uint64_t *)vkey, row_ptr, col, key, r_first);
    else
        k_bucket_rows<false><<<nb, BKC_NT, rows_lds(lb, false), s>>>(
            bo, nblk, n, lb, S, nbr, (const uint16_t *)vrlo, (const uint32_t *)vcol,
            (const uint64_t *)vkey, row_ptr, col, key, nullptr);
    MSF_HIP(hipGetLastError());
    return MSF_OK;
}

// Pass C keeps 2^lb row counters (and with MIN 2^lb row minima) in LDS;
// above 64 KB the kernel must be allowed a larger dynamic LDS allocation,
// which is requested once per variant (at most the 160 KB of a CU).
template <bool MIN>
static bool rows_lds_ok(int lb)
{
    const size_t need = rows_lds(lb, MIN);
    if (need <= 65536) return true;
    static int granted = -1;  // -1 unknown, else the granted byte count
    if (granted < 0) {
        const size_t cap = 160 * 1024;
        const size_t top = rows_lds(BK_MAX_LB, MIN);
        const int want = (int)(top < cap ? top : cap);
        granted = hipFuncSetAttribute((const void *)k_bucket_rows<MIN>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, want) ==
                          hipSuccess
                      ? want
                      : 65536;
        (void)hipGetLastError();
    }
    return need <= (size_t)granted;
}

msf_status build_adjacency(Ctx *c, int32_t n, int64_t m, const int32_t *d_edges, const void *d_w,
                           msf_wtype wt, int S, Adj *a, uint32_t *row_ptr, uint32_t *col,
                           uint64_t *key, uint32_t *chunk_row, uint64_t *r_first,
                           bool *first_done)
{
    if (first_done) *first_done = false;
    launch_fill_u32(c->stream, &c->dcnt->err, 0u, 1);
    if (S < 1 || n < 32 * S) S = 1;
    int lb = bucket_bits(n, S);
    const bool bucketed = c->bucketed_build && m > 0 && n > 0 && lb <= BK_MAX_LB &&
                          rows_lds_ok<false>(lb);
    if (!bucketed) S = 1;  // the atomic fallback stores one slice
    TwoLevel tl;
    uint32_t slice_w = (uint32_t)n;
    if (S > 1) slice_w = (uint32_t)((((int64_t)n + S - 1) / S + 31) & ~(int64_t)31);
    if (m == 0 || n == 0) {
        launch_fill_u32(c->stream, row_ptr, 0u, (size_t)n + 1);
        launch_fill_u32(c->stream, &c->dcnt->count, 0u, 1);
    } else if (bucketed && S == 1 && c->bucketed_build == 1 && two_level_params(n, m, &tl)) {
        MSF_TRY(build_two_level(c, n, m, d_edges, d_w, wt, tl, row_ptr, col, key, r_first));
        if (first_done) *first_done = r_first != nullptr;
    } else if (bucketed) {
        const bool fuse = r_first && rows_lds_ok<true>(lb);
        MSF_TRY(build_bucketed(c, n, m, d_edges, d_w, wt, lb, S, slice_w, row_ptr, col, key,
                               fuse ? r_first : nullptr));
        if (first_done) *first_done = fuse;
    } else {
        MSF_TRY(build_atomic(c, n, m, d_edges, d_w, wt, row_ptr, col, key));
    }
    a->n = n;
    a->m = m;
    a->sl = SliceInfo{};
    a->sl.S = S;
    a->sl.slice_w = slice_w;
    a->row_ptr = row_ptr;
    a->col = col;
    a->key = key;
    a->chunk_row = chunk_row;
    a->edges = d_edges;
    a->w = d_w;
    a->wtype = wt;
    launch_slice_info(c->stream, *a, c->dcnt);
    MSF_HIP(hipGetLastError());
    return MSF_OK;
}

}  // namespace msf
