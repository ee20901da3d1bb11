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
constexpr int SCAN_NT = 256;
constexpr int SCAN_IT = 8;
constexpr int SCAN_TILE = SCAN_NT * SCAN_IT;

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

msf_status scan_u32(Ctx *c, const uint32_t *in, uint32_t *out, int64_t N, uint32_t *total_out)
{
    const int64_t ntiles = (N + SCAN_TILE - 1) / SCAN_TILE;
    if (ntiles == 0) {
        launch_fill_u32(c->stream, out, 0u, 1);
        if (total_out) launch_fill_u32(c->stream, total_out, 0u, 1);
        return MSF_OK;
    }
    void *st;
    msf_status rc = ws_get(c, WS_STATUS, sizeof(uint64_t) * (size_t)ntiles, &st);
    if (rc) return rc;
    launch_fill_u64(c->stream, (uint64_t *)st, 0ull, (size_t)ntiles);
    launch_fill_u32(c->stream, &c->dcnt->ticket, 0u, 1);
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
// chunk_row[c] = the row holding entry min(c*CHUNK, nnz-1): the largest r
// with row_ptr[r] <= that entry.

uint32_t sweep_nchunks(uint32_t nnz) { return (nnz + SWEEP_CHUNK - 1) / SWEEP_CHUNK; }

__global__ void k_chunk_rows(const uint32_t *__restrict__ row_ptr, int32_t n, uint32_t nnz,
                             uint32_t *__restrict__ chunk_row, uint32_t nchunks)
{
    uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nchunks) return;
    if (nnz == 0) {
        chunk_row[c] = 0;
        return;
    }
    uint64_t pos = (uint64_t)c * SWEEP_CHUNK;
    if (pos > nnz - 1) pos = nnz - 1;
    // largest r in [0, n-1] with row_ptr[r] <= pos
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        int32_t mid = lo + (hi - lo + 1) / 2;
        if (row_ptr[mid] <= pos) lo = mid;
        else hi = mid - 1;
    }
    chunk_row[c] = (uint32_t)lo;
}

void launch_chunk_rows(hipStream_t s, const uint32_t *row_ptr, int32_t n, uint32_t nnz,
                       uint32_t *chunk_row, uint32_t nchunks)
{
    unsigned g = (nchunks + 1 + 255) / 256;
    k_chunk_rows<<<g, 256, 0, s>>>(row_ptr, n, nnz, chunk_row, nchunks);
}

// ---------------------------------------------------------------- host ---

msf_status build_adjacency(Ctx *c, int32_t n, int64_t m, const int32_t *d_edges, const void *d_w,
                           msf_wtype wt, Adj *a, uint32_t *row_ptr, uint32_t *col, uint64_t *key,
                           uint32_t *deg, uint2 *slot, uint32_t *chunk_row)
{
    hipStream_t s = c->stream;
    launch_fill_u32(s, deg, 0u, (size_t)n);
    launch_fill_u32(s, &c->dcnt->err, 0u, 1);
    const unsigned ge = grid_for((size_t)m, 256, 16384);
    if (m > 0) {
        if (wt == MSF_W_F32)
            k_degree<MSF_W_F32><<<ge, 256, 0, s>>>(d_edges, d_w, m, n, deg, slot, c->dcnt);
        else
            k_degree<MSF_W_U32><<<ge, 256, 0, s>>>(d_edges, d_w, m, n, deg, slot, c->dcnt);
    }
    msf_status rc = scan_u32(c, deg, row_ptr, n, &c->dcnt->count);
    if (rc) return rc;
    if (m > 0) {
        if (wt == MSF_W_F32)
            k_scatter<MSF_W_F32><<<ge, 256, 0, s>>>(d_edges, d_w, m, slot, row_ptr, col, key);
        else
            k_scatter<MSF_W_U32><<<ge, 256, 0, s>>>(d_edges, d_w, m, slot, row_ptr, col, key);
    }
    MSF_HIP(hipGetLastError());
    a->n = n;
    a->m = m;
    a->row_ptr = row_ptr;
    a->col = col;
    a->key = key;
    a->chunk_row = chunk_row;
    a->edges = d_edges;
    a->w = d_w;
    a->wtype = wt;
    return MSF_OK;
}

}  // namespace msf
