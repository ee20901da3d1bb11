// Vertex order of a kept graph (msf_graph_create): vertices renumbered by
// decreasing degree class, so the parent entries the multilinear kernel
// gathers most (those of high-degree columns) share a few cache lines.
//
// The adjacency matrix A of section 2 is stored as P A P^T for this
// permutation P: the same matrix with rows and columns renumbered, so every
// call on the graph computes the same values.  Edge ids are unchanged;
// the calls that take or return per-vertex vectors translate them.
//
// The order: class(v) = bit length of deg(v) (stored directions, loops
// excluded), classes in decreasing order, and vertex ids increasing inside a
// class (a stable counting sort, so the order is deterministic).  In R-MAT
// graphs a few percent of the vertices hold most edge ends; with this order
// their parents fit in each XCD's L2.
//
// The graph is first built in the caller's order (the degrees are its row
// lengths, with no atomics); its rows are then copied to their new places,
// a wave per segment of at most RL_SEG entries, columns renumbered.  Built
// directly in the new order, the hub rows would crowd a few placement
// buckets and serialise the build.
#include <algorithm>

#include "msf_internal.hpp"
#include "wave.hpp"

namespace msf {

namespace {

constexpr int RL_CLASSES = 33;   // bit lengths 0..32
constexpr int RL_TILE = 4096;    // vertices per counting tile (one wave)

__device__ __forceinline__ uint32_t rl_slot(uint32_t deg)
{
    // slot 0 holds the largest degrees
    return (uint32_t)(RL_CLASSES - 1) - (deg ? 32u - (uint32_t)__builtin_clz(deg) : 0u);
}

// Per tile (one wave): vertices of each class, into tab[slot * ntiles + tile].
__global__ __launch_bounds__(64) void k_rl_count(const uint32_t *__restrict__ deg, int32_t n,
                                                 uint32_t ntiles, uint32_t *__restrict__ tab)
{
    __shared__ uint32_t s_c[RL_CLASSES];
    const uint32_t tile = blockIdx.x;
    if (threadIdx.x < RL_CLASSES) s_c[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t lo = tile * RL_TILE;
    const uint32_t hi = min((uint32_t)n, lo + RL_TILE);
    for (uint32_t v = lo + threadIdx.x; v < hi; v += 64) atomicAdd(&s_c[rl_slot(deg[v])], 1u);
    __syncthreads();
    if (threadIdx.x < RL_CLASSES) tab[(size_t)threadIdx.x * ntiles + tile] = s_c[threadIdx.x];
}

// Stable placement: the wave walks its tile in id order, 64 vertices at a
// time; lanes of one class take consecutive positions in lane order.
// off[slot * ntiles + tile] is the exclusive scan of tab (slot-major).
__global__ __launch_bounds__(64) void k_rl_place(const uint32_t *__restrict__ deg, int32_t n,
                                                 uint32_t ntiles, const uint32_t *__restrict__ off,
                                                 uint32_t *__restrict__ perm,
                                                 uint32_t *__restrict__ inv)
{
    __shared__ uint32_t s_next[RL_CLASSES];
    const uint32_t tile = blockIdx.x;
    if (threadIdx.x < RL_CLASSES) s_next[threadIdx.x] = off[(size_t)threadIdx.x * ntiles + tile];
    __syncthreads();
    const uint32_t lo = tile * RL_TILE;
    const uint32_t hi = min((uint32_t)n, lo + RL_TILE);
    for (uint32_t b = lo; b < hi; b += 64) {
        const uint32_t v = b + threadIdx.x;
        const bool in = v < hi;
        const uint32_t my = in ? rl_slot(deg[v]) : RL_CLASSES;
        uint64_t left = __ballot(in);
        while (left) {
            const uint32_t first = (uint32_t)__builtin_ctzll(left);
            const uint32_t cls = (uint32_t)__shfl((int)my, (int)first, 64);
            const uint64_t mask = __ballot(in && my == cls);
            if (in && my == cls) {
                const uint32_t pos = s_next[cls] + (uint32_t)__popcll(mask & lanemask_lt());
                perm[pos] = v;
                inv[v] = pos;
            }
            if (threadIdx.x == 0) s_next[cls] += (uint32_t)__popcll(mask);
            __syncthreads();
            left &= ~mask;
        }
    }
}

// out = inv applied to both ends of every edge (endpoints already checked;
// out may be edges: each thread reads its edge before writing it).
__global__ void k_rl_edges(const int32_t *edges, int64_t m, const uint32_t *__restrict__ inv,
                           int32_t *out)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
        const int2 uv = reinterpret_cast<const int2 *>(edges)[e];
        reinterpret_cast<int2 *>(out)[e] = make_int2((int32_t)inv[uv.x], (int32_t)inv[uv.y]);
    }
}

// q[i] = p[perm[i]]: a caller's parent vector in the graph's order (the
// values stay caller vertex ids).
__global__ void k_rl_gather(const uint32_t *__restrict__ p, const uint32_t *__restrict__ perm,
                            int32_t n, uint32_t *__restrict__ q)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        q[i] = p[perm[i]];
}

// labels[perm[i]] = perm[q[i]]: vertex labels of the graph's order back to
// caller ids.
__global__ void k_rl_labels(const uint32_t *__restrict__ q, const uint32_t *__restrict__ perm,
                            int32_t n, uint32_t *__restrict__ labels)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        labels[perm[i]] = perm[q[i]];
}

unsigned grid_of(int64_t n) { return (unsigned)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 16384); }

// deg[v] = stored entries of row v of a one-slice adjacency.
__global__ void k_rl_deg_rp(const uint32_t *__restrict__ rp, int32_t n, uint32_t *__restrict__ deg)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        deg[v] = rp[v + 1] - rp[v];
}

// Entries a wave copies per segment of a renumbered row.
constexpr uint32_t RL_SEG = 256;

// nd[k] = entries of new row k (old row perm[k]), sc[k] = its segments.
__global__ void k_rl_newdeg(const uint32_t *__restrict__ deg, const uint32_t *__restrict__ perm,
                            int32_t n, uint32_t *__restrict__ nd, uint32_t *__restrict__ sc)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const uint32_t d = deg[perm[k]];
        nd[k] = d;
        sc[k] = (d + RL_SEG - 1u) / RL_SEG;
    }
}

// seg_row[s] = the new row segment s belongs to.
__global__ void k_rl_segrows(const uint32_t *__restrict__ so, int32_t n,
                             uint32_t *__restrict__ seg_row)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
        for (uint32_t s = so[k]; s < so[k + 1]; ++s) seg_row[s] = (uint32_t)k;
}

// One wave per segment (grid-stride up to the segment count *ns): the
// segment's entries of old row perm[k] go to new row k in the same order,
// columns renumbered.
__global__ __launch_bounds__(256) void k_rl_permute(
    const uint32_t *__restrict__ rp0, const uint32_t *__restrict__ col0,
    const uint64_t *__restrict__ key0, const uint32_t *__restrict__ perm,
    const uint32_t *__restrict__ inv, const uint32_t *__restrict__ rp,
    const uint32_t *__restrict__ so, const uint32_t *__restrict__ seg_row,
    const uint32_t *__restrict__ ns, uint32_t *__restrict__ col, uint64_t *__restrict__ key)
{
    const uint32_t lane = __lane_id();
    const uint32_t total = *ns;
    const uint32_t nw = gridDim.x * (blockDim.x / 64u);
    for (uint32_t s = blockIdx.x * (blockDim.x / 64u) + (threadIdx.x >> 6); s < total; s += nw) {
        const uint32_t k = seg_row[s];
        const uint32_t j0 = (s - so[k]) * RL_SEG;
        const uint32_t ob = rp0[perm[k]], nb = rp[k], len = rp[k + 1] - nb;
        const uint32_t je = j0 + RL_SEG < len ? j0 + RL_SEG : len;
        for (uint32_t j = j0 + lane; j < je; j += 64u) {
            col[nb + j] = inv[col0[ob + j]];
            key[nb + j] = key0[ob + j];
        }
    }
}

}  // namespace

size_t relabel_segments_cap(int32_t n, int64_t nnz)
{
    return (size_t)(nnz > 0 ? nnz : 0) / RL_SEG + (size_t)(n > 0 ? n : 0) + 1;
}

// Stable counting sort of the vertices by degree class: perm, inv.
static msf_status order_by_degree(Ctx *c, int32_t n, const uint32_t *deg, uint32_t *tab,
                                  uint32_t *perm, uint32_t *inv)
{
    hipStream_t s = c->stream;
    const uint32_t ntiles = (uint32_t)(((int64_t)n + RL_TILE - 1) / RL_TILE);
    if (n <= 0) return MSF_OK;
    k_rl_count<<<ntiles, 64, 0, s>>>(deg, n, ntiles, tab);
    MSF_TRY(scan_u32(c, tab, tab + (size_t)RL_CLASSES * ntiles + 1, (int64_t)RL_CLASSES * ntiles,
                     nullptr));
    k_rl_place<<<ntiles, 64, 0, s>>>(deg, n, ntiles, tab + (size_t)RL_CLASSES * ntiles + 1, perm,
                                     inv);
    MSF_HIP(hipGetLastError());
    return MSF_OK;
}

msf_status relabel_csr_by_degree(Ctx *c, int32_t n, const uint32_t *rp0, const uint32_t *col0,
                                 const uint64_t *key0, uint32_t *deg, uint32_t *tab,
                                 uint32_t *perm, uint32_t *inv, uint32_t *seg,
                                 uint32_t *seg_row, uint32_t *rp, uint32_t *col, uint64_t *key)
{
    hipStream_t s = c->stream;
    if (n <= 0) return MSF_OK;
    k_rl_deg_rp<<<grid_of(n), 256, 0, s>>>(rp0, n, deg);
    MSF_TRY(order_by_degree(c, n, deg, tab, perm, inv));
    uint32_t *nd = deg + n, *sc = seg, *so = seg + n;
    k_rl_newdeg<<<grid_of(n), 256, 0, s>>>(deg, perm, n, nd, sc);
    MSF_TRY(scan_u32(c, nd, rp, (int64_t)n, nullptr));  // rp[n]: the total
    MSF_TRY(scan_u32(c, sc, so, (int64_t)n, nullptr));  // so[n]: the segment count
    k_rl_segrows<<<grid_of(n), 256, 0, s>>>(so, n, seg_row);
    k_rl_permute<<<8192, 256, 0, s>>>(rp0, col0, key0, perm, inv, rp, so, seg_row, so + n, col,
                                      key);
    MSF_HIP(hipGetLastError());
    return MSF_OK;
}

void launch_relabel_edges(hipStream_t s, int32_t *edges, int64_t m, const uint32_t *inv)
{
    if (m > 0) k_rl_edges<<<grid_of(m), 256, 0, s>>>(edges, m, inv, edges);
}

size_t relabel_table_words(int32_t n)
{
    const size_t ntiles = ((size_t)(n > 0 ? n : 1) + RL_TILE - 1) / RL_TILE;
    return 2 * (size_t)RL_CLASSES * ntiles + 2;
}

void launch_relabel_gather(hipStream_t s, const uint32_t *p, const uint32_t *perm, int32_t n,
                           uint32_t *q)
{
    if (n > 0) k_rl_gather<<<grid_of(n), 256, 0, s>>>(p, perm, n, q);
}

void launch_relabel_labels(hipStream_t s, const uint32_t *q, const uint32_t *perm, int32_t n,
                           uint32_t *labels)
{
    if (n > 0) k_rl_labels<<<grid_of(n), 256, 0, s>>>(q, perm, n, labels);
}

}  // namespace msf
