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

// deg[v] += 1 for each end of every edge that is not a loop; endpoints
// outside [0, n) raise ERR_ENDPOINT and are skipped.
__global__ void k_rl_degree(const int32_t *__restrict__ edges, int64_t m, int32_t n,
                            uint32_t *__restrict__ deg, Counters *cnt)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
        const int32_t u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || v < 0 || u >= n || v >= n) {
            bad = true;
            continue;
        }
        if (u == v) continue;
        atomicAdd(deg + u, 1u);
        atomicAdd(deg + v, 1u);
    }
    if (__ballot(bad) && __lane_id() == 0) atomicOr(&cnt->err, ERR_ENDPOINT);
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

// edges_out = inv applied to both ends (endpoints already checked).
__global__ void k_rl_edges(const int32_t *__restrict__ edges, int64_t m,
                           const uint32_t *__restrict__ inv, int32_t *__restrict__ out)
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

}  // namespace

msf_status relabel_by_degree(Ctx *c, int32_t n, int64_t m, const int32_t *d_edges, uint32_t *deg,
                             uint32_t *tab, uint32_t *perm, uint32_t *inv, int32_t *edges_out)
{
    hipStream_t s = c->stream;
    const uint32_t ntiles = (uint32_t)(((int64_t)n + RL_TILE - 1) / RL_TILE);
    launch_fill_u32(s, deg, 0u, (size_t)n);
    launch_fill_u32(s, &c->dcnt->err, 0u, 1);
    if (m > 0) k_rl_degree<<<grid_of(m), 256, 0, s>>>(d_edges, m, n, deg, c->dcnt);
    // the endpoints index inv below: stop here if any is out of range
    MSF_TRY(read_counters(c));
    MSF_TRY(decode_err(c->hcnt->err));
    if (n > 0) {
        k_rl_count<<<ntiles, 64, 0, s>>>(deg, n, ntiles, tab);
        MSF_TRY(scan_u32(c, tab, tab + (size_t)RL_CLASSES * ntiles + 1,
                         (int64_t)RL_CLASSES * ntiles, nullptr));
        k_rl_place<<<ntiles, 64, 0, s>>>(deg, n, ntiles, tab + (size_t)RL_CLASSES * ntiles + 1,
                                         perm, inv);
    }
    if (m > 0) k_rl_edges<<<grid_of(m), 256, 0, s>>>(d_edges, m, inv, edges_out);
    MSF_HIP(hipGetLastError());
    return MSF_OK;
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
