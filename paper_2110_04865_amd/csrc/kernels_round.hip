// Per-round kernels of Algorithm 2 with complete shortcutting (section 4.2),
// plus output compaction and the standalone shortcut of an arbitrary parent
// vector.
//
// State between kernels (see msf_internal.hpp): p is a star forest at the
// start of every round; R lists the roots that may still have an outgoing
// edge; r[i] holds root i's minimum outgoing key after the sweep.
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

// Append `pred` lanes of the wave to list[] through one atomic per wave.
// Every lane of the wave must call it (convergent).
__device__ __forceinline__ void wave_append(bool pred, uint32_t value, uint32_t *list,
                                            uint32_t *counter)
{
    const uint64_t mask = __ballot(pred);
    if (!mask) return;
    const int leader = __builtin_ctzll(mask);
    uint32_t base = 0;
    if ((int)__lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
    base = __shfl(base, leader, 64);
    if (pred) list[base + (uint32_t)__popcll(mask & lanemask_lt())] = value;
}

}  // namespace

// ----------------------------------------------------------- root list --
// R = vertices with at least one stored entry (isolated vertices are
// finished roots from the start).

__global__ void k_init_roots(const uint32_t *__restrict__ row_ptr, int32_t n, uint32_t *R,
                             Counters *cnt)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x; b < n; b += stride) {
        const int64_t i = b + threadIdx.x;
        const bool act = i < n && row_ptr[i + 1] > row_ptr[i];
        wave_append(act, (uint32_t)i, R, &cnt->nR);
    }
}

void launch_init_roots(hipStream_t s, const uint32_t *row_ptr, int32_t n, uint32_t *R,
                       Counters *dcnt)
{
    if (n > 0) k_init_roots<<<grid_for((size_t)n), 256, 0, s>>>(row_ptr, n, R, dcnt);
}

// ---------------------------------------------------------------- hook --
// Algorithm 2 line 11: root i takes the parent of the far endpoint of its
// minimum outgoing edge.  The EDGE pair carries the edge id; the target is
// recovered from the edge's endpoints (exactly one of them is in i's star).
// Writes go to h, never to p, so concurrent readers of p see one version.
// r[i] is reset to empty for the next round.

__global__ void k_hook(const uint32_t *__restrict__ R, uint32_t nR, uint64_t *__restrict__ r,
                       const uint32_t *__restrict__ p, const int32_t *__restrict__ edges,
                       uint32_t *__restrict__ h, uint32_t *__restrict__ hedge)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < nR; k += stride) {
        const uint32_t i = R[k];
        const uint64_t key = r[i];
        if (key != KEY_INF) {
            r[i] = KEY_INF;
            const uint32_t e = (uint32_t)key;
            const uint32_t a = p[edges[2 * (size_t)e]];
            const uint32_t b = p[edges[2 * (size_t)e + 1]];
            h[i] = (a == i) ? b : a;
            hedge[i] = e;
        } else {
            h[i] = i;
            hedge[i] = NONE32;
        }
    }
}

void launch_hook(hipStream_t s, const uint32_t *R, uint32_t nR, uint64_t *r, const uint32_t *p,
                 const int32_t *edges, uint32_t *h, uint32_t *hedge)
{
    if (nR) k_hook<<<grid_for(nR), 256, 0, s>>>(R, nR, r, p, edges, h, hedge);
}

// ----------------------------------------------------------- tie break --
// Algorithm 2 lines 12-14: a 2-cycle (i hooks on k and k on i) is the only
// cycle hooking can form (section 2.3, with keys distinct); its smaller id
// reverts to being a root and the larger keeps the hook, so the shared edge
// enters the forest once.  Roots without an outgoing edge are finished for
// good (their component is complete) and leave R.  Kept hooks flag their
// edge and join the shortcut frontier F; reverted roots stay in R.

__global__ void k_tiebreak(const uint32_t *__restrict__ R, uint32_t nR, uint32_t *h,
                           const uint32_t *__restrict__ hedge, uint8_t *__restrict__ in_forest,
                           uint32_t *__restrict__ Rnext, uint32_t *__restrict__ F, Counters *cnt)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t b = blockIdx.x * blockDim.x; b < nR; b += stride) {
        const uint32_t k = b + threadIdx.x;
        bool stay = false, hooked = false;
        uint32_t i = 0;
        if (k < nR) {
            i = R[k];
            const uint32_t t = load_relaxed_u32(h + i);
            if (t != i) {
                const uint32_t back = load_relaxed_u32(h + t);
                if (back == i && i < t) {
                    store_relaxed_u32(h + i, i);
                    stay = true;
                } else {
                    in_forest[hedge[i]] = 1;
                    hooked = true;
                }
            }
        }
        wave_append(stay, i, Rnext, &cnt->nR);
        wave_append(hooked, i, F, &cnt->nF);
    }
}

void launch_tiebreak(hipStream_t s, const uint32_t *R, uint32_t nR, uint32_t *h,
                     const uint32_t *hedge, uint8_t *in_forest, uint32_t *Rnext, uint32_t *F,
                     Counters *dcnt)
{
    if (nR) k_tiebreak<<<grid_for(nR), 256, 0, s>>>(R, nR, h, hedge, in_forest, Rnext, F, dcnt);
}

// ------------------------------------------------------------- shortcut --
// Complete shortcutting restricted to the roots that hooked (the "changed"
// set of Algorithm 3): each thread chases its hook chain to the final root,
// writing every improvement back so other chases jump further.  Every value
// read of h[x] is an ancestor of x (or x itself for a final root, which is
// never written), and the hook forest is acyclic after tie breaking, so each
// chase ends after at most the height of its tree.

__global__ void k_chase(const uint32_t *__restrict__ F, uint32_t nF, uint32_t *h, Counters *cnt)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t longest = 0;
    bool broken = false;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < nF; k += stride) {
        const uint32_t i = F[k];
        uint32_t x = load_relaxed_u32(h + i);
        uint32_t steps = 0;
        for (;;) {
            const uint32_t y = load_relaxed_u32(h + x);
            if (y == x) break;
            x = y;
            store_relaxed_u32(h + i, x);
            // a chain can hold at most nF hooked roots; longer means a cycle,
            // which tie breaking rules out -- report it instead of spinning
            if (++steps > nF) {
                broken = true;
                break;
            }
        }
        longest = steps > longest ? steps : longest;
    }
    if (__ballot(broken) && __lane_id() == 0) atomicOr(&cnt->err, ERR_CYCLE);
    for (int d = 32; d >= 1; d >>= 1) {
        uint32_t o = __shfl_xor(longest, d, 64);
        longest = o > longest ? o : longest;
    }
    if (__lane_id() == 0 && longest) atomicMax(&cnt->max_chase, longest);
}

void launch_chase(hipStream_t s, const uint32_t *F, uint32_t nF, uint32_t *h, Counters *dcnt)
{
    if (nF) k_chase<<<grid_for(nF), 256, 0, s>>>(F, nF, h, dcnt);
}

// p[v] <- h[p[v]] for every vertex that still has stored entries: p[v] is an
// old root and h maps it to its new root, so p is again a star forest.
// Vertices without entries are never read again.

__global__ void k_update_parents(const uint32_t *__restrict__ row_ptr, int32_t n,
                                 uint32_t *__restrict__ p, const uint32_t *__restrict__ h,
                                 Counters *cnt)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t rows = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (row_ptr[i + 1] > row_ptr[i]) {
            p[i] = h[p[i]];
            ++rows;
        }
    }
    rows = wave_sum(rows);
    if (__lane_id() == 0 && rows) atomicAdd(&cnt->rows, rows);
}

void launch_update_parents(hipStream_t s, const uint32_t *row_ptr, int32_t n, uint32_t *p,
                           const uint32_t *h, Counters *dcnt)
{
    launch_fill_u32(s, &dcnt->rows, 0u, 1);
    if (n) k_update_parents<<<grid_for((size_t)n), 256, 0, s>>>(row_ptr, n, p, h, dcnt);
}

// --------------------------------------------------------------- output --
// Forest flags -> ascending edge ids (order-preserving compaction with a
// decoupled look-back), the count, and the forest weight.  uint32 weights
// sum exactly in u64; float32 weights are added exactly as integers in
// units of 2^-149 (the smallest float32 subnormal) split over 32-bit digits
// held in int64 lanes, so the result is independent of the order in which
// waves finish; infinities are counted separately.

constexpr int OUT_NT = 256;
constexpr int OUT_IT = 16;
constexpr int OUT_TILE = OUT_NT * OUT_IT;
constexpr int ACC_DIGITS = 10;

template <int WT>
__global__ __launch_bounds__(OUT_NT) void k_output(const uint8_t *__restrict__ flags, int64_t m,
                                                  const void *__restrict__ w,
                                                  int32_t *__restrict__ ids, uint64_t *status,
                                                  Counters *cnt)
{
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_lds[OUT_NT / 64 + 1];
    __shared__ uint64_t s_prefix;
    if (threadIdx.x == 0) s_tile = atomicAdd(&cnt->ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t base = (int64_t)tile * OUT_TILE + (int64_t)threadIdx.x * OUT_IT;
    uint8_t f[OUT_IT];
    if (base + OUT_IT <= m) {
        const uint4 v = *reinterpret_cast<const uint4 *>(flags + base);
        const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < OUT_IT; ++k) f[k] = (uint8_t)(wd[k >> 2] >> (8 * (k & 3)));
    } else {
#pragma unroll
        for (int k = 0; k < OUT_IT; ++k) f[k] = (base + k < m) ? flags[base + k] : 0;
    }
    uint32_t cntl = 0;
#pragma unroll
    for (int k = 0; k < OUT_IT; ++k) cntl += f[k] ? 1u : 0u;
    uint32_t btot;
    const uint32_t lex = block_excl_sum<OUT_NT>(cntl, s_lds, &btot);
    if (threadIdx.x < 64) {
        const uint64_t e = lookback(status, tile, (uint64_t)btot);
        if (threadIdx.x == 0) s_prefix = e;
    }
    __syncthreads();
    uint32_t pos = (uint32_t)s_prefix + lex;
    uint64_t su = 0;
    int64_t acc[ACC_DIGITS];
#pragma unroll
    for (int d = 0; d < ACC_DIGITS; ++d) acc[d] = 0;
    uint32_t pinf = 0, ninf = 0;
#pragma unroll
    for (int k = 0; k < OUT_IT; ++k) {
        if (!f[k]) continue;
        const int64_t e = base + k;
        ids[pos++] = (int32_t)e;
        const uint32_t b = ((const uint32_t *)w)[e];
        if (WT == MSF_W_U32) {
            su += b;
        } else {
            const uint32_t ex = (b >> 23) & 0xFFu;
            const bool neg = (b >> 31) != 0;
            if (ex == 0xFFu) {
                if (neg) ++ninf;
                else ++pinf;
                continue;
            }
            const uint64_t mant = ex ? ((b & 0x7FFFFFu) | 0x800000u) : (b & 0x7FFFFFu);
            const uint32_t sh = ex ? ex - 1u : 0u;  // value = mant * 2^(sh-149)
            const uint64_t x = mant << (sh & 31u);
            const uint32_t di = sh >> 5;
            const int64_t lo = (int64_t)(x & 0xFFFFFFFFull), hi = (int64_t)(x >> 32);
#pragma unroll
            for (int d = 0; d < ACC_DIGITS; ++d) {
                int64_t add = (d == (int)di) ? lo : ((d == (int)di + 1) ? hi : 0);
                acc[d] += neg ? -add : add;
            }
        }
    }
    if (WT == MSF_W_U32) {
        su = wave_sum(su);
        if (__lane_id() == 0 && su) atomicAdd((unsigned long long *)&cnt->total_u64, (unsigned long long)su);
    } else {
        const bool any = __ballot(cntl != 0) != 0;
        if (any) {
#pragma unroll
            for (int d = 0; d < ACC_DIGITS; ++d) {
                const int64_t v = wave_sum(acc[d]);
                if (__lane_id() == 0 && v)
                    atomicAdd((unsigned long long *)&cnt->acc[d], (unsigned long long)v);
            }
            pinf = wave_sum(pinf);
            ninf = wave_sum(ninf);
            if (__lane_id() == 0 && (pinf | ninf)) {
                if (pinf) atomicAdd(&cnt->inf_pos, pinf);
                if (ninf) atomicAdd(&cnt->inf_neg, ninf);
            }
        }
    }
    const int64_t ntiles = (m + OUT_TILE - 1) / OUT_TILE;
    if ((int64_t)tile == ntiles - 1 && threadIdx.x == 0) cnt->count = (uint32_t)(s_prefix + btot);
}

void launch_output(hipStream_t s, const uint8_t *in_forest, int64_t m, const void *w, msf_wtype wt,
                   int32_t *ids, uint64_t *status, Counters *dcnt)
{
    const int64_t ntiles = (m + OUT_TILE - 1) / OUT_TILE;
    if (ntiles == 0) return;
    launch_fill_u64(s, status, 0ull, (size_t)ntiles);
    launch_fill_u32(s, &dcnt->ticket, 0u, 1);
    if (wt == MSF_W_F32)
        k_output<MSF_W_F32><<<(unsigned)ntiles, OUT_NT, 0, s>>>(in_forest, m, w, ids, status, dcnt);
    else
        k_output<MSF_W_U32><<<(unsigned)ntiles, OUT_NT, 0, s>>>(in_forest, m, w, ids, status, dcnt);
}

int64_t output_tiles(int64_t m) { return (m + OUT_TILE - 1) / OUT_TILE; }

// Round the exact accumulator to the nearest double, ties to even.
__global__ void k_finalize_total(Counters *cnt, int wt)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (wt == MSF_W_U32) {
        cnt->total_f64 = (double)cnt->total_u64;  // correctly rounded conversion
        return;
    }
    if (cnt->inf_pos || cnt->inf_neg) {
        cnt->total_f64 = (cnt->inf_pos && cnt->inf_neg) ? __builtin_nan("")
                         : (cnt->inf_pos ? __builtin_inf() : -__builtin_inf());
        return;
    }
    // carry-propagate signed digits into 32-bit digits of a two's complement
    // number of ACC_DIGITS*32 bits
    uint32_t dig[ACC_DIGITS];
    int64_t carry = 0;
    for (int d = 0; d < ACC_DIGITS; ++d) {
        const int64_t v = cnt->acc[d] + carry;
        dig[d] = (uint32_t)(v & 0xFFFFFFFFll);
        carry = v >> 32;  // arithmetic shift: floor division
    }
    const bool neg = carry < 0;
    if (neg) {  // magnitude = two's complement negation
        uint64_t c = 1;
        for (int d = 0; d < ACC_DIGITS; ++d) {
            const uint64_t v = (uint64_t)(uint32_t)~dig[d] + c;
            dig[d] = (uint32_t)v;
            c = v >> 32;
        }
    }
    int top = -1;
    for (int d = ACC_DIGITS - 1; d >= 0 && top < 0; --d)
        if (dig[d]) top = d * 32 + 31 - __builtin_clz(dig[d]);
    double out = 0.0;
    if (top >= 0) {
        auto bit = [&](int i) -> uint32_t { return i < 0 ? 0u : (dig[i >> 5] >> (i & 31)) & 1u; };
        uint64_t q = 0;
        const int lo = top - 52;  // lowest kept bit
        for (int i = top; i >= lo && i >= 0; --i) q = (q << 1) | bit(i);
        int scale = lo;  // value = q * 2^(scale - 149) before rounding
        if (lo < 0) {
            scale = 0;
            q = 0;
            for (int i = top; i >= 0; --i) q = (q << 1) | bit(i);
        } else {
            const uint32_t rb = bit(lo - 1);
            uint32_t sticky = 0;
            for (int i = lo - 2; i >= 0 && !sticky; --i) sticky |= bit(i);
            if (rb && (sticky || (q & 1u))) {
                ++q;
                if (q == (1ull << 53)) {
                    q >>= 1;
                    ++scale;
                }
            }
        }
        out = __builtin_ldexp((double)q, scale - 149);
    }
    cnt->total_f64 = neg ? -out : out;
}

void launch_finalize_total(hipStream_t s, Counters *dcnt, msf_wtype wt)
{
    k_finalize_total<<<1, 64, 0, s>>>(dcnt, (int)wt);
}

// ------------------------------------------- shortcut of arbitrary p ----
// Complete shortcutting of a caller's parent vector: synchronous-start,
// in-place pointer jumping q[i] <- q[q[i]] over a shrinking frontier of
// vertices whose parent is not yet a fixed point.  A rooted forest of
// height d converges in at most ceil(log2 d) + 1 passes.  Cycles are
// detected afterwards: every final target must be a root of the input
// (p[q[i]] == q[i]); an even cycle may collapse onto false fixed points,
// an odd one never settles, and both fail that test.

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
    if (n) k_check_parents<<<grid_for((size_t)n), 256, 0, s>>>(p, n, dcnt);
}

__global__ void k_jump_init(const uint32_t *__restrict__ q, int32_t n, uint32_t *F, Counters *cnt)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x; b < n; b += stride) {
        const int64_t i = b + threadIdx.x;
        bool act = false;
        if (i < n) {
            const uint32_t x = q[i];
            act = q[x] != x;
        }
        wave_append(act, (uint32_t)i, F, &cnt->nF);
    }
}

void launch_jump_init(hipStream_t s, const uint32_t *q, int32_t n, uint32_t *F, Counters *dcnt)
{
    if (n) k_jump_init<<<grid_for((size_t)n), 256, 0, s>>>(q, n, F, dcnt);
}

__global__ void k_jump_pass(const uint32_t *__restrict__ Fin, uint32_t nF, uint32_t *q,
                            uint32_t *__restrict__ Fout, Counters *cnt)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t b = blockIdx.x * blockDim.x; b < nF; b += stride) {
        const uint32_t k = b + threadIdx.x;
        bool again = false;
        uint32_t i = 0;
        if (k < nF) {
            i = Fin[k];
            const uint32_t x = load_relaxed_u32(q + i);
            const uint32_t y = load_relaxed_u32(q + x);
            store_relaxed_u32(q + i, y);
            again = load_relaxed_u32(q + y) != y;
        }
        wave_append(again, i, Fout, &cnt->nR);
    }
}

void launch_jump_pass(hipStream_t s, const uint32_t *Fin, uint32_t nF, uint32_t *q, uint32_t *Fout,
                      Counters *dcnt)
{
    if (nF) k_jump_pass<<<grid_for(nF), 256, 0, s>>>(Fin, nF, q, Fout, dcnt);
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

void launch_check_roots(hipStream_t s, const uint32_t *p, const uint32_t *q, int32_t n,
                        Counters *dcnt)
{
    if (n) k_check_roots<<<grid_for((size_t)n), 256, 0, s>>>(p, q, n, dcnt);
}

}  // namespace msf
