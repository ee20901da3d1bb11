/*
 * Seeded synthetic graph generators.
 *
 * Test and benchmark infrastructure shared by the oracle and the HIP path.
 * This file holds no minimum-spanning-forest arithmetic: it only emits
 * undirected edge lists (int32 endpoint pairs) and edge weights.
 *
 * Randomness is counter based: every value is a pure function of
 * (seed, stream, index), so any output can be regenerated piecewise and in
 * parallel.  The mixing function is SplitMix64's finaliser (Steele, Lea and
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014).
 *
 * Workload shapes follow the paper's evaluation (section 7): R-MAT graphs
 * for skewed social networks, high-diameter grids standing in for the
 * DIMACS road networks, and uniform random (Erdos-Renyi) graphs.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- RNG --- */

static inline uint64_t mix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

/* One 64-bit draw for (seed, stream, index); index < 2^40, stream < 2^24. */
uint64_t gen_draw(uint64_t seed, uint64_t stream, uint64_t index)
{
    return mix64(mix64(seed) ^ (stream << 40) ^ index);
}

/* Uniform integer in [0, n) from 32 random bits (multiply-shift). */
static inline uint32_t below(uint32_t bits32, uint32_t n)
{
    return (uint32_t)(((uint64_t)bits32 * (uint64_t)n) >> 32);
}

/* Stream ids.  Batched graph g uses streams STREAM_GRAPH0 + 4*g + {0..3}. */
enum {
    STREAM_TOPO = 1,
    STREAM_WEIGHT = 2,
    STREAM_PERM = 3,
    STREAM_DROP = 4,
    STREAM_SIZES = 5,
    STREAM_GRAPH0 = 16
};

/* ------------------------------------------------------------ weights --- */

/*
 * wtype 0: uint32 weight = top 32 bits of the draw.
 * wtype 1: float32 weight k * 2^-24 with k = 1 + (x >> 40) mod (2^24 - 1),
 *          so every weight is exactly representable and lies in (0, 1).
 */
void gen_weights(uint64_t seed, uint64_t stream, int64_t m, int wtype, void *out)
{
    int64_t e;
    if (wtype == 0) {
        uint32_t *w = (uint32_t *)out;
#pragma omp parallel for schedule(static)
        for (e = 0; e < m; ++e)
            w[e] = (uint32_t)(gen_draw(seed, stream, (uint64_t)e) >> 32);
    } else {
        float *w = (float *)out;
#pragma omp parallel for schedule(static)
        for (e = 0; e < m; ++e) {
            uint64_t x = gen_draw(seed, stream, (uint64_t)e);
            uint32_t k = 1u + (uint32_t)((x >> 40) % 16777215ull);
            w[e] = (float)ldexp((double)k, -24);
        }
    }
}

/* --------------------------------------------------------- radix sort --- */

/* LSD radix sort of 64-bit keys holding `bits` significant low bits. */
static void radix_sort_u64(uint64_t *a, uint64_t *tmp, int64_t n, int bits)
{
    const int RB = 11, R = 1 << RB;
    int passes = (bits + RB - 1) / RB, pass;
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    int64_t *hist = (int64_t *)malloc(sizeof(int64_t) * (size_t)nt * R);
    for (pass = 0; pass < passes; ++pass) {
        int shift = pass * RB;
        memset(hist, 0, sizeof(int64_t) * (size_t)nt * R);
#pragma omp parallel num_threads(nt)
        {
            int t = 0;
#ifdef _OPENMP
            t = omp_get_thread_num();
#endif
            int64_t lo = n * t / nt, hi = n * (t + 1) / nt, i;
            int64_t *h = hist + (size_t)t * R;
            for (i = lo; i < hi; ++i)
                h[(a[i] >> shift) & (R - 1)]++;
#pragma omp barrier
#pragma omp single
            {
                int64_t sum = 0;
                int d, tt;
                for (d = 0; d < R; ++d)
                    for (tt = 0; tt < nt; ++tt) {
                        int64_t c = hist[(size_t)tt * R + d];
                        hist[(size_t)tt * R + d] = sum;
                        sum += c;
                    }
            }
            for (i = lo; i < hi; ++i) {
                uint64_t v = a[i];
                tmp[h[(v >> shift) & (R - 1)]++] = v;
            }
        }
        memcpy(a, tmp, sizeof(uint64_t) * (size_t)n);
    }
    free(hist);
}

/* ------------------------------------------------------ Erdos-Renyi ----- */

/*
 * G(n, m): draw (u, v) uniformly with u != v, canonicalise to (min, max) and
 * reject duplicates until m distinct edges are accepted.  Acceptance order is
 * the edge id.  Returns 0, or -1 if m exceeds n(n-1)/2 or memory runs out.
 */
int gen_er(int32_t n, int64_t m, uint64_t seed, uint64_t stream, int32_t *edges)
{
    if (m == 0)
        return 0;
    if (n < 2 || (double)m > (double)n * (n - 1) / 2.0)
        return -1;
    uint64_t cap = 16;
    while (cap < (uint64_t)m * 2)
        cap <<= 1;
    uint64_t *tab = (uint64_t *)calloc(cap, sizeof(uint64_t));
    if (!tab)
        return -1;
    int64_t acc = 0;
    uint64_t i = 0;
    while (acc < m) {
        uint64_t x = gen_draw(seed, stream, i++);
        uint32_t a = below((uint32_t)(x >> 32), (uint32_t)n);
        uint32_t b = below((uint32_t)x, (uint32_t)n);
        if (a == b)
            continue;
        if (a > b) {
            uint32_t t = a;
            a = b;
            b = t;
        }
        uint64_t key = ((uint64_t)a << 32 | b) + 1; /* 0 marks an empty slot */
        uint64_t s = mix64(key) & (cap - 1);
        int dup = 0;
        while (tab[s]) {
            if (tab[s] == key) {
                dup = 1;
                break;
            }
            s = (s + 1) & (cap - 1);
        }
        if (dup)
            continue;
        tab[s] = key;
        edges[2 * acc] = (int32_t)a;
        edges[2 * acc + 1] = (int32_t)b;
        ++acc;
    }
    free(tab);
    return 0;
}

/* --------------------------------------------------------------- R-MAT -- */

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos 2004) with 2^scale vertices and
 * ef * 2^scale draws.  Each draw descends `scale` levels choosing a quadrant
 * with probabilities a, b, c, 1-a-b-c (32 random bits per level).  Vertex ids
 * are relabelled by a seeded Fisher-Yates permutation, self-loops are dropped,
 * pairs are canonicalised to (min, max), sorted and deduplicated; the rank in
 * that order is the edge id.
 *
 * Call with edges == NULL to get the edge count only (the full generation is
 * still done); otherwise `edges` must hold 2 * (count) int32.
 * Returns the number of undirected edges, or -1 on allocation failure.
 */
int64_t gen_rmat(int scale, int ef, double a, double b, double c, uint64_t seed,
                 uint64_t stream_base, int32_t *edges, int64_t edges_cap)
{
    int64_t n = (int64_t)1 << scale;
    int64_t T = (int64_t)ef << scale;
    uint64_t ta = (uint64_t)(a * 4294967296.0);
    uint64_t tb = (uint64_t)((a + b) * 4294967296.0);
    uint64_t tc = (uint64_t)((a + b + c) * 4294967296.0);
    int per = (scale + 1) / 2; /* draws per edge, two levels per draw */
    uint64_t topo = stream_base + STREAM_TOPO, pst = stream_base + STREAM_PERM;

    uint32_t *perm = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)T);
    uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)T);
    if (!perm || !key || !tmp) {
        free(perm);
        free(key);
        free(tmp);
        return -1;
    }
    int64_t i;
    for (i = 0; i < n; ++i)
        perm[i] = (uint32_t)i;
    for (i = n - 1; i > 0; --i) {
        uint64_t x = gen_draw(seed, pst, (uint64_t)i);
        uint32_t j = (uint32_t)(((x >> 32) * (uint64_t)(i + 1)) >> 32);
        uint32_t t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
    }

#pragma omp parallel for schedule(static)
    for (i = 0; i < T; ++i) {
        uint64_t row = 0, col = 0, x = 0;
        int lvl;
        for (lvl = 0; lvl < scale; ++lvl) {
            uint64_t r32;
            if ((lvl & 1) == 0) {
                x = gen_draw(seed, topo, (uint64_t)i * per + (uint64_t)(lvl >> 1));
                r32 = x >> 32;
            } else {
                r32 = x & 0xFFFFFFFFull;
            }
            uint64_t rb = 0, cb = 0;
            if (r32 < ta) {
            } else if (r32 < tb) {
                cb = 1;
            } else if (r32 < tc) {
                rb = 1;
            } else {
                rb = 1;
                cb = 1;
            }
            row = (row << 1) | rb;
            col = (col << 1) | cb;
        }
        uint64_t u = perm[row], v = perm[col];
        if (u > v) {
            uint64_t t = u;
            u = v;
            v = t;
        }
        /* self-loops become the all-ones sentinel and sort to the end */
        key[i] = (u == v) ? ~0ull : ((u << scale) | v);
    }
    radix_sort_u64(key, tmp, T, 2 * scale + 1 > 64 ? 64 : 2 * scale + 1);
    /* the sentinel has bit 2*scale set, so including it in the sort width
       keeps it after every real pair */
    int64_t cnt = 0;
    for (i = 0; i < T; ++i) {
        if (key[i] == ~0ull || (key[i] >> (2 * scale)) != 0)
            break;
        if (cnt > 0 && key[i] == key[cnt - 1])
            continue;
        key[cnt++] = key[i];
    }
    if (edges) {
        if (cnt > edges_cap) {
            cnt = -1;
        } else {
            uint64_t mask = ((uint64_t)1 << scale) - 1;
#pragma omp parallel for schedule(static)
            for (i = 0; i < cnt; ++i) {
                edges[2 * i] = (int32_t)(key[i] >> scale);
                edges[2 * i + 1] = (int32_t)(key[i] & mask);
            }
        }
    }
    free(perm);
    free(key);
    free(tmp);
    return cnt;
}

/* ---------------------------------------------------------------- grid -- */

/* Number of 7-point-stencil edges of an sx*sy*sz grid. */
int64_t gen_grid_full_edges(int32_t sx, int32_t sy, int32_t sz)
{
    return (int64_t)(sx - 1) * sy * sz + (int64_t)sx * (sy - 1) * sz +
           (int64_t)sx * sy * (sz - 1);
}

/*
 * 3D grid with vertex id x + sx*(y + sy*z).  Edges are enumerated per vertex
 * in id order as +x, +y, +z; exactly `drop` of them, chosen by a seeded
 * partial Fisher-Yates shuffle, are removed.  The rank among kept edges is
 * the edge id.  Returns the kept count, or -1 on bad arguments/allocation.
 */
int64_t gen_grid(int32_t sx, int32_t sy, int32_t sz, int64_t drop, uint64_t seed,
                 uint64_t stream_base, int32_t *edges)
{
    int64_t M = gen_grid_full_edges(sx, sy, sz);
    if (drop < 0 || drop > M || M >= ((int64_t)1 << 32))
        return -1;
    uint32_t *idx = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(M > 0 ? M : 1));
    uint8_t *gone = (uint8_t *)calloc((size_t)(M > 0 ? M : 1), 1);
    if (!idx || !gone) {
        free(idx);
        free(gone);
        return -1;
    }
    int64_t i;
    for (i = 0; i < M; ++i)
        idx[i] = (uint32_t)i;
    uint64_t dst = stream_base + STREAM_DROP;
    for (i = 0; i < drop; ++i) {
        uint64_t x = gen_draw(seed, dst, (uint64_t)i);
        int64_t span = M - i;
        int64_t j = i + (int64_t)(((x >> 32) * (uint64_t)span) >> 32);
        uint32_t t = idx[i];
        idx[i] = idx[j];
        idx[j] = t;
    }
    for (i = 0; i < drop; ++i)
        gone[idx[i]] = 1;
    free(idx);
    int64_t k = 0, e = 0;
    int32_t x, y, z;
    for (z = 0; z < sz; ++z)
        for (y = 0; y < sy; ++y)
            for (x = 0; x < sx; ++x) {
                int32_t v = x + sx * (y + sy * z);
                if (x + 1 < sx) {
                    if (!gone[e]) {
                        edges[2 * k] = v;
                        edges[2 * k + 1] = v + 1;
                        ++k;
                    }
                    ++e;
                }
                if (y + 1 < sy) {
                    if (!gone[e]) {
                        edges[2 * k] = v;
                        edges[2 * k + 1] = v + sx;
                        ++k;
                    }
                    ++e;
                }
                if (z + 1 < sz) {
                    if (!gone[e]) {
                        edges[2 * k] = v;
                        edges[2 * k + 1] = v + sx * sy;
                        ++k;
                    }
                    ++e;
                }
            }
    free(gone);
    return k;
}

/* ------------------------------------------------------------- batched -- */

/*
 * Vertex counts of a batch: n_g = floor(lo * (hi/lo)^U), U uniform in [0,1).
 */
void gen_batch_sizes(int32_t G, int32_t lo, int32_t hi, uint64_t seed, int32_t *n_out)
{
    int32_t g;
    double ratio = (double)hi / (double)lo;
    for (g = 0; g < G; ++g) {
        uint64_t x = gen_draw(seed, STREAM_SIZES, (uint64_t)g);
        double u = (double)(x >> 11) * 0x1.0p-53;
        int32_t v = (int32_t)floor((double)lo * pow(ratio, u));
        if (v < lo)
            v = lo;
        if (v >= hi)
            v = hi - 1;
        n_out[g] = v;
    }
}

/*
 * Fill a batch of G Erdos-Renyi graphs whose sizes and offsets the caller
 * computed: graph g has vtx_off[g+1]-vtx_off[g] vertices and
 * edge_off[g+1]-edge_off[g] edges, written with local vertex ids at
 * edges[2*edge_off[g]].  Weights use the same per-graph stream family.
 * Returns 0, or the (1-based) index of the first graph that failed.
 */
int gen_batch_fill(int32_t G, const int64_t *vtx_off, const int64_t *edge_off, uint64_t seed,
                   int wtype, int32_t *edges, void *weights)
{
    int32_t g;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (g = 0; g < G; ++g) {
        int32_t n = (int32_t)(vtx_off[g + 1] - vtx_off[g]);
        int64_t m = edge_off[g + 1] - edge_off[g];
        uint64_t sb = STREAM_GRAPH0 + 4 * (uint64_t)g;
        if (gen_er(n, m, seed, sb, edges + 2 * edge_off[g]) != 0) {
#pragma omp critical
            if (!bad || g + 1 < bad)
                bad = g + 1;
            continue;
        }
        if (wtype == 0)
            gen_weights(seed, sb + 1, m, 0, (uint32_t *)weights + edge_off[g]);
        else
            gen_weights(seed, sb + 1, m, 1, (float *)weights + edge_off[g]);
    }
    return bad;
}
