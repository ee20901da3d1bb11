/*
 * Host-side sanitizer run of the oracle and the seeded input generators
 * (test infrastructure, plain C; built with gcc -fsanitize=address,undefined
 * by tests/test_host_sanitize.py).  Small graphs from every generator go
 * through every oracle routine, with checks that hold for any input:
 *   - a spanning forest has n - (number of components) edges (section 2);
 *   - with p the identity, the multilinear kernel of section 3.1 with the
 *     projection of Algorithm 2 gives each vertex the smallest key of an
 *     edge at it (brute force over the edge list);
 *   - with p = the component labels no edge joins two stars, so every r is
 *     empty;
 *   - the labels form a rooted forest of height one whose roots are the
 *     labels themselves (find_roots).
 * Prints "ok" and returns 0 when every check passes.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t oracle_kruskal(int32_t n, int64_t nkeys, const uint64_t *sorted_keys, const int32_t *edges,
                       uint8_t *in_forest);
void oracle_multilinear(int32_t n, int64_t m, const int32_t *edges, const uint64_t *keys,
                        const uint32_t *p, uint64_t *r);
int oracle_find_roots(int32_t n, const uint32_t *p, uint32_t *root);
int64_t oracle_components(int32_t n, int64_t m, const int32_t *edges, int32_t *label);

void gen_weights(uint64_t seed, uint64_t stream, int64_t m, int wtype, void *out);
int gen_er(int32_t n, int64_t m, uint64_t seed, uint64_t stream, int32_t *edges);
int64_t gen_rmat(int scale, int ef, double a, double b, double c, uint64_t seed,
                 uint64_t stream_base, int32_t *edges, int64_t edges_cap);
int64_t gen_grid_full_edges(int32_t sx, int32_t sy, int32_t sz);
int64_t gen_grid(int32_t sx, int32_t sy, int32_t sz, int64_t drop, uint64_t seed,
                 uint64_t stream_base, int32_t *edges);
void gen_batch_sizes(int32_t G, int32_t lo, int32_t hi, uint64_t seed, int32_t *n_out);
int gen_batch_fill(int32_t G, const int64_t *vtx_off, const int64_t *edge_off, uint64_t seed,
                   int wtype, int32_t *edges, void *weights);

static int failures = 0;

static void fail(const char *name, const char *what)
{
    printf("FAIL %s: %s\n", name, what);
    ++failures;
}

static int cmp_u64(const void *a, const void *b)
{
    const uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static void check_graph(const char *name, int32_t n, int64_t m, const int32_t *edges,
                        const uint32_t *w)
{
    const size_t nn = (size_t)(n > 0 ? n : 1), mm = (size_t)(m > 0 ? m : 1);
    uint64_t *keys = malloc(8 * mm), *sorted = malloc(8 * mm), *r = malloc(8 * nn);
    uint64_t *best = malloc(8 * nn);
    uint8_t *in_forest = calloc(mm, 1);
    int32_t *label = malloc(4 * nn);
    uint32_t *p = malloc(4 * nn), *root = malloc(4 * nn);
    int64_t nk = 0, e;
    int32_t i;
    for (e = 0; e < m; ++e) {
        keys[e] = ((uint64_t)w[e] << 32) | (uint64_t)e;
        if (edges[2 * e] != edges[2 * e + 1]) sorted[nk++] = keys[e];
    }
    qsort(sorted, (size_t)nk, 8, cmp_u64);
    const int64_t f = oracle_kruskal(n, nk, sorted, edges, in_forest);
    const int64_t comps = oracle_components(n, m, edges, label);
    if (comps < 0) fail(name, "components rejected the edges");
    if (f != (int64_t)n - comps) fail(name, "forest size is not n - components");
    int64_t flagged = 0;
    for (e = 0; e < m; ++e) flagged += in_forest[e];
    if (flagged != f) fail(name, "forest flags disagree with the count");

    /* identity parents: each vertex's smallest incident key */
    for (i = 0; i < n; ++i) {
        p[i] = (uint32_t)i;
        best[i] = UINT64_MAX;
    }
    for (e = 0; e < m; ++e) {
        const int32_t u = edges[2 * e], v = edges[2 * e + 1];
        if (u == v) continue;
        if (keys[e] < best[u]) best[u] = keys[e];
        if (keys[e] < best[v]) best[v] = keys[e];
    }
    oracle_multilinear(n, m, edges, keys, p, r);
    for (i = 0; i < n; ++i)
        if (r[i] != best[i]) {
            fail(name, "identity multilinear differs from the smallest incident key");
            break;
        }

    /* component stars: no edge leaves a star */
    for (i = 0; i < n; ++i) p[i] = (uint32_t)label[i];
    oracle_multilinear(n, m, edges, keys, p, r);
    for (i = 0; i < n; ++i)
        if (r[i] != UINT64_MAX) {
            fail(name, "an edge joins two components");
            break;
        }
    if (oracle_find_roots(n, p, root) != 0) fail(name, "labels are not a rooted forest");
    for (i = 0; i < n; ++i)
        if (root[i] != p[i]) {
            fail(name, "a label is not its own root");
            break;
        }
    free(keys);
    free(sorted);
    free(r);
    free(best);
    free(in_forest);
    free(label);
    free(p);
    free(root);
}

int main(void)
{
    /* Erdos-Renyi */
    {
        const int32_t n = 300;
        const int64_t m = 1200;
        int32_t *edges = malloc(8 * (size_t)m);
        uint32_t *w = malloc(4 * (size_t)m);
        if (gen_er(n, m, 11, 0, edges) != 0) fail("er", "generator failed");
        gen_weights(11, 1, m, 0, w);
        check_graph("er", n, m, edges, w);
        free(edges);
        free(w);
    }
    /* R-MAT scale 10, edge factor 8 */
    {
        const int64_t cap = (int64_t)8 << 10;
        int32_t *edges = malloc(8 * (size_t)cap);
        const int64_t m = gen_rmat(10, 8, 0.57, 0.19, 0.19, 12, 0, edges, cap);
        if (m <= 0) fail("rmat", "generator failed");
        uint32_t *w = malloc(4 * (size_t)(m > 0 ? m : 1));
        gen_weights(12, 7, m, 0, w);
        if (m > 0) check_graph("rmat", 1 << 10, m, edges, w);
        free(edges);
        free(w);
    }
    /* 3D grid 9 x 7 x 5 with edges dropped (several components) */
    {
        const int64_t full = gen_grid_full_edges(9, 7, 5), drop = full / 3;
        int32_t *edges = malloc(8 * (size_t)(full - drop));
        const int64_t m = gen_grid(9, 7, 5, drop, 13, 0, edges);
        if (m != full - drop) fail("grid", "generator failed");
        uint32_t *w = malloc(4 * (size_t)(m > 0 ? m : 1));
        gen_weights(13, 9, m, 0, w);
        if (m > 0) check_graph("grid", 9 * 7 * 5, m, edges, w);
        free(edges);
        free(w);
    }
    /* a batch of small Erdos-Renyi graphs, each checked alone */
    {
        const int32_t G = 6;
        int32_t nv[6];
        int64_t vo[7], eo[7];
        gen_batch_sizes(G, 16, 200, 14, nv);
        vo[0] = eo[0] = 0;
        for (int g = 0; g < G; ++g) {
            vo[g + 1] = vo[g] + nv[g];
            eo[g + 1] = eo[g] + 2 * (int64_t)nv[g];
        }
        int32_t *edges = malloc(8 * (size_t)eo[G]);
        uint32_t *w = malloc(4 * (size_t)eo[G]);
        if (gen_batch_fill(G, vo, eo, 14, 0, edges, w) != 0) fail("batch", "generator failed");
        for (int g = 0; g < G; ++g)
            check_graph("batch", nv[g], eo[g + 1] - eo[g], edges + 2 * eo[g], w + eo[g]);
        free(edges);
        free(w);
    }
    /* degenerate: no edges, one vertex */
    {
        int32_t e0[2] = {0, 0};
        uint32_t w0[1] = {5};
        check_graph("single self-loop", 1, 1, e0, w0);
        check_graph("empty", 4, 0, e0, w0);
    }
    if (failures) return 1;
    printf("ok\n");
    return 0;
}
