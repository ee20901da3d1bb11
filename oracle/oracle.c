/*
 * CPU oracle for the algebraic Awerbuch-Shiloach MSF hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link
 * or call this file; it shares no code with the HIP library.  Only the tests,
 * the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * Plain, slow and obviously correct loops, each the definition of what the
 * GPU path computes:
 *
 *  - oracle_kruskal: the minimum spanning forest under the total edge order
 *    key(e) = (weight key, edge id).  The paper's method reaches exactly the
 *    minimum spanning forest (section 2, problem statement; Algorithm 2
 *    returns its weight), and with ties broken by edge id that forest is
 *    unique, so Kruskal's algorithm (edges in increasing key order, keep an
 *    edge iff it joins two different trees) is its plain definition.
 *    The caller passes the keys already sorted (a library sort is a step).
 *
 *  - oracle_multilinear: the all-at-once multilinear kernel of section 3.1
 *    fused with the projection of Algorithm 2 (minimum outgoing edge of each
 *    vertex, projected onto its parent): for every stored direction i->j of
 *    every edge with p[i] != p[j], r[p[i]] = min(r[p[i]], key).
 *
 *  - oracle_multilinear_rows: the same over the stored directions whose row
 *    lies in a given subset of the vertices (one owner's share when the
 *    rows of A are split, section 5).
 *
 *  - oracle_find_roots: the result of complete shortcutting (section 4.2):
 *    every vertex points at the root of its tree in the parent forest.
 *
 *  - oracle_components: the connected components that the connectivity
 *    variant of the Awerbuch-Shiloach algorithm computes (section 2.4),
 *    by their plain definition: union-find over every edge, each vertex
 *    labelled with the smallest vertex id of its component.
 */
#include <stdint.h>
#include <stdlib.h>

/* --------------------------------------------------------- Kruskal ------ */

static int32_t dsu_find(int32_t *parent, int32_t x)
{
    while (parent[x] != x) {
        parent[x] = parent[parent[x]]; /* path halving */
        x = parent[x];
    }
    return x;
}

/*
 * sorted_keys[k] = (wkey << 32) | eid for the k-th smallest key, self-loops
 * already excluded.  edges[2*eid], edges[2*eid+1] are the endpoints.
 * in_forest[eid] is set to 1 for forest edges (caller zeroes it).
 * Returns the number of forest edges.
 */
int64_t oracle_kruskal(int32_t n, int64_t nkeys, const uint64_t *sorted_keys, const int32_t *edges,
                       uint8_t *in_forest)
{
    int32_t *parent = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *size = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t k, count = 0;
    int32_t i;
    if (!parent || !size) {
        free(parent);
        free(size);
        return -1;
    }
    for (i = 0; i < n; ++i) {
        parent[i] = i;
        size[i] = 1;
    }
    for (k = 0; k < nkeys && count < (int64_t)n - 1; ++k) {
        uint32_t e = (uint32_t)(sorted_keys[k] & 0xFFFFFFFFu);
        int32_t a = dsu_find(parent, edges[2 * (int64_t)e]);
        int32_t b = dsu_find(parent, edges[2 * (int64_t)e + 1]);
        if (a == b)
            continue;
        if (size[a] < size[b]) {
            int32_t t = a;
            a = b;
            b = t;
        }
        parent[b] = a; /* union by size */
        size[a] += size[b];
        in_forest[e] = 1;
        ++count;
    }
    free(parent);
    free(size);
    return count;
}

/* ---------------------------------------------------- multilinear ------- */

/*
 * keys[e] = (wkey << 32) | e.  r (length n) receives UINT64_MAX where no
 * entry qualifies.  Self-loops (u == v) never qualify since p[u] == p[v].
 */
void oracle_multilinear(int32_t n, int64_t m, const int32_t *edges, const uint64_t *keys,
                        const uint32_t *p, uint64_t *r)
{
    int64_t e;
    int32_t i;
    for (i = 0; i < n; ++i)
        r[i] = UINT64_MAX;
    for (e = 0; e < m; ++e) {
        int32_t u = edges[2 * e], v = edges[2 * e + 1];
        uint32_t pu = p[u], pv = p[v];
        if (pu == pv)
            continue;
        if (keys[e] < r[pu]) /* direction u -> v */
            r[pu] = keys[e];
        if (keys[e] < r[pv]) /* direction v -> u */
            r[pv] = keys[e];
    }
}

/*
 * The same kernel over the stored directions whose row is in a subset of the
 * vertices (row_in[i] != 0): the share of the minima that one owner of
 * those rows computes when the rows of A are split among several owners,
 * each holding the whole parent vector (section 5).
 */
void oracle_multilinear_rows(int32_t n, int64_t m, const int32_t *edges, const uint64_t *keys,
                             const uint32_t *p, const uint8_t *row_in, uint64_t *r)
{
    int64_t e;
    int32_t i;
    for (i = 0; i < n; ++i)
        r[i] = UINT64_MAX;
    for (e = 0; e < m; ++e) {
        int32_t u = edges[2 * e], v = edges[2 * e + 1];
        uint32_t pu = p[u], pv = p[v];
        if (pu == pv)
            continue;
        if (row_in[u] && keys[e] < r[pu]) /* direction u -> v, row u */
            r[pu] = keys[e];
        if (row_in[v] && keys[e] < r[pv]) /* direction v -> u, row v */
            r[pv] = keys[e];
    }
}

/* ----------------------------------------------------- root finding ----- */

/*
 * root[i] = the vertex reached from i by following p until p[x] == x.
 * Returns 0, or -1 if some walk enters a cycle of length >= 2 (p is then not
 * a rooted forest), or -2 if some p[i] is out of range.
 * Uses state[] marks: 0 unvisited, 1 on the current walk, 2 resolved.
 */
int oracle_find_roots(int32_t n, const uint32_t *p, uint32_t *root)
{
    uint8_t *state = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    uint32_t *stack = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    int32_t i;
    int rc = 0;
    if (!state || !stack) {
        free(state);
        free(stack);
        return -3;
    }
    for (i = 0; i < n; ++i)
        if (p[i] >= (uint32_t)n) {
            rc = -2;
            goto done;
        }
    for (i = 0; i < n && rc == 0; ++i) {
        int32_t top = 0;
        uint32_t x = (uint32_t)i;
        while (state[x] == 0 && p[x] != x) {
            state[x] = 1;
            stack[top++] = x;
            x = p[x];
        }
        if (state[x] == 1) { /* walked back onto the current path */
            rc = -1;
            break;
        }
        uint32_t r = (state[x] == 2) ? root[x] : x;
        if (state[x] == 0) {
            state[x] = 2;
            root[x] = x;
        }
        while (top > 0) {
            uint32_t y = stack[--top];
            root[y] = r;
            state[y] = 2;
        }
    }
done:
    free(state);
    free(stack);
    return rc;
}

/* ------------------------------------------------ connected components -- */

/*
 * label[i] = the smallest vertex id in i's connected component (edges taken
 * as undirected, self-loops and parallel edges allowed).  Union-find with
 * path halving; every union keeps the smaller root, so each final root is
 * its component's smallest vertex.  Returns the number of components, or -1
 * if an endpoint is outside [0, n).
 */
int64_t oracle_components(int32_t n, int64_t m, const int32_t *edges, int32_t *label)
{
    int32_t *parent = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t e, comps = 0;
    int32_t i;
    if (!parent)
        return -2;
    for (i = 0; i < n; ++i)
        parent[i] = i;
    for (e = 0; e < m; ++e) {
        int32_t u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || v < 0 || u >= n || v >= n) {
            free(parent);
            return -1;
        }
        int32_t a = dsu_find(parent, u), b = dsu_find(parent, v);
        if (a < b)
            parent[b] = a;
        else if (b < a)
            parent[a] = b;
    }
    for (i = 0; i < n; ++i) {
        label[i] = dsu_find(parent, i);
        if (label[i] == i)
            ++comps;
    }
    free(parent);
    return comps;
}
