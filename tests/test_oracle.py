"""Pins of the CPU oracle against facts that do not come from the oracle.

Every check here is independent of the oracle's own code path: brute-force
enumeration of spanning forests, a library MST (scipy) on distinct weights,
closed forms, the cycle-property certificate, a library connected-components
count, exact rational arithmetic for float totals, and a second formulation
(dense, two-step, as written in Algorithm 2) for the multilinear kernel.
"""
import itertools
import math
import random
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, minimum_spanning_tree

import gen
import oracle

U32, F32 = oracle.W_U32, oracle.W_F32


# ----------------------------------------------------------- helpers ----

def components(n, edges):
    """Connected components by breadth-first search (test-local)."""
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    comp = [-1] * n
    c = 0
    for s in range(n):
        if comp[s] >= 0:
            continue
        comp[s] = c
        stack = [s]
        while stack:
            x = stack.pop()
            for y in adj[x]:
                if comp[y] < 0:
                    comp[y] = c
                    stack.append(y)
        c += 1
    return c, comp


def brute_force_msf(n, edges, w):
    """Enumerate every spanning forest; pick min (sum w, sum eid).

    For integer weights this is the forest that is minimal under the order
    (w, eid): perturbing w_e by eps*e with eps*sum(e) < 1 makes all weights
    distinct without reordering unequal ones, and the unique MSF under the
    perturbed weights minimises sum(w) + eps*sum(e)."""
    c, _ = components(n, [tuple(e) for e in edges])
    k = n - c
    cand = [i for i, (a, b) in enumerate(edges) if a != b]
    best = None
    for sub in itertools.combinations(cand, k):
        cc, _ = components(n, [tuple(edges[i]) for i in sub])
        if cc != c:
            continue
        score = (sum(w[i] for i in sub), sum(sub))
        if best is None or score < best[0]:
            best = (score, sub)
    return sorted(best[1]) if best else []


def random_multigraph(rng, n, m, wmax, selfloops=True):
    edges = []
    for _ in range(m):
        a = rng.randrange(n)
        b = rng.randrange(n) if (selfloops or n == 1) else rng.choice([x for x in range(n) if x != a])
        edges.append((a, b))
    w = [rng.randint(0, wmax) for _ in range(m)]
    return np.array(edges, dtype=np.int32).reshape(-1, 2), w


def cycle_property_ok(n, edges, keys, ids):
    """Every non-forest edge is the largest key on its fundamental cycle and
    the forest connects its endpoints (certificate of the unique MSF)."""
    fs = set(int(i) for i in ids)
    adj = [[] for _ in range(n)]
    for i in fs:
        a, b = int(edges[i][0]), int(edges[i][1])
        adj[a].append((b, i))
        adj[b].append((a, i))
    parent = [-1] * n
    pkey = [0] * n
    depth = [-1] * n
    for s in range(n):
        if depth[s] >= 0:
            continue
        depth[s] = 0
        stack = [s]
        while stack:
            x = stack.pop()
            for y, i in adj[x]:
                if depth[y] < 0:
                    depth[y] = depth[x] + 1
                    parent[y] = x
                    pkey[y] = int(keys[i])
                    stack.append(y)
    # forest must be acyclic: |F| = n - components(F)
    c, _ = components(n, [tuple(edges[i]) for i in fs])
    if len(fs) != n - c:
        return False
    for i in range(len(edges)):
        if i in fs:
            continue
        a, b = int(edges[i][0]), int(edges[i][1])
        if a == b:
            continue
        mx = -1
        x, y = a, b
        while x != y:
            if depth[x] < 0 or depth[y] < 0:
                return False
            if depth[x] >= depth[y]:
                if parent[x] < 0:
                    return False  # different trees: forest not spanning
                mx = max(mx, pkey[x])
                x = parent[x]
            else:
                if parent[y] < 0:
                    return False
                mx = max(mx, pkey[y])
                y = parent[y]
        if not int(keys[i]) > mx:
            return False
    return True


# ------------------------------------------------------- brute force ----

@pytest.mark.parametrize("seed", range(60))
def test_bruteforce_tiny_uint(seed):
    rng = random.Random(seed)
    n = rng.randint(1, 7)
    m = rng.randint(0, 10)
    edges, w = random_multigraph(rng, n, m, wmax=rng.choice([1, 3, 1000]))
    ids, cnt, tot = oracle.msf(n, edges, np.array(w, dtype=np.uint32), U32)
    want = brute_force_msf(n, edges.tolist(), w)
    assert list(ids) == want
    assert cnt == len(want)
    assert tot[0] == sum(w[i] for i in want)


@pytest.mark.parametrize("seed", range(30))
def test_bruteforce_tiny_float(seed):
    rng = random.Random(1000 + seed)
    n = rng.randint(2, 7)
    m = rng.randint(1, 10)
    edges, _ = random_multigraph(rng, n, m, 0)
    # integer-valued floats, negatives and both zeros (which compare equal)
    vals = [rng.choice([-3.0, -1.0, -0.0, 0.0, 1.0, 2.0, 5.0]) for _ in range(m)]
    w = np.array(vals, dtype=np.float32)
    ids, cnt, tot = oracle.msf(n, edges, w, F32)
    want = brute_force_msf(n, edges.tolist(), [int(x) for x in vals])
    assert list(ids) == want
    assert tot[1] == float(sum(vals[i] for i in want))


# --------------------------------------------------------- library MST --

@pytest.mark.parametrize("seed,n,m", [(1, 300, 1200), (2, 2000, 12000), (3, 5000, 8000)])
def test_scipy_mst_distinct_weights(seed, n, m):
    e, _ = gen.er(n, m, seed=seed)
    rng = np.random.default_rng(seed)
    w = (rng.permutation(m) + 1).astype(np.uint32)  # distinct, nonzero
    ids, cnt, _ = oracle.msf(n, e, w, U32)
    A = sp.coo_matrix((w.astype(np.float64), (e[:, 0], e[:, 1])), shape=(n, n)).tocsr()
    T = minimum_spanning_tree(A).tocoo()
    got = {(min(a, b), max(a, b)) for a, b in e[ids]}
    want = {(min(a, b), max(a, b)) for a, b in zip(T.row, T.col)}
    assert got == want
    assert cnt == T.nnz


def test_scipy_mst_rmat_float():
    n, e, w = gen.rmat(12, 16, seed=7, wtype=F32)
    # make float weights distinct: keep the first occurrence of each value
    _, first = np.unique(w, return_index=True)
    keep = np.sort(first)
    e, w = e[keep], w[keep]
    ids, cnt, _ = oracle.msf(n, e, w, F32)
    A = sp.coo_matrix((w.astype(np.float64), (e[:, 0], e[:, 1])), shape=(n, n)).tocsr()
    T = minimum_spanning_tree(A).tocoo()
    got = {(min(a, b), max(a, b)) for a, b in e[ids]}
    want = {(min(a, b), max(a, b)) for a, b in zip(T.row, T.col)}
    assert got == want


# -------------------------------------------------------- closed forms --

def test_tree_input_keeps_all_edges():
    rng = np.random.default_rng(5)
    n = 1000
    par = np.array([rng.integers(0, i) for i in range(1, n)])
    e = np.stack([np.arange(1, n), par], axis=1).astype(np.int32)
    w = rng.integers(0, 2**32, size=n - 1, dtype=np.uint64).astype(np.uint32)
    ids, cnt, tot = oracle.msf(n, e, w, U32)
    assert cnt == n - 1 and list(ids) == list(range(n - 1))
    assert tot[0] == int(w.astype(np.uint64).sum())


@pytest.mark.parametrize("n", [3, 4, 17, 100])
def test_cycle_drops_max_key(n):
    rng = np.random.default_rng(n)
    e = np.stack([np.arange(n), (np.arange(n) + 1) % n], axis=1).astype(np.int32)
    w = rng.integers(0, 5, size=n).astype(np.uint32)  # many ties
    ids, cnt, _ = oracle.msf(n, e, w, U32)
    key = [(int(w[i]), i) for i in range(n)]
    drop = max(range(n), key=lambda i: key[i])
    assert cnt == n - 1 and drop not in set(ids.tolist())


@pytest.mark.parametrize("n", [2, 5, 30])
def test_complete_graph_i_plus_j_is_star(n):
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    e = np.array(pairs, dtype=np.int32)
    w = np.array([i + j for i, j in pairs], dtype=np.uint32)
    ids, cnt, tot = oracle.msf(n, e, w, U32)
    assert sorted(tuple(e[i]) for i in ids) == [(0, j) for j in range(1, n)]
    assert tot[0] == n * (n - 1) // 2


@pytest.mark.parametrize("n", [2, 6, 25])
def test_complete_graph_equal_weights_lex_ids(n):
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    e = np.array(pairs, dtype=np.int32)
    ids, _, _ = oracle.msf(n, e, np.full(len(pairs), 7, dtype=np.uint32), U32)
    assert list(ids) == list(range(n - 1))  # (0,1) .. (0,n-1)


def test_empty_and_degenerate():
    for n in (0, 1, 5):
        ids, cnt, tot = oracle.msf(n, np.zeros((0, 2), np.int32), np.zeros(0, np.uint32), U32)
        assert cnt == 0 and len(ids) == 0 and tot == (0, 0.0)
    e = np.array([[0, 0], [1, 1], [2, 2]], dtype=np.int32)
    ids, cnt, _ = oracle.msf(3, e, np.array([1, 2, 3], np.uint32), U32)
    assert cnt == 0
    # parallel edges: the smaller key wins, equal weights -> smaller id
    e = np.array([[0, 1], [1, 0], [0, 1]], dtype=np.int32)
    ids, _, _ = oracle.msf(2, e, np.array([5, 5, 4], np.uint32), U32)
    assert list(ids) == [2]
    ids, _, _ = oracle.msf(2, e, np.array([5, 5, 6], np.uint32), U32)
    assert list(ids) == [0]


def test_disjoint_copies_scale_total():
    n, e, w = 4096, *gen.er(4096, 32768, seed=11)
    ids, cnt, tot = oracle.msf(n, e, w, U32)
    k = 3
    ee = np.concatenate([e + i * n for i in range(k)])
    ww = np.concatenate([w] * k)
    ids3, cnt3, tot3 = oracle.msf(k * n, ee, ww, U32)
    assert cnt3 == k * cnt and tot3[0] == k * tot[0]
    assert list(ids3) == [int(i) + j * len(e) for j in range(k) for i in ids]


def test_invalid_inputs_raise():
    with pytest.raises(ValueError):
        oracle.msf(2, np.array([[0, 2]], np.int32), np.array([1], np.uint32), U32)
    with pytest.raises(ValueError):
        oracle.msf(2, np.array([[0, 1]], np.int32), np.array([np.nan], np.float32), F32)
    with pytest.raises(ValueError):
        oracle.msf(2, np.array([[-1, 1]], np.int32), np.array([1], np.uint32), U32)


# --------------------------------------------- counts and certificates --

@pytest.mark.parametrize("seed,n,m", [(1, 3000, 2000), (2, 3000, 6000), (3, 500, 5000)])
def test_count_is_n_minus_components(seed, n, m):
    e, w = gen.er(n, m, seed=seed)
    ids, cnt, _ = oracle.msf(n, e, w, U32)
    A = sp.coo_matrix((np.ones(m), (e[:, 0], e[:, 1])), shape=(n, n))
    c, lab = connected_components(A, directed=False)
    assert cnt == n - c
    # forest spans the same partition
    F = sp.coo_matrix((np.ones(cnt), (e[ids, 0], e[ids, 1])), shape=(n, n))
    cf, labf = connected_components(F, directed=False)
    assert cf == c
    assert len(set(zip(lab.tolist(), labf.tolist()))) == c


def test_count_grid_with_many_components():
    n, e, w = gen.grid(12, 12, 12, 0.4, seed=9)
    ids, cnt, _ = oracle.msf(n, e, w, U32)
    A = sp.coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n, n))
    c, _ = connected_components(A, directed=False)
    assert cnt == n - c and c > 1


@pytest.mark.parametrize("seed", range(6))
def test_cycle_property_certificate(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(50, 1500))
    m = int(rng.integers(n // 2, 4 * n))
    e, w = gen.er(n, m, seed=100 + seed)
    if seed % 2:
        w = (w % 16).astype(np.uint32)  # heavy ties
    ids, _, _ = oracle.msf(n, e, w, U32)
    keys = oracle.edge_keys(w, U32)
    assert cycle_property_ok(n, e.tolist(), keys, ids)


def test_cycle_property_detects_planted_error():
    n, e, w = 200, *gen.er(200, 800, seed=3)
    ids, _, _ = oracle.msf(n, e, w, U32)
    keys = oracle.edge_keys(w, U32)
    non = sorted(set(range(len(e))) - set(ids.tolist()))
    bad = np.array(sorted(ids.tolist()[1:] + [non[0]]))
    assert not cycle_property_ok(n, e.tolist(), keys, bad)


# --------------------------------------------------------- weight keys --

def test_float_keys_follow_float_order():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(5000).astype(np.float32) * 1e3,
                        np.array([0.0, -0.0, np.inf, -np.inf, 1e-45, -1e-45,
                                  3.4e38, -3.4e38], np.float32)])
    k = oracle.weight_keys(x, F32)
    for i in range(0, len(x), 7):
        for j in range(0, len(x), 13):
            assert (x[i] < x[j]) == (k[i] < k[j])
            assert (x[i] == x[j]) == (k[i] == k[j])


def test_float_total_is_exact_rounding():
    rng = np.random.default_rng(2)
    w = (rng.standard_normal(2000) * 10.0 ** rng.integers(-30, 30, 2000)).astype(np.float32)
    ids = np.arange(0, 2000, 3)
    _, got = oracle.total(w, ids, F32)
    exact = sum(Fraction(float(w[i])) for i in ids)
    assert got == float(exact)


def test_grid_weights_sum_exactly():
    # float weights on the k*2^-24 lattice: any order of float64 addition
    # is exact below 2^53 * 2^-24
    w = gen.weights(100000, gen.W_F32, seed=3)
    s_fwd = 0.0
    for x in w.astype(np.float64):
        s_fwd += x
    s_rev = 0.0
    for x in w.astype(np.float64)[::-1]:
        s_rev += x
    assert s_fwd == s_rev == oracle.total(w, np.arange(len(w)), F32)[1]


# ---------------------------------------------------------- multilinear --

def dense_two_step(n, edges, keys, p):
    """The multilinear kernel and projection of Algorithm 2 over a dense adjacency matrix of keys:
    q_i = min_j f(p_i, a_ij, p_j) with f = a_ij iff p_i != p_j, then
    r_k = min{q_i : p_i = k}."""
    INF = (1 << 64) - 1
    A = [[INF] * n for _ in range(n)]
    for e, (a, b) in enumerate(edges):
        if a != b:
            A[a][b] = min(A[a][b], int(keys[e]))
            A[b][a] = min(A[b][a], int(keys[e]))
    q = [min([A[i][j] if p[i] != p[j] else INF for j in range(n)] + [INF]) for i in range(n)]
    r = [INF] * n
    for i in range(n):
        r[p[i]] = min(r[p[i]], q[i])
    return r


@pytest.mark.parametrize("seed", range(25))
def test_multilinear_matches_dense_formulation(seed):
    rng = random.Random(seed)
    n = rng.randint(1, 25)
    m = rng.randint(0, 60)
    edges, w = random_multigraph(rng, n, m, rng.choice([3, 10**9]))
    w = np.array(w, dtype=np.uint32)
    kind = seed % 3
    if kind == 0:      # arbitrary parent vector (not a forest)
        p = [rng.randrange(n) for _ in range(n)]
    elif kind == 1:    # star forest
        roots = [rng.randrange(n) for _ in range(max(1, n // 3))]
        p = [rng.choice(roots) for _ in range(n)]
        for r_ in roots:
            p[r_] = r_
    else:
        p = list(range(n))
    got = oracle.multilinear(n, edges, w, U32, p)
    want = dense_two_step(n, edges.tolist(), oracle.edge_keys(w, U32), p)
    assert [int(x) for x in got] == want


@pytest.mark.parametrize("seed", range(15))
def test_multilinear_rows_matches_dense_row_block(seed):
    """One owner's share (section 5): the dense two-step formulation over the
    block of rows A[rows, :] only (q_i = empty outside it), and the shares of
    a partition of the rows combine by minimum into the whole kernel."""
    rng = random.Random(100 + seed)
    n = rng.randint(1, 25)
    m = rng.randint(0, 60)
    edges, w = random_multigraph(rng, n, m, rng.choice([3, 10**9]))
    w = np.array(w, dtype=np.uint32)
    roots = [rng.randrange(n) for _ in range(max(1, n // 3))]
    p = [rng.choice(roots) for _ in range(n)]
    for r_ in roots:
        p[r_] = r_
    if seed % 2:
        p = [rng.randrange(n) for _ in range(n)]
    keys = oracle.edge_keys(w, U32)
    INF = (1 << 64) - 1
    # contiguous row ranges, as an owner of a row block holds them
    cuts = sorted({0, n, *[rng.randint(0, n) for _ in range(3)]})
    combined = [INF] * n
    for lo, hi in zip(cuts, cuts[1:]):
        rows = list(range(lo, hi))
        got = [int(x) for x in oracle.multilinear(n, edges, w, U32, p, rows=rows)]
        masked = np.zeros(n, bool)
        masked[lo:hi] = True
        assert got == [int(x) for x in oracle.multilinear(n, edges, w, U32, p, rows=masked)]
        A = [[INF] * n for _ in range(n)]
        for e, (a, b) in enumerate(edges.tolist()):
            if a != b:
                A[a][b] = min(A[a][b], int(keys[e]))
                A[b][a] = min(A[b][a], int(keys[e]))
        q = [min([A[i][j] if p[i] != p[j] else INF for j in range(n)] + [INF])
             if lo <= i < hi else INF for i in range(n)]
        want = [INF] * n
        for i in range(n):
            want[p[i]] = min(want[p[i]], q[i])
        assert got == want
        combined = [min(a, b) for a, b in zip(combined, got)]
    assert combined == [int(x) for x in oracle.multilinear(n, edges, w, U32, p)]
    assert all(int(x) == INF for x in oracle.multilinear(n, edges, w, U32, p, rows=[]))


# -------------------------------------------------------------- roots --

def test_find_roots_matches_pointer_doubling():
    rng = np.random.default_rng(4)
    for n in (1, 10, 1000, 100000):
        p = np.array([rng.integers(0, i + 1) for i in range(n)], dtype=np.uint32) if n < 2000 \
            else np.minimum(np.arange(n), rng.integers(0, n, n)).astype(np.uint32)
        perm = rng.permutation(n).astype(np.uint32)
        inv = np.empty_like(perm)
        inv[perm] = np.arange(n, dtype=np.uint32)
        q = perm[p[inv]]  # relabelled forest (parents no longer smaller)
        d = q.copy()
        while True:
            dd = d[d]
            if np.array_equal(dd, d):
                break
            d = dd
        assert np.array_equal(oracle.find_roots(q), d)


def test_find_roots_long_chain_and_cycles():
    n = 200000
    p = np.maximum(np.arange(n) - 1, 0).astype(np.uint32)
    assert (oracle.find_roots(p) == 0).all()
    with pytest.raises(ValueError):
        oracle.find_roots(np.array([1, 0, 2], np.uint32))  # 2-cycle
    with pytest.raises(ValueError):
        oracle.find_roots(np.array([1, 2, 0, 3], np.uint32))  # 3-cycle
    with pytest.raises(ValueError):
        oracle.find_roots(np.array([0, 5], np.uint32))


# ----------------------------------------------- Algorithm 2 by rounds --

@pytest.mark.parametrize("seed", range(12))
def test_as_rounds_equals_kruskal(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 3000))
    m = int(rng.integers(0, min(6 * n, n * (n - 1) // 2) + 1))
    e, w = gen.er(n, m, seed=50 + seed) if m else (np.zeros((0, 2), np.int32), np.zeros(0, np.uint32))
    if seed % 3 == 0:
        w = (w % 4).astype(np.uint32)
    res = oracle.as_rounds(n, e, w, U32)
    ids, cnt, tot = oracle.msf(n, e, w, U32)
    assert np.array_equal(res["ids"], ids) and res["total"] == tot
    hooks, roots = res["hooks"], res["roots"]
    # each round's hooks merge that many trees
    for k in range(len(hooks) - 1):
        assert roots[k] - roots[k + 1] == hooks[k]
    assert sum(hooks) == cnt
    # at least half of the trees with an outgoing edge hook each round,
    # so rounds that hook are at most floor(log2 n)
    assert sum(1 for h in hooks if h) <= max(0, int(math.floor(math.log2(n))))


def test_as_rounds_grid_and_rmat():
    for n, e, w, wt in [(*gen.grid(10, 10, 10, 0.05, seed=3), U32), (*gen.rmat(10, 16, seed=2), F32)]:
        res = oracle.as_rounds(n, e, w, wt)
        ids, cnt, tot = oracle.msf(n, e, w, wt)
        assert np.array_equal(res["ids"], ids) and res["total"] == tot


# ---------------------------------------------------------- generators --

def test_generators_deterministic_and_simple():
    e1, w1 = gen.er(4096, 32768, seed=1)
    e2, w2 = gen.er(4096, 32768, seed=1)
    assert np.array_equal(e1, e2) and np.array_equal(w1, w2)
    assert (e1[:, 0] < e1[:, 1]).all()
    assert len({(a, b) for a, b in e1.tolist()}) == 32768
    n, e, w = gen.rmat(14, 16, seed=2)
    assert (e[:, 0] < e[:, 1]).all()
    key = e[:, 0].astype(np.int64) * n + e[:, 1]
    assert (np.diff(key) > 0).all()
    assert w.dtype == np.float32 and (w > 0).all() and (w < 1).all()
    k = np.round(w.astype(np.float64) * 2**24)
    assert np.array_equal(k * 2.0**-24, w.astype(np.float64))


def test_grid_counts():
    assert gen.grid_full_edges(256, 256, 256) == 50135040
    n, e, w = gen.grid(6, 5, 4, 0.05, seed=3)
    M = gen.grid_full_edges(6, 5, 4)
    assert len(e) == M - int(0.05 * M)
    d = e[:, 1] - e[:, 0]
    assert set(np.unique(d).tolist()) <= {1, 6, 30}


@pytest.mark.slow
def test_grid_256_exact_edge_count():
    n, e, w = gen.workload_grid_256()
    assert n == 16777216 and len(e) == 47628288


def test_batch_sizes():
    vo, eo, e, w = gen.batch(300, seed=4)
    nn = np.diff(vo)
    assert nn.min() >= 64 and nn.max() < 65536
    assert np.array_equal(np.diff(eo), 4 * nn)
    for g in range(0, 300, 37):
        loc = e[eo[g]:eo[g + 1]]
        assert loc.min() >= 0 and loc.max() < nn[g]


# ------------------------------------------------ connected components --
# oracle.components is pinned by breadth-first search (test-local, above),
# by scipy's connected_components (a library routine of its own) and by
# closed forms: the labels must give exactly the same partition, and each
# label must be the smallest vertex of its component.

def _same_partition_min_labels(n, lab, comp):
    lab = np.asarray(lab, dtype=np.int64)
    comp = np.asarray(comp, dtype=np.int64)
    # label -> component and component -> label are both functions
    pairs = set(zip(lab.tolist(), comp.tolist()))
    assert len(pairs) == len(set(lab.tolist())) == len(set(comp.tolist()))
    # each label is the smallest vertex of its component
    smallest = {}
    for v in range(n):
        smallest.setdefault(int(comp[v]), v)
    assert all(lab[v] == smallest[int(comp[v])] for v in range(n))


@pytest.mark.parametrize("seed", range(40))
def test_components_equal_bfs_tiny(seed):
    rng = random.Random(1000 + seed)
    n = rng.randint(0, 30)
    m = rng.randint(0, 40) if n else 0
    edges = [(rng.randrange(n), rng.randrange(n)) for _ in range(m)]
    lab, cnt = oracle.components(n, np.array(edges, dtype=np.int32).reshape(-1, 2))
    c, comp = components(n, edges)
    assert cnt == c
    _same_partition_min_labels(n, lab, comp)


@pytest.mark.parametrize("kind", ["rmat", "grid", "sparse"])
def test_components_equal_scipy(kind):
    if kind == "rmat":
        n, e, _ = gen.rmat(14, 4, seed=9)
    elif kind == "grid":
        n, e, _ = gen.grid(20, 20, 20, 0.4, seed=5)
    else:
        n, m = 20000, 9000
        e, _ = gen.er(n, m, seed=8)
    lab, cnt = oracle.components(n, e)
    A = sp.coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n, n))
    c, comp = connected_components(A, directed=False)
    assert cnt == c
    # same partition: the pairs (label, scipy label) form a bijection
    pairs = np.unique(np.stack([lab.astype(np.int64), comp.astype(np.int64)]), axis=1)
    assert pairs.shape[1] == c == len(np.unique(lab))
    # labels are component minima: the smallest vertex carrying each label is that label
    first = np.full(n, -1, dtype=np.int64)
    order = np.arange(n)[::-1]
    first[lab[order]] = order
    assert np.all(first[np.unique(lab)] == np.unique(lab))


def test_components_closed_forms():
    # no edges: every vertex alone
    lab, c = oracle.components(5, np.zeros((0, 2), np.int32))
    assert c == 5 and list(lab) == [0, 1, 2, 3, 4]
    # a path in reverse order is one component labelled 0
    n = 50
    e = np.array([[i + 1, i] for i in reversed(range(n - 1))], np.int32)
    lab, c = oracle.components(n, e)
    assert c == 1 and np.all(lab == 0)
    # k disjoint copies of a triangle plus a loop: k components labelled 3j
    k = 7
    e = np.array([[3 * j + a, 3 * j + b] for j in range(k)
                  for a, b in ((0, 1), (1, 2), (2, 2))], np.int32)
    lab, c = oracle.components(3 * k, e)
    assert c == k and list(lab) == [3 * (i // 3) for i in range(3 * k)]
    with pytest.raises(ValueError):
        oracle.components(3, np.array([[0, 3]], np.int32))


def test_oracle_reproduces_stored_goldens():
    """The stored expected values under tests/golden/ (written by
    make_golden.py from this oracle) still come out of it unchanged."""
    import json
    import os
    here = os.path.join(os.path.dirname(__file__), "golden")
    cases = [("er4096_seed1.json", *gen.workload_er_4096(), U32),
             ("grid16_seed3.json", *gen.grid(16, 16, 16, 0.05, seed=3), U32),
             ("rmat12_seed2.json", *gen.rmat(12, 16, seed=2), F32)]
    for fname, n, e, w, wt in cases:
        g = json.load(open(os.path.join(here, fname)))
        ids, cnt, tot = oracle.msf(n, e, w, wt)
        assert cnt == g["count"] and int(ids.sum()) == g["id_sum"], fname
        assert (tot[0] == g["total_u64"]) if "total_u64" in g else (tot[1] == g["total_f64"])
        if "first_ids" in g:
            assert list(ids[:16]) == g["first_ids"]
        if "hooks_per_round" in g:
            assert oracle.as_rounds(n, e, w, wt)["hooks"] == g["hooks_per_round"]
