"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Bar: the forest is unique under the (weight, edge id) order, so edge ids,
count and both totals must match the oracle exactly (tolerance 0).  The
multilinear kernel and the shortcut are compared element by element with
their oracle definitions.
"""
import math
import os
import random
import sys

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U32, F32 = oracle.W_U32, oracle.W_F32
MSF_MAX_EDGES = 2 ** 31 - 2048  # include/msf.h


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_04865_amd as p
    p.lib()
    return p


@pytest.fixture(scope="module")
def ctx(pkg):
    c = pkg.Context(0)
    yield c
    c.close()


@pytest.fixture
def wide_path():
    """Keep small graphs on the device-wide round loop (tests of its
    internals: filtering, head sweep, slices, first round, builds)."""
    old = os.environ.get("MSF_SMALL_M")
    os.environ["MSF_SMALL_M"] = "0"
    yield
    if old is None:
        os.environ.pop("MSF_SMALL_M", None)
    else:
        os.environ["MSF_SMALL_M"] = old


def dev(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a.reshape(-1).copy()).to("cuda:0")


def check_solve(ctx, pkg, n, e, w, wt, label, device=True):
    say(label, f"n={n} m={len(e)} wt={wt} device={device}")
    want_ids, want_cnt, want_tot = oracle.msf(n, e, w, wt)
    if device:
        ids, cnt, tot = ctx.solve(n, dev(e), dev(w), wtype=wt)
        torch.cuda.synchronize()
        got = ids.cpu().numpy().astype(np.int64)
    else:
        got, cnt, tot = ctx.solve(n, e, w, wtype=wt)
        got = got.astype(np.int64)
    assert cnt == want_cnt, (label, cnt, want_cnt)
    assert np.array_equal(got, want_ids), label
    if wt == U32:
        assert tot[0] == want_tot[0], (label, tot, want_tot)
    assert tot[1] == want_tot[1] or (math.isnan(tot[1]) and math.isnan(want_tot[1])), \
        (label, tot, want_tot)
    return ctx.stats()


# ----------------------------------------------------------- small cases --

def test_er4096_many_seeds(ctx, pkg):
    for seed in range(1, 11):
        e, w = gen.er(4096, 32768, seed=seed)
        check_solve(ctx, pkg, 4096, e, w, U32, f"er4096 seed={seed}", device=seed % 2 == 0)


GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden_cases():
    """(file, n, e, w, wt) of every stored expected value (tests/golden/)."""
    n, e, w = gen.workload_er_4096()
    yield "er4096_seed1.json", n, e, w, U32
    n, e, w = gen.grid(16, 16, 16, 0.05, seed=3)
    yield "grid16_seed3.json", n, e, w, U32
    n, e, w = gen.rmat(12, 16, seed=2)
    yield "rmat12_seed2.json", n, e, w, F32


def test_stored_goldens(ctx, pkg):
    import json
    for fname, n, e, w, wt in golden_cases():
        g = json.load(open(os.path.join(GOLDEN, fname)))
        ids, cnt, tot = ctx.solve(n, e, w, wtype=wt)
        ids = np.asarray(ids, dtype=np.int64)
        assert cnt == g["count"], fname
        assert int(ids.sum()) == g["id_sum"], fname
        if "total_u64" in g:
            assert tot[0] == g["total_u64"], fname
        else:
            assert tot[1] == g["total_f64"], fname
        if "first_ids" in g:
            assert list(ids[:len(g["first_ids"])]) == g["first_ids"], fname
        if "hooks_per_round" in g:
            hooks = [h for h in g["hooks_per_round"] if h]
            assert ctx.stats()["hooks"][:len(hooks)] == hooks, fname


def test_tiny_random_graphs(ctx, pkg):
    rng = random.Random(7)
    for t in range(150):
        n = rng.randint(0, 40)
        m = rng.randint(0, 120) if n > 0 else 0
        e = np.array([[rng.randrange(n), rng.randrange(n)] for _ in range(m)],
                     dtype=np.int32).reshape(-1, 2)
        if t % 2:
            w = np.array([rng.randint(0, 5) for _ in range(m)], dtype=np.uint32)
            wt = U32
        else:
            w = np.array([rng.choice([-2.5, -0.0, 0.0, 1.0, 3.25, 1e-30, -1e30])
                          for _ in range(m)], dtype=np.float32)
            wt = F32
        check_solve(ctx, pkg, n, e, w, wt, f"tiny t={t}", device=(t % 3 == 0 and m > 0))


def test_ragged_sizes_span_tiles(ctx, pkg):
    # nnz around multiples of the 1024-entry sweep chunk and the 4096-edge
    # output tile, plus a long row (star) spanning many chunks
    for m in (511, 512, 513, 1023, 2047, 2049, 4095, 4097, 5000):
        n = max(64, m // 3)
        e, w = gen.er(n, m, seed=m)
        check_solve(ctx, pkg, n, e, w, U32, f"ragged m={m}")
    n = 20000
    e = np.stack([np.zeros(n - 1, np.int32), np.arange(1, n, dtype=np.int32)], 1)
    e2, _ = gen.er(n, 30000, seed=5)
    e = np.concatenate([e, e2])
    w = gen.weights(len(e), gen.W_U32, seed=9)
    check_solve(ctx, pkg, n, e, w, U32, "star+er")


def test_isolated_and_empty_rows(ctx, pkg):
    # long runs of isolated vertices between and after the used ones
    e = np.array([[0, 1], [1, 2], [2000000, 2000001], [0, 2], [2000001, 1999999]], np.int32)
    w = np.array([5, 3, 9, 1, 2], np.uint32)
    check_solve(ctx, pkg, 3000000, e, w, U32, "isolated runs")
    check_solve(ctx, pkg, 5, np.zeros((0, 2), np.int32), np.zeros(0, np.uint32), U32, "m=0",
                device=False)
    check_solve(ctx, pkg, 0, np.zeros((0, 2), np.int32), np.zeros(0, np.uint32), U32, "n=0",
                device=False)


def test_float_specials(ctx, pkg):
    e, _ = gen.er(300, 900, seed=3)
    rng = np.random.default_rng(3)
    for case in range(4):
        w = (rng.standard_normal(900) * 10.0 ** rng.integers(-30, 30, 900)).astype(np.float32)
        if case == 1:
            w[::7] = np.inf
        if case == 2:
            w[::5] = -np.inf
        if case == 3:
            w[::11] = -0.0
            w[1::11] = 0.0
        check_solve(ctx, pkg, 300, e, w, F32, f"float specials {case}")


def test_ties_and_parallel_edges(ctx, pkg):
    e, _ = gen.er(2000, 12000, seed=4)
    e = np.concatenate([e, e[::3], e[::7, ::-1]])  # parallel edges, both orientations
    w = (np.arange(len(e)) % 4).astype(np.uint32)
    check_solve(ctx, pkg, 2000, e, w, U32, "ties+parallel")
    w = np.full(len(e), 7, np.uint32)
    check_solve(ctx, pkg, 2000, e, w, U32, "all equal")


def test_forced_allocation_failure_leaves_outputs_and_context(pkg, wide_path):
    """A workspace allocation refused from the host (MSF_TEST_FAIL_ALLOC_AFTER
    = k: the allocation after k others fails once, no allocator call is
    made) at every point of a solve in turn: the call ends with MSF_ENOMEM,
    the caller's output is untouched, and the same context then solves the
    graph to the oracle's forest.  Paths: the head sweep (runs set up after
    the build) and the full sweep filtered every round (buffers taken in
    the middle of the rounds)."""
    ENOMEM = 2
    cases = [
        ("heads rmat12", {"MSF_HEADS": "2"}, *gen.rmat(12, 16, seed=61), F32),
        ("filtered grid12", {"MSF_HEADS": "0", "MSF_FILTER": "2"},
         *gen.grid(12, 12, 12, 0.05, seed=62), U32),
    ]
    for label, env, n, e, w, wt in cases:
        want_ids, want_cnt, want_tot = oracle.msf(n, e, w, wt)
        de, dw = dev(e), dev(w)
        refused = 0
        for k in range(64):
            keys = dict(env, MSF_TEST_FAIL_ALLOC_AFTER=str(k))
            old = {q: os.environ.get(q) for q in keys}
            os.environ.update(keys)
            try:
                c = pkg.Context(0)
            finally:
                for q, v in old.items():
                    if v is None:
                        os.environ.pop(q, None)
                    else:
                        os.environ[q] = v
            say("forced allocation failure", label, f"after {k}")
            out = torch.full((n,), -7, dtype=torch.int32, device="cuda:0")
            failed = False
            try:
                c.solve(n, de, dw, wtype=wt, out=out)
            except pkg.MSFError as ex:
                assert ex.status == ENOMEM, (label, k, str(ex))
                failed = True
            torch.cuda.synchronize()
            if failed:
                refused += 1
                assert bool((out == -7).all()), (label, k)
            # the hook fires once: the context solves normally afterwards
            ids, cnt, tot = c.solve(n, de, dw, wtype=wt)
            torch.cuda.synchronize()
            assert cnt == want_cnt, (label, k)
            assert np.array_equal(ids.cpu().numpy().astype(np.int64), want_ids), (label, k)
            assert tot[1] == want_tot[1], (label, k)
            c.close()
            if not failed:
                break
        else:
            pytest.fail(f"{label}: a solve still allocated after 64 refusals")
        assert refused >= 3, (label, refused)


def test_invalid_inputs_on_the_head_sweep_path(pkg, wide_path):
    """With the head sweep on, the run set-up is enqueued right after the
    build, before the host reads the build's error flags: a bad endpoint or
    a NaN weight among valid edges must still end the call with
    MSF_EINVAL, leave the output untouched, and leave the context solving
    the valid graph to the oracle's forest (the build skips invalid edges in
    every pass, so the set-up runs over a consistent adjacency)."""
    EINVAL = 1
    n, e, w = gen.rmat(11, 16, seed=63)
    old = os.environ.get("MSF_HEADS")
    os.environ["MSF_HEADS"] = "2"
    try:
        c = pkg.Context(0)
    finally:
        if old is None:
            os.environ.pop("MSF_HEADS", None)
        else:
            os.environ["MSF_HEADS"] = old
    bad_end = e.copy()
    bad_end[len(e) // 2, 1] = n
    bad_w = w.copy()
    bad_w[len(w) // 3] = np.float32(np.nan)
    for label, ee, ww in (("endpoint", bad_end, w), ("nan", e, bad_w)):
        say("invalid on the head-sweep path", label)
        out = torch.full((n,), -7, dtype=torch.int32, device="cuda:0")
        with pytest.raises(pkg.MSFError) as info:
            c.solve(n, dev(ee), dev(ww), wtype=F32, out=out)
        assert info.value.status == EINVAL, (label, str(info.value))
        torch.cuda.synchronize()
        assert bool((out == -7).all()), label
        st = check_solve(c, pkg, n, e, w, F32, f"valid after {label}")
        assert st["runs"] > 0, label
    c.close()


def test_invalid_inputs_leave_outputs_untouched(ctx, pkg):
    L = pkg.lib()
    import ctypes
    for e, w, wt, what in [
        (np.array([[0, 1], [1, 5]], np.int32), np.array([1, 2], np.uint32), U32, "endpoint"),
        (np.array([[0, 1], [-1, 0]], np.int32), np.array([1, 2], np.uint32), U32, "negative"),
        (np.array([[0, 1]], np.int32), np.array([np.nan], np.float32), F32, "nan"),
    ]:
        say("invalid", what)
        ids = np.full(4, -5, np.int32)
        cnt = ctypes.c_int64(-9)
        tot = pkg.Total(123, 4.5)
        rc = L.msf_solve(ctx._h, 3, len(w), ctypes.c_void_p(e.ctypes.data),
                         ctypes.c_void_p(w.ctypes.data), wt, 0,
                         ctypes.c_void_p(ids.ctypes.data), ctypes.byref(cnt), ctypes.byref(tot))
        assert rc == 1, what
        assert cnt.value == -9 and (ids == -5).all() and tot.u64 == 123
    with pytest.raises(pkg.MSFError):
        ctx.solve(-1, np.zeros((0, 2), np.int32), np.zeros(0, np.uint32), wtype=U32)
    # edge counts above the limit are rejected before any array is touched
    e = np.zeros((1, 2), np.int32)
    w = np.zeros(1, np.uint32)
    for m in (MSF_MAX_EDGES + 1, 2 ** 31 - 1, 2 ** 31):
        say("invalid m", m)
        ids = np.full(4, -5, np.int32)
        cnt = ctypes.c_int64(-9)
        rc = L.msf_solve(ctx._h, 3, m, ctypes.c_void_p(e.ctypes.data),
                         ctypes.c_void_p(w.ctypes.data), U32, 0,
                         ctypes.c_void_p(ids.ctypes.data), ctypes.byref(cnt), None)
        assert rc == 1 and cnt.value == -9 and (ids == -5).all(), m


# ---------------------------------------------------- per-round behaviour --

def test_rounds_match_algorithm2_oracle(ctx, pkg):
    for label, (n, e, w, wt) in {
        "er": (2000, *gen.er(2000, 8000, seed=2), U32),
        "rmat12": (*gen.rmat(12, 16, seed=2), F32),
        "grid16": (*gen.grid(16, 16, 16, 0.05, seed=3), U32),
        "grid12-40": (*gen.grid(12, 12, 12, 0.4, seed=3), U32),
    }.items():
        ref = oracle.as_rounds(n, e, w, wt)
        st = check_solve(ctx, pkg, n, e, w, wt, f"rounds {label}")
        hooks = [h for h in ref["hooks"] if h]
        assert st["hooks"][:len(hooks)] == hooks, (label, st["hooks"], hooks)
        assert st["hook_rounds"] == len(hooks)
        assert st["hook_rounds"] <= max(1, int(math.floor(math.log2(max(n, 2)))))


@pytest.mark.usefixtures("wide_path")
def test_device_driven_rounds_match(pkg):
    """Rounds driven on the device, as direct launches (1) and as replays of
    a HIP graph captured once per solve (2), give the oracle's forests and
    hooks per round, like the host-stepped loop (0); a second pass over the
    same graphs replays the cached graph, and the graphs alternate so it is
    captured again between them."""
    rng = np.random.default_rng(95)
    graphs = [("rmat14", *gen.rmat(14, 16, seed=96), F32),
              ("grid16", *gen.grid(16, 16, 16, 0.05, seed=97), U32),
              ("grid14 40% dropped", *gen.grid(14, 14, 14, 0.4, seed=98), U32),
              ("er", 20000, *gen.er(20000, 80000, seed=99), U32),
              ("path", 3000, np.array([[i, i + 1] for i in range(2999)], np.int32),
               np.arange(2999, 0, -1).astype(np.uint32), U32),
              ("multi", 300, rng.integers(0, 300, size=(5000, 2)).astype(np.int32),
               rng.integers(0, 4, size=5000).astype(np.uint32), U32)]
    want_path = {"2": 3, "1": 2, "0": 0}
    for mode in ("2", "1", "0"):
        with env_set(MSF_GRAPH_ROUNDS=mode):
            c = pkg.Context(0)
        for rep in range(2):
            for label, n, e, w, wt in graphs:
                st = check_solve(c, pkg, n, e, w, wt, f"rounds mode={mode} rep={rep} {label}",
                                 device=rep == 0)
                assert st["path"] == want_path[mode], (label, st["path"])
                hooks = [h for h in oracle.as_rounds(n, e, w, wt)["hooks"] if h]
                assert st["hooks"][:len(hooks)] == hooks, (label, st["hooks"], hooks)
        c.close()


@pytest.mark.usefixtures("wide_path")
def test_round_invariants_checked_on_device(pkg):
    """MSF_CHECK_ROUNDS=1: after every shortcut every tree is a star, and
    the roots at the start of each round (counted on the device) equal the
    oracle's Algorithm 2 run (as_rounds) round by round, so the roots drop by
    exactly the kept hooks; with the head sweep, the full sweep and every
    filtering policy."""
    graphs = [("rmat14", *gen.rmat(14, 16, seed=91), F32),
              ("grid14 40% dropped", *gen.grid(14, 14, 14, 0.4, seed=92), U32),
              ("er", 5000, *gen.er(5000, 20000, seed=93), U32),
              ("path", 3000, np.array([[i, i + 1] for i in range(2999)], np.int32),
               np.arange(2999, 0, -1).astype(np.uint32), U32)]
    for heads, filt in (("2", "1"), ("0", "0"), ("0", "2")):
        with env_set(MSF_CHECK_ROUNDS="1", MSF_HEADS=heads, MSF_FILTER=filt):
            c = pkg.Context(0)
        for label, n, e, w, wt in graphs:
            st = check_solve(c, pkg, n, e, w, wt, f"checked heads={heads} filter={filt} {label}")
            ref = oracle.as_rounds(n, e, w, wt)
            k = st["rounds"]
            assert k >= 1 and st["roots"][:k] == ref["roots"][:k], (label, st["roots"], ref["roots"])
            assert st["hooks"][:k] == ref["hooks"][:k], (label, st["hooks"], ref["hooks"])
        c.close()


@pytest.mark.usefixtures("wide_path")
def test_filter_policies_are_result_invariant(pkg):
    """The filtering policies belong to the full sweep (the head sweep passes
    internal entries over by itself), so the head sweep is off here."""
    n, e, w = gen.grid(24, 24, 24, 0.05, seed=3)
    n2, e2, w2 = gen.rmat(13, 16, seed=2)
    old = os.environ.get("MSF_FILTER")
    old_heads = os.environ.get("MSF_HEADS")
    os.environ["MSF_HEADS"] = "0"
    try:
        for mode in ("0", "1", "2"):
            os.environ["MSF_FILTER"] = mode
            c = pkg.Context(0)
            st = check_solve(c, pkg, n, e, w, U32, f"filter mode {mode} grid")
            if mode == "2":
                assert st["filtered"] >= 1
            check_solve(c, pkg, n2, e2, w2, F32, f"filter mode {mode} rmat")
            c.close()
    finally:
        if old is None:
            os.environ.pop("MSF_FILTER", None)
        else:
            os.environ["MSF_FILTER"] = old
        if old_heads is None:
            os.environ.pop("MSF_HEADS", None)
        else:
            os.environ["MSF_HEADS"] = old_heads


@pytest.mark.usefixtures("wide_path")
def test_head_sweep_matches_oracle_and_full_sweep(pkg):
    """Rounds after the first sweep key-sorted runs and pass internal
    entries over (head sweep; MSF_HEADS=2 forces it at any size) or sweep
    every entry (MSF_HEADS=0):
    both give the oracle's forest and the oracle's hook count in every round
    (so every round's minima agree).  Cases: a grid (entries turn internal
    round by round, so long internal stretches reach the per-run second
    phase), skewed R-MAT (rows of thousands of entries split into many runs),
    equal weights (order by edge id), few distinct weights and weights far
    apart beside close ones (equal sort words inside runs, settled on the full
    keys or by the 64-bit network), a multigraph with loops and repeated
    pairs, more vertices than edges, a path (one run per row, many rounds),
    and entry counts off the 64-entry chunk grid."""
    rng = np.random.default_rng(41)
    nm = 2000
    multi_e = rng.integers(0, nm, size=(15000, 2)).astype(np.int32)
    multi_w = rng.integers(0, 20, size=15000).astype(np.uint32)
    npath = 3001
    path_e = np.stack([np.arange(npath - 1), np.arange(1, npath)], 1).astype(np.int32)
    path_w = rng.permutation(npath - 1).astype(np.uint32)
    eq_e, _ = gen.er(3000, 20000, seed=43)
    eq_w = np.full(len(eq_e), 7, dtype=np.uint32)
    # few distinct weights (equal keys inside runs, ordered by edge id) and
    # weights far apart next to weights close together (the chunk sort's
    # 32-bit words drop the low bits, so distinct keys share words)
    fw_n, fw_e, _ = gen.rmat(15, 16, seed=48)
    fw_w = rng.integers(0, 4096, size=len(fw_e)).astype(np.uint32)
    mg_n, mg_e, _ = gen.rmat(14, 16, seed=49)
    mg_w = ((rng.integers(0, 4, size=len(mg_e)) << 30) |
            rng.integers(0, 128, size=len(mg_e))).astype(np.uint32)
    graphs = [
        ("rmat15 few weights", fw_n, fw_e, fw_w, U32),
        ("rmat14 split weights", mg_n, mg_e, mg_w, U32),
        ("grid20", *gen.grid(20, 20, 20, 0.05, seed=42), U32),
        ("rmat15", *gen.rmat(15, 16, seed=44), F32),
        ("equal weights", 3000, eq_e, eq_w, U32),
        ("multi", nm, multi_e, multi_w, U32),
        ("sparse", 40000, *gen.er(40000, 15000, seed=45), U32),
        ("path", npath, path_e, path_w, U32),
        ("ragged 37", 40, *gen.er(40, 37, seed=46), U32),
        ("ragged 1000", 300, *gen.er(300, 1000, seed=47, wtype=F32), F32),
    ]
    old = os.environ.get("MSF_HEADS")
    try:
        for heads in ("2", "0"):
            os.environ["MSF_HEADS"] = heads
            c = pkg.Context(0)
            for label, n, e, w, wt in graphs:
                st = check_solve(c, pkg, n, e, w, wt, f"heads={heads} {label}")
                ref = oracle.as_rounds(n, e, w, wt)
                hooks = [h for h in ref["hooks"] if h]
                assert st["hooks"][:len(hooks)] == hooks, (label, st["hooks"], hooks)
                if heads == "2":
                    assert st["runs"] > 0, label
                    assert st["head_sweeps"] in (st["rounds"], max(st["rounds"] - 1, 0)), \
                        (label, st["rounds"], st["head_sweeps"])
                else:
                    assert st["runs"] == 0 and st["head_sweeps"] == 0, label
            c.close()
    finally:
        if old is None:
            os.environ.pop("MSF_HEADS", None)
        else:
            os.environ["MSF_HEADS"] = old


# ---------------------------------------------------------- multilinear --

def multilinear_case(ctx, pkg, n, e, w, wt, p, label):
    say("multilinear", label, f"n={n} m={len(e)}")
    g = pkg.Graph(ctx, n, e, w, wtype=wt)
    dp = dev(np.asarray(p, np.uint32))
    dr = torch.empty(max(n, 1), dtype=torch.int64, device="cuda:0")
    ctx.multilinear(g, dp, dr)
    torch.cuda.synchronize()
    got = dr.cpu().numpy()[:n].view(np.uint64)
    want = oracle.multilinear(n, e, w, wt, p)
    assert np.array_equal(got, want), label
    # the pairwise formulation (pairs stored, then reduced) gives the same r
    dr2 = torch.empty(max(n, 1), dtype=torch.int64, device="cuda:0")
    ctx.multilinear_pairwise(g, dp, dr2)
    torch.cuda.synchronize()
    assert np.array_equal(dr2.cpu().numpy()[:n].view(np.uint64), want), label + " pairwise"
    g.close()


def hub_graph(n, hubs, seed):
    """A few hubs joined to every vertex, plus a sparse random graph: most
    stored entries lie in rows longer than one wave of the sweep (the kernel
    then reuses the value of r it read before gathering)."""
    e2, _ = gen.er(n, 2 * n, seed=seed)
    hub = np.stack([np.repeat(np.arange(hubs, dtype=np.int32), n - hubs),
                    np.tile(np.arange(hubs, n, dtype=np.int32), hubs)], 1)
    e = np.concatenate([hub, e2])
    return e, gen.weights(len(e), gen.W_U32, seed=seed + 1)


def test_multilinear_matches_definition(ctx, pkg):
    rng = np.random.default_rng(1)
    for label, (n, e, w, wt) in {
        "er4096": (4096, *gen.er(4096, 32768, seed=1), U32),
        "rmat14": (*gen.rmat(14, 16, seed=2), F32),
        "grid20": (*gen.grid(20, 20, 20, 0.05, seed=3), U32),
        "ragged": (3001, *gen.er(3001, 7777, seed=8), U32),
        "hubs": (5000, *hub_graph(5000, 6, seed=9), U32),
    }.items():
        ident = np.arange(n, dtype=np.uint32)
        multilinear_case(ctx, pkg, n, e, w, wt, ident, label + " identity")
        roots = rng.choice(n, size=max(1, n // 50), replace=False).astype(np.uint32)
        star = roots[rng.integers(0, len(roots), n)]
        star[roots] = roots
        multilinear_case(ctx, pkg, n, e, w, wt, star, label + " stars")
        arb = rng.integers(0, n, n).astype(np.uint32)
        multilinear_case(ctx, pkg, n, e, w, wt, arb, label + " arbitrary")
        sorted_blocks = (np.arange(n) // 7 * 7).astype(np.uint32)  # runs of equal roots
        multilinear_case(ctx, pkg, n, e, w, wt, sorted_blocks, label + " blocks")


def stored_row_cuts(n, e, order, parts):
    """Cut positions of `parts` contiguous stored-row ranges balanced by
    stored entries (both directions of every non-loop edge)."""
    e = np.asarray(e, np.int64)
    keep = e[:, 0] != e[:, 1]
    deg = np.bincount(e[keep].reshape(-1), minlength=n)
    pre = np.concatenate([[0], np.cumsum(deg[order])])
    tot = int(pre[-1])
    cuts = [0] + [int(np.searchsorted(pre, tot * k // parts, side="left")) for k in range(1, parts)]
    return sorted(set(cuts + [n]))


def test_multilinear_rows_shares(ctx, pkg):
    """One owner's share of the multilinear kernel (rows of A split among
    owners that all hold p, section 5): each share equals the oracle's
    kernel over those rows, and the shares combine by minimum into the
    whole kernel.  Ranges balanced by entries, plus empty, one-row and
    whole ranges; both stored orders."""
    rng = np.random.default_rng(91)
    graphs = [("rmat14", *gen.rmat(14, 16, seed=92), F32),
              ("grid18", *gen.grid(18, 18, 18, 0.05, seed=93), U32),
              ("er ragged", 3001, *gen.er(3001, 7777, seed=94), U32)]
    for order_env in ("1", "0"):
        with env_set(MSF_GRAPH_ORDER=order_env):
            c = pkg.Context(0)
        for label, n, e, w, wt in graphs:
            g = pkg.Graph(c, n, e, w, wtype=wt)
            od = torch.empty(n, dtype=torch.int32, device="cuda:0")
            c.graph_order(g, od)
            order = od.cpu().numpy().astype(np.int64)
            assert np.array_equal(np.sort(order), np.arange(n)), label
            if order_env == "0":
                assert np.array_equal(order, np.arange(n)), label
            roots = rng.choice(n, size=max(1, n // 40), replace=False).astype(np.uint32)
            star = roots[rng.integers(0, len(roots), n)]
            star[roots] = roots
            whole = oracle.multilinear(n, e, w, wt, star)
            cuts = stored_row_cuts(n, e, order, 8)
            ranges = list(zip(cuts, cuts[1:])) + [(0, 0), (n // 2, n // 2 + 1), (0, n)]
            dr = torch.empty(n, dtype=torch.int64, device="cuda:0")
            comb = np.full(n, np.iinfo(np.uint64).max, np.uint64)
            for lo, hi in ranges:
                say("multilinear rows", label, f"order={order_env} rows [{lo}, {hi})")
                dr.fill_(0)
                c.multilinear_rows(g, dev(star), dr, lo, hi)
                torch.cuda.synchronize()
                got = dr.cpu().numpy().view(np.uint64)
                want = oracle.multilinear(n, e, w, wt, star, rows=order[lo:hi])
                assert np.array_equal(got, want), (label, lo, hi)
                if (lo, hi) in list(zip(cuts, cuts[1:])):
                    comb = np.minimum(comb, got)
            assert np.array_equal(comb, whole), label
            for lo, hi in ((1, 0), (-1, 3), (0, n + 1)):
                with pytest.raises(pkg.MSFError):
                    c.multilinear_rows(g, dev(star), dr, lo, hi)
            g.close()
        c.close()


def test_kernels_after_device_driven_rounds(pkg):
    """A solve whose rounds ran on the device (and components on such a
    path) leave nothing behind that the next call on the context sees: the
    multilinear kernel, both forms, on a graph made before them."""
    with env_set(MSF_SMALL_M="0", MSF_HEADS="0"):
        c = pkg.Context(0)
    n = 4096
    e, w = gen.er(n, 32768, seed=97)
    g = pkg.Graph(c, n, e, w, wtype=U32)
    rng = np.random.default_rng(98)
    roots = rng.choice(n, size=60, replace=False).astype(np.uint32)
    star = roots[rng.integers(0, len(roots), n)]
    star[roots] = roots
    want = oracle.multilinear(n, e, w, U32, star)
    dr = torch.empty(n, dtype=torch.int64, device="cuda:0")
    lab = torch.empty(n, dtype=torch.int32, device="cuda:0")
    for step in ("solve", "components"):
        if step == "solve":
            st = check_solve(c, pkg, n, e, w, U32, "device-driven rounds")
            assert st["path"] == 3, st["path"]
        else:
            c.components(g, lab)
        for form in (c.multilinear, c.multilinear_pairwise):
            dr.fill_(0)
            form(g, dev(star), dr)
            torch.cuda.synchronize()
            assert np.array_equal(dr.cpu().numpy().view(np.uint64), want), (step, form)
    g.close()
    c.close()


def test_context_close_releases_its_graphs(pkg):
    """Closing a context first releases the graphs made on it, so a graph
    object that outlives its context is inert (msf_graph_destroy needs the
    context's stream)."""
    c = pkg.Context(0)
    e, w = gen.er(500, 2000, seed=96)
    g = pkg.Graph(c, 500, e, w, wtype=U32)
    c.close()
    assert g._h is None
    g.close()
    del g
    c2 = pkg.Context(0)
    g2 = pkg.Graph(c2, 500, e, w, wtype=U32)
    lab = torch.empty(500, dtype=torch.int32, device="cuda:0")
    c2.components(g2, lab)
    g2.close()
    c2.close()


def kernel_at(n, e, w, wt, p, sample, rows=None):
    """The oracle's kernel at the roots in `sample` only: over the edges with
    an end in one of their trees (the only edges that can reach them), with
    each key's edge id mapped back from the sub-list to the whole list."""
    INF = np.iinfo(np.uint64).max
    in_s = np.isin(p, sample)
    sel = in_s[e[:, 0]] | in_s[e[:, 1]]
    ids = np.nonzero(sel)[0]
    if len(ids) == 0:
        return np.full(len(sample), INF, np.uint64)
    want = oracle.multilinear(n, e[sel], w[sel], wt, p, rows=rows)[sample]
    low = (want & np.uint64(0xFFFFFFFF)).astype(np.int64)
    mapped = ids[np.minimum(low, len(ids) - 1)].astype(np.uint64)
    return np.where(want == INF, want, (want & ~np.uint64(0xFFFFFFFF)) | mapped)


def test_multilinear_rows_full_size(ctx, pkg):
    """R-MAT s22 cut into 8 entry-balanced stored-row ranges, p = the
    parents after round 1 of the solve (its hooks and tie break, shortcut):
    the shares combine by minimum into the whole kernel's r, no share is
    below it, and sampled roots match the oracle's kernel over their rows."""
    n, e, w, wt, _ = full_case("rmat s22")
    say("multilinear rows", "rmat s22", f"n={n} m={len(e)}")
    g = pkg.Graph(ctx, n, dev(e), dev(w), wtype=wt)
    od = torch.empty(n, dtype=torch.int32, device="cuda:0")
    ctx.graph_order(g, od)
    order = od.cpu().numpy().astype(np.int64)
    # round-1 parents from the oracle's first round: each vertex's minimum
    # edge hooks it (identity p), the smaller of a mutual pair stays root,
    # then the roots of that forest
    r1 = oracle.multilinear(n, e, w, wt, np.arange(n, dtype=np.uint32))
    h = np.arange(n, dtype=np.int64)
    has = r1 != np.iinfo(np.uint64).max
    eid = (r1[has] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    v = np.nonzero(has)[0]
    a, b = e[eid, 0].astype(np.int64), e[eid, 1].astype(np.int64)
    h[v] = np.where(a == v, b, a)
    mutual = has & (h[h] == np.arange(n)) & (np.arange(n) < h)
    h[mutual] = np.nonzero(mutual)[0]
    p = oracle.find_roots(h.astype(np.uint32))
    dp = dev(p)
    dr = torch.empty(n, dtype=torch.int64, device="cuda:0")
    ctx.multilinear(g, dp, dr)
    torch.cuda.synchronize()
    whole = dr.cpu().numpy().view(np.uint64).copy()
    comb = np.full(n, np.iinfo(np.uint64).max, np.uint64)
    cuts = stored_row_cuts(n, e, order, 8)
    rng = np.random.default_rng(95)
    # roots of trees with edges (isolated vertices are roots of their own)
    cand = np.unique(p[np.bincount(e.reshape(-1), minlength=n) > 0])
    for lo, hi in zip(cuts, cuts[1:]):
        ctx.multilinear_rows(g, dp, dr, lo, hi)
        torch.cuda.synchronize()
        got = dr.cpu().numpy().view(np.uint64).copy()
        assert np.all(got >= whole), (lo, hi)
        comb = np.minimum(comb, got)
        rows = np.zeros(n, bool)
        rows[order[lo:hi]] = True
        sample = rng.choice(cand, size=20, replace=False)
        assert np.array_equal(got[sample], kernel_at(n, e, w, wt, p, sample, rows)), (lo, hi)
    assert np.array_equal(comb, whole)
    # the whole kernel itself, at sampled roots
    sample = rng.choice(cand, size=50, replace=False)
    assert np.array_equal(whole[sample], kernel_at(n, e, w, wt, p, sample))
    g.close()


def test_graph_vertex_order_is_invisible(pkg):
    """Kept graphs store their vertices by decreasing degree class
    (MSF_GRAPH_ORDER=1, the default) or in the caller's order (0): the
    multilinear kernel (both forms), components and the original AS rounds
    give identical results either way."""
    graphs = [("rmat14", *gen.rmat(14, 16, seed=81), F32),
              ("grid10", *gen.grid(10, 10, 10, 0.2, seed=82), U32),
              ("er", 3000, *gen.er(3000, 9000, seed=83), U32)]
    for order in ("1", "0"):
        with env_set(MSF_GRAPH_ORDER=order):
            c = pkg.Context(0)
        res = []
        for label, n, e, w, wt in graphs:
            res.append((label, n, e, w, wt, pkg.Graph(c, n, e, w, wtype=wt)))
        for label, n, e, w, wt, g in res:
            r = torch.empty(n, dtype=torch.int64, device="cuda:0")
            rs = np.random.default_rng(85)
            roots = rs.choice(n, size=max(1, n // 9), replace=False).astype(np.uint32)
            star = roots[rs.integers(0, len(roots), n)]
            star[roots] = roots
            c.multilinear(g, dev(star), r)
            torch.cuda.synchronize()
            r1 = r.cpu().numpy().view(np.uint64).copy()
            assert np.array_equal(r1, oracle.multilinear(n, e, w, wt, star)), (order, label)
            r.fill_(0)
            c.multilinear_pairwise(g, dev(star), r)
            torch.cuda.synchronize()
            assert np.array_equal(r.cpu().numpy().view(np.uint64), r1), (order, label)
            lab = torch.empty(n, dtype=torch.int32, device="cuda:0")
            c.components(g, lab)
            flags = torch.empty(len(e), dtype=torch.uint8, device="cuda:0")
            c.solve_starcheck(g, flags)
            torch.cuda.synchronize()
            got = lab.cpu().numpy().view(np.uint32).astype(np.int64)
            want, ncomp = oracle.components(n, e)
            assert np.array_equal(got[got], got) and np.array_equal(got, got[want]), (order, label)
            assert len(np.unique(got)) == ncomp, (order, label)
            ids = np.nonzero(flags.cpu().numpy())[0]
            assert np.array_equal(ids, oracle.msf(n, e, w, wt)[0]), (order, label)
            g.close()
        c.close()


def test_multilinear_rejects_bad_parent(ctx, pkg):
    n, e, w = 100, *gen.er(100, 300, seed=1)
    g = pkg.Graph(ctx, n, e, w, wtype=U32)
    p = np.arange(n, dtype=np.uint32)
    p[5] = 1000
    dr = torch.zeros(n, dtype=torch.int64, device="cuda:0")
    with pytest.raises(pkg.MSFError):
        ctx.multilinear(g, dev(p), dr)
    with pytest.raises(pkg.MSFError):
        ctx.multilinear_pairwise(g, dev(p), dr)
    torch.cuda.synchronize()
    assert (dr.cpu().numpy() == 0).all()
    g.close()


# ------------------------------------------------------------- shortcut --

def test_shortcut_matches_find_roots(ctx, pkg):
    rng = np.random.default_rng(2)
    for n in (1, 2, 1000, 65537, 1 << 20):
        par = np.minimum(np.arange(n), rng.integers(0, n, n)).astype(np.uint32)
        perm = rng.permutation(n).astype(np.uint32)
        inv = np.empty_like(perm)
        inv[perm] = np.arange(n, dtype=np.uint32)
        p = perm[par[inv]]
        say("shortcut", n)
        dp = dev(p)
        passes = ctx.shortcut(dp)
        torch.cuda.synchronize()
        got = dp.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, oracle.find_roots(p)), n
        assert passes <= max(1, math.ceil(math.log2(max(n, 2)))) + 1
    # a long chain: depth n-1
    n = 1 << 18
    p = np.maximum(np.arange(n) - 1, 0).astype(np.uint32)[rng.permutation(n)]
    p = np.arange(n, dtype=np.uint32)
    order = rng.permutation(n)
    p[order[1:]] = order[:-1]
    say("shortcut chain", n)
    dp = dev(p)
    ctx.shortcut(dp)
    torch.cuda.synchronize()
    assert np.array_equal(dp.cpu().numpy().view(np.uint32), oracle.find_roots(p))


def test_shortcut_rejects_cycles(ctx, pkg):
    for p in ([1, 0, 2], [1, 2, 0, 3], [0, 2, 3, 1, 4, 4], [0, 7]):
        say("shortcut cycle", p)
        p = np.array(p, np.uint32)
        dp = dev(p)
        with pytest.raises(pkg.MSFError):
            ctx.shortcut(dp)
        torch.cuda.synchronize()
        assert np.array_equal(dp.cpu().numpy().view(np.uint32), p)  # untouched


def test_shortcut_strategies_match_find_roots(ctx, pkg):
    """Full passes, the frontier and the switch between them give the same roots."""
    rng = np.random.default_rng(5)
    cases = []
    for n in (1, 2, 1000, 65537, 1 << 20):
        par = np.minimum(np.arange(n), rng.integers(0, n, n)).astype(np.uint32)
        perm = rng.permutation(n).astype(np.uint32)
        inv = np.empty_like(perm)
        inv[perm] = np.arange(n, dtype=np.uint32)
        cases.append((f"random forest n={n}", perm[par[inv]]))
    n = 1 << 18
    p = np.arange(n, dtype=np.uint32)
    order = rng.permutation(n)
    p[order[1:]] = order[:-1]
    cases.append(("chain", p))
    strategies = [("frontier", pkg.SHORTCUT_FRONTIER, 0.0), ("full", pkg.SHORTCUT_FULL, 0.0),
                  ("switch 0", pkg.SHORTCUT_SWITCH, 0.0),
                  ("switch .25", pkg.SHORTCUT_SWITCH, 0.25),
                  ("switch 1", pkg.SHORTCUT_SWITCH, 1.0)]
    for label, p in cases:
        want = oracle.find_roots(p)
        cap = max(1, math.ceil(math.log2(max(len(p), 2)))) + 1
        for sname, st, frac in strategies:
            say("shortcut strategy", sname, label)
            dp = dev(p)
            passes = ctx.shortcut_strategy(dp, st, frac)
            torch.cuda.synchronize()
            assert np.array_equal(dp.cpu().numpy().view(np.uint32), want), (sname, label)
            assert passes <= cap, (sname, label, passes)
    for bad in ([1, 0, 2], [1, 2, 0, 3], [0, 2, 3, 1, 4, 4]):
        p = np.array(bad, np.uint32)
        for sname, st, frac in strategies:
            say("shortcut strategy cycle", sname, bad)
            dp = dev(p)
            with pytest.raises(pkg.MSFError):
                ctx.shortcut_strategy(dp, st, frac)
            torch.cuda.synchronize()
            assert np.array_equal(dp.cpu().numpy().view(np.uint32), p)
    dp = dev(np.array([0, 0, 1], np.uint32))
    for st, frac in ((7, 0.0), (pkg.SHORTCUT_SWITCH, 1.5), (pkg.SHORTCUT_SWITCH, float("nan"))):
        with pytest.raises(pkg.MSFError):
            ctx.shortcut_strategy(dp, st, frac)
    torch.cuda.synchronize()
    assert np.array_equal(dp.cpu().numpy().view(np.uint32), [0, 0, 1])


# ------------------------------------------------- one-workgroup solves --

def test_small_graphs_take_one_workgroup(ctx, pkg):
    """msf_solve of small graphs runs in one workgroup (state in LDS); the
    same graphs on the device-wide round loop give the same forests, and
    both equal the oracle's, with the oracle's hooks per round."""
    rng = np.random.default_rng(61)
    cases = [("er4096", 4096, *gen.er(4096, 32768, seed=3), U32),
             ("rmat12", *gen.rmat(12, 16, seed=4), F32),
             ("grid16", *gen.grid(16, 16, 16, 0.05, seed=5), U32),
             ("path", 3000, np.array([[i, i + 1] for i in range(2999)], np.int32),
              np.full(2999, 5, np.uint32), U32),
             ("multi", 300, rng.integers(0, 300, size=(5000, 2)).astype(np.int32),
              rng.integers(0, 4, size=5000).astype(np.uint32), U32),
             ("two vertices", 2, np.array([[0, 1], [1, 0], [0, 0]], np.int32),
              np.array([3, 3, 1], np.uint32), U32),
             ("limit", 7000, *gen.er(7000, 50000, seed=6), U32)]
    for label, n, e, w, wt in cases:
        st = check_solve(ctx, pkg, n, e, w, wt, "small " + label, device=len(e) % 2 == 0)
        assert st["path"] == 1, (label, st)
        hooks = [h for h in oracle.as_rounds(n, e, w, wt)["hooks"] if h]
        assert st["hooks"][:len(hooks)] == hooks, (label, st["hooks"], hooks)
    with env_set(MSF_SMALL_M="0"):
        c = pkg.Context(0)
    for label, n, e, w, wt in cases:
        st = check_solve(c, pkg, n, e, w, wt, "wide " + label)
        # the device-driven rounds, replayed from a captured graph
        assert st["path"] == 3, (label, st["path"])
        hooks = [h for h in oracle.as_rounds(n, e, w, wt)["hooks"] if h]
        assert st["hooks"][:len(hooks)] == hooks, (label, st["hooks"], hooks)
    c.close()


def test_small_path_rejects_bad_input_untouched(ctx, pkg):
    n = 100
    e = np.array([[0, 1], [1, 2], [2, 100]], np.int32)  # 100 is out of range
    w = np.array([1.0, 2.0, 3.0], np.float32)
    out = torch.full((n,), -5, dtype=torch.int32, device="cuda:0")
    with pytest.raises(pkg.MSFError) as ex:
        ctx.solve(n, dev(e), dev(w), wtype=F32, out=out)
    assert ex.value.status == 1
    e[2, 1] = 3
    w[1] = np.nan
    with pytest.raises(pkg.MSFError) as ex:
        ctx.solve(n, dev(e), dev(w), wtype=F32, out=out)
    assert ex.value.status == 1
    torch.cuda.synchronize()
    assert bool((out == -5).all())


# ------------------------------------------------------------ components --

def test_components_match_oracle(ctx, pkg):
    """Connectivity variant: the partition equals the oracle's components
    (union-find; the oracle is itself pinned against BFS and scipy)."""
    cases = {
        "er4096": (4096, *gen.er(4096, 32768, seed=1)),
        "sparse many components": (20000, *gen.er(20000, 9000, seed=3)),
        "rmat14": (*gen.rmat(14, 16, seed=2, wtype=U32),),
        "grid20": (*gen.grid(20, 20, 20, 0.3, seed=3),),
        "isolated runs": (3000000, np.array([[0, 1], [1, 2], [2000000, 2000001], [0, 2],
                                             [2000001, 1999999]], np.int32),
                          np.array([5, 3, 9, 1, 2], np.uint32)),
        "one vertex": (1, np.zeros((0, 2), np.int32), np.zeros(0, np.uint32)),
        "loops and parallel edges": (5, np.array([[0, 0], [1, 2], [2, 1], [3, 3], [1, 2]],
                                                 np.int32), np.array([1, 1, 1, 1, 1], np.uint32)),
    }
    # the default choice; the solve's rounds with the head sweep for every
    # graph (MSF_HEADS=2); the device-driven rounds for every graph up to
    # 2^20 vertices (MSF_HEADS=0); the solve's rounds with the full sweep
    # (MSF_HEADS=0, MSF_GRAPH_ROUNDS=0); kept graphs in degree order and in
    # the caller's order
    for heads, order, gr in (("1", "1", "2"), ("2", "1", "2"), ("0", "1", "2"), ("2", "0", "2"),
                             ("0", "1", "0"), ("0", "0", "0")):
        with env_set(MSF_HEADS=heads, MSF_GRAPH_ORDER=order, MSF_GRAPH_ROUNDS=gr):
            c = pkg.Context(0)
        try:
            for label, (n, e, w) in cases.items():
                check_components(c, pkg, n, e, w,
                                 f"heads={heads} order={order} graph_rounds={gr} {label}")
        finally:
            c.close()


def check_components(c, pkg, n, e, w, label):
    say("components", label, f"n={n} m={len(e)}")
    g = pkg.Graph(c, n, e, w, wtype=U32)
    lab = torch.empty(max(n, 1), dtype=torch.int32, device="cuda:0")
    rounds = c.components(g, lab)
    torch.cuda.synchronize()
    got = lab.cpu().numpy()[:n].view(np.uint32).astype(np.int64)
    want, ncomp = oracle.components(n, e)
    want = want.astype(np.int64)
    # the same partition: labels are roots of their own component, and
    # the oracle's label (the component's smallest vertex) maps one-to-one
    # onto the GPU's labels
    assert (got < n).all() and np.array_equal(got[got], got), label
    assert np.array_equal(got, got[want]), label
    assert len(np.unique(got)) == ncomp, label
    assert rounds <= max(1, math.ceil(math.log2(max(n, 2)))) + 1, (label, rounds)
    # the graph is only read: the kernel on it still gives the oracle's r
    if 0 < n <= 100000 and len(e):
        dr = torch.empty(n, dtype=torch.int64, device="cuda:0")
        c.multilinear(g, dev(np.arange(n, dtype=np.uint32)), dr)
        torch.cuda.synchronize()
        assert np.array_equal(dr.cpu().numpy().view(np.uint64),
                              oracle.multilinear(n, e, w, U32, np.arange(n))), label
    g.close()
    return rounds


@pytest.mark.parametrize("label", ["rmat s22", "grid 256"])
def test_components_full_size(ctx, pkg, label):
    """msf_components on the full workloads (head-sweep rounds on R-MAT s22,
    device-driven rounds on the grid) against the oracle's components."""
    n, e, w, wt, _ = full_case(label)
    if wt == F32:
        w = w.view(np.uint32)  # any weights: components do not depend on them
    rounds = check_components(ctx, pkg, n, e, w, label)
    st = ctx.stats()
    if label == "rmat s22":
        assert st["head_sweeps"] == st["rounds"] and rounds == st["hook_rounds"], st


def test_starcheck_rounds_give_the_msf(ctx, pkg):
    """Original AS rounds (star check, one-step shortcut): the oracle's forest."""
    cases = {
        "er4096": (4096, *gen.er(4096, 32768, seed=1), U32),
        "rmat14": (*gen.rmat(14, 16, seed=2), F32),
        "grid20": (*gen.grid(20, 20, 20, 0.05, seed=3), U32),
        "sparse": (20000, *gen.er(20000, 9000, seed=3), U32),
        "equal weights": (3000, gen.er(3000, 12000, seed=9)[0], np.ones(12000, np.uint32), U32),
        "loops and parallel": (5, np.array([[0, 0], [1, 2], [2, 1], [3, 3], [1, 2], [4, 1]],
                                           np.int32), np.array([1, 7, 7, 1, 3, 2], np.uint32),
                               U32),
        "no edges": (7, np.zeros((0, 2), np.int32), np.zeros(0, np.uint32), U32),
    }
    for label, (n, e, w, wt) in cases.items():
        say("starcheck", label, f"n={n} m={len(e)}")
        g = pkg.Graph(ctx, n, e, w, wtype=wt)
        flags = torch.full((max(len(e), 1),), 9, dtype=torch.uint8, device="cuda:0")
        rounds = ctx.solve_starcheck(g, flags)
        torch.cuda.synchronize()
        g.close()
        got = np.nonzero(flags.cpu().numpy()[:len(e)])[0]
        ids, cnt, _ = oracle.msf(n, e, w, wt)
        assert np.array_equal(got, np.asarray(ids, np.int64)), label
        assert len(got) == cnt, label
        assert (len(e) == 0) == (rounds == 0), (label, rounds)


# --------------------------------------------------------------- batched --

def test_batched_equals_oracle_per_graph(ctx, pkg):
    vo, eo, e, w = gen.batch(200, seed=4)
    say("batched 200 graphs", int(vo[-1]), int(eo[-1]))
    ids, counts, totals = ctx.solve_batched(vo, eo, e, w, wtype=U32)
    for g in range(200):
        n = int(vo[g + 1] - vo[g])
        ee, ww = e[eo[g]:eo[g + 1]], w[eo[g]:eo[g + 1]]
        wi, wc, wtot = oracle.msf(n, ee, ww, U32)
        assert counts[g] == wc, g
        assert np.array_equal(ids[vo[g]:vo[g] + wc].astype(np.int64), wi), g
        assert totals[g][0] == wtot[0] and totals[g][1] == wtot[1], g


def test_batched_device_float_and_solo_agree(ctx, pkg):
    vo, eo, e, _ = gen.batch(64, seed=6, lo=16, hi=3000)
    w = gen.weights(len(e), gen.W_F32, seed=6)
    w[::13] = -w[::13]
    say("batched device f32", int(vo[-1]), int(eo[-1]))
    ids, counts, totals = ctx.solve_batched(vo, eo, dev(e), dev(w), wtype=F32)
    torch.cuda.synchronize()
    ids = ids.cpu().numpy()
    for g in range(64):
        n = int(vo[g + 1] - vo[g])
        ee, ww = e[eo[g]:eo[g + 1]], w[eo[g]:eo[g + 1]]
        si, sc, stot = ctx.solve(n, ee, ww, wtype=F32)
        wi, wc, wtot = oracle.msf(n, ee, ww, F32)
        assert sc == wc == counts[g], g
        assert np.array_equal(si.astype(np.int64), wi)
        assert np.array_equal(ids[vo[g]:vo[g] + wc].astype(np.int64), wi)
        assert totals[g][1] == stot[1] == wtot[1]


def mixed_batch(seed=41):
    """Graphs of every kind the batched solve meets: empty, single vertex,
    loops and parallel edges, tiny and large ones (state in LDS and in the
    global slot for every candidate), a path, equal weights, float specials."""
    rng = np.random.default_rng(seed)
    graphs = [(0, np.zeros((0, 2), np.int32)), (1, np.zeros((0, 2), np.int32)),
              (5, np.array([[0, 0], [1, 2], [2, 1], [3, 3], [1, 2], [4, 0]], np.int32)),
              (3000, np.array([[i, i + 1] for i in range(2999)], np.int32))]
    for n in list(rng.integers(2, 200, 40)) + list(rng.integers(200, 6000, 20)) + \
            [9000, 17000, 33000, 65536]:
        n = int(n)
        m = int(rng.integers(0, 5 * n))
        graphs.append((n, rng.integers(0, n, size=(m, 2)).astype(np.int32)))
    vo = np.zeros(len(graphs) + 1, np.int64)
    eo = np.zeros(len(graphs) + 1, np.int64)
    for g, (n, e) in enumerate(graphs):
        vo[g + 1] = vo[g] + n
        eo[g + 1] = eo[g] + len(e)
    e = np.concatenate([x[1] for x in graphs]).astype(np.int32)
    w_u = rng.integers(0, 1 << 32, size=len(e), dtype=np.uint64).astype(np.uint32)
    w_u[eo[3]:eo[4]] = 7  # the path: equal weights
    w_f = (rng.integers(1, 1 << 24, size=len(e)) * 2.0 ** -24).astype(np.float32)
    w_f[::17] = -w_f[::17]
    w_f[5] = np.inf
    w_f[6] = -0.0
    return vo, eo, e, w_u, w_f


def check_batched(ctx, vo, eo, e, w, wt, label, device=False):
    G = len(vo) - 1
    if device:
        ids, counts, totals = ctx.solve_batched(vo, eo, dev(e), dev(w), wtype=wt)
        torch.cuda.synchronize()
        ids = ids.cpu().numpy()
    else:
        ids, counts, totals = ctx.solve_batched(vo, eo, e, w, wtype=wt)
    for g in range(G):
        n = int(vo[g + 1] - vo[g])
        wi, wc, wtot = oracle.msf(n, e[eo[g]:eo[g + 1]], w[eo[g]:eo[g + 1]], wt)
        assert counts[g] == wc, (label, g)
        assert np.array_equal(ids[vo[g]:vo[g] + wc].astype(np.int64), wi), (label, g)
        assert totals[g][1] == wtot[1] or (math.isnan(totals[g][1]) and math.isnan(wtot[1])), \
            (label, g, totals[g], wtot)
        if wt == U32:
            assert totals[g][0] == wtot[0], (label, g)
    return ctx.stats()


def test_batched_every_candidate_is_result_invariant(ctx, pkg):
    """Every launch configuration of the persistent batched kernel gives the
    oracle's forests (the tuner's choice cannot change a result)."""
    vo, eo, e, w_u, w_f = mixed_batch()
    cands = pkg.batch_configs()
    with env_set(MSF_BATCH_CONFIG="0"):
        for i, cfg in enumerate(cands):
            os.environ["MSF_BATCH_CONFIG"] = str(i)
            say("batched candidate", i, cfg)
            st = check_batched(ctx, vo, eo, e, w_u, U32, f"cand {i} u32", device=i % 2 == 0)
            assert st["batch_config"] == i and st["batch_graphs"] == len(vo) - 1, st
            check_batched(ctx, vo, eo, e, w_f, F32, f"cand {i} f32", device=i % 2 == 1)


def test_batched_large_graphs_go_one_by_one(ctx, pkg):
    """Graphs above the persistent kernel's limits (over 2^20 vertices) are
    solved one by one in the same call, beside the persistent ones."""
    rng = np.random.default_rng(5)
    graphs = [(1500, rng.integers(0, 1500, size=(4000, 2))),
              ((1 << 20) + 77, rng.integers(0, (1 << 20) + 77, size=(900000, 2))),
              (700, rng.integers(0, 700, size=(2000, 2)))]
    vo = np.cumsum([0] + [n for n, _ in graphs]).astype(np.int64)
    eo = np.cumsum([0] + [len(x) for _, x in graphs]).astype(np.int64)
    e = np.concatenate([x for _, x in graphs]).astype(np.int32)
    w = rng.integers(0, 1000, size=len(e)).astype(np.uint32)
    st = check_batched(ctx, vo, eo, e, w, U32, "one large", device=True)
    assert st["batch_large"] == 1 and st["batch_graphs"] == 2, st


def test_batched_union_mode_matches(pkg):
    """The disjoint-union path (MSF_BATCH_MODE=0) gives the same forests."""
    vo, eo, e, w_u, w_f = mixed_batch(seed=43)
    with env_set(MSF_BATCH_MODE="0"):
        c = pkg.Context(0)
    st = check_batched(c, vo, eo, e, w_u, U32, "union u32")
    assert st["batch_config"] == -1
    check_batched(c, vo, eo, e, w_f, F32, "union f32", device=True)
    c.close()


def test_batched_rejects_nan_and_leaves_outputs(ctx, pkg):
    vo, eo, e, w_u, w_f = mixed_batch(seed=44)
    w_f[int(eo[-2]) + 3] = np.nan  # in the last (largest) graph
    out = torch.full((int(vo[-1]),), -7, dtype=torch.int32, device="cuda:0")
    with pytest.raises(pkg.MSFError) as ex:
        ctx.solve_batched(vo, eo, dev(e), dev(w_f), wtype=F32, out=out)
    assert ex.value.status == 1
    torch.cuda.synchronize()
    assert bool((out == -7).all())


def test_batched_tuning_cache(ctx, pkg, tmp_path):
    """The tuner stores its choice per batch shape in MSF_TUNE_CACHE and a
    later call (here: a fresh process state is not needed, the file is read
    on first use) keeps using it."""
    vo, eo, e, w_u, _ = mixed_batch(seed=45)
    path = tmp_path / "tune.txt"
    with env_set(MSF_TUNE_CACHE=str(path)):
        os.environ.pop("MSF_BATCH_CONFIG", None)
        st1 = check_batched(ctx, vo, eo, e, w_u, U32, "tuned")
        st2 = check_batched(ctx, vo, eo, e, w_u, U32, "cached")
    assert st1["batch_config"] == st2["batch_config"] >= 0
    if path.exists():  # written when this process tuned the shape itself
        arch, nb, db, wt, idx = path.read_text().split()[:5]
        assert arch.startswith("gfx") and int(idx) == st1["batch_config"]


def test_batched_rejects_out_of_graph_endpoint(ctx, pkg):
    vo = np.array([0, 3, 6], np.int64)
    eo = np.array([0, 1, 2], np.int64)
    e = np.array([[0, 1], [2, 3]], np.int32)  # 3 is outside graph 1 (n=3)
    w = np.array([1, 2], np.uint32)
    with pytest.raises(pkg.MSFError):
        ctx.solve_batched(vo, eo, e, w, wtype=U32)


# ------------------------------------------------------------ full sizes --

def test_full_rmat_s22(ctx, pkg):
    n, e, w = gen.workload_rmat_s22()
    st = check_solve(ctx, pkg, n, e, w, F32, "rmat s22 full")
    say("rmat s22 stats", st)
    # the two-level build's own interval lies inside the build interval,
    # which also holds the run set-up and the run sort
    assert 0.0 < st["adjacency_ms"] < st["build_ms"], st
    assert st["adjacency_ms"] + st["pass_ms"][1] <= st["build_ms"], st


def test_full_grid_256(ctx, pkg):
    n, e, w = gen.workload_grid_256()
    st = check_solve(ctx, pkg, n, e, w, U32, "grid 256^3 full")
    say("grid stats", st)


def test_full_batch_every_graph(ctx, pkg):
    """All 10^4 graphs of the full batch against the oracle, one by one."""
    vo, eo, e, w = gen.workload_batch_10k()
    say("batch 10k full", int(vo[-1]), int(eo[-1]))
    ids, counts, totals = ctx.solve_batched(vo, eo, dev(e), dev(w), wtype=U32)
    torch.cuda.synchronize()
    ids = ids.cpu().numpy()
    for g in range(10000):
        n = int(vo[g + 1] - vo[g])
        ee, ww = e[eo[g]:eo[g + 1]], w[eo[g]:eo[g + 1]]
        wi, wc, wtot = oracle.msf(n, ee, ww, U32)
        assert counts[g] == wc, g
        assert np.array_equal(ids[vo[g]:vo[g] + wc].astype(np.int64), wi), g
        assert totals[g][0] == wtot[0] and totals[g][1] == wtot[1], g


class env_set:
    """Set MSF_* environment variables for contexts created inside."""

    def __init__(self, **kv):
        self.kv = kv

    def __enter__(self):
        self.old = {k: os.environ.get(k) for k in self.kv}
        os.environ.update(self.kv)

    def __exit__(self, *a):
        for k, v in self.old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


_FULL = {}


def full_case(label):
    """(n, e, w, wt, oracle result) of a full-size workload, kept for reuse."""
    if label not in _FULL:
        if label == "rmat s22":
            n, e, w = gen.workload_rmat_s22()
            wt = F32
        else:
            n, e, w = gen.workload_grid_256()
            wt = U32
        _FULL.clear()  # one full-size graph in host memory at a time
        _FULL[label] = (n, e, w, wt, oracle.msf(n, e, w, wt))
    return _FULL[label]


def check_full(c, label, mode):
    n, e, w, wt, (want_ids, want_cnt, want_tot) = full_case(label)
    say(label, mode, f"n={n} m={len(e)}")
    ids, cnt, tot = c.solve(n, dev(e), dev(w), wtype=wt)
    torch.cuda.synchronize()
    assert cnt == want_cnt, (label, mode)
    assert np.array_equal(ids.cpu().numpy().astype(np.int64), want_ids), (label, mode)
    assert tot[1] == want_tot[1] and (wt == F32 or tot[0] == want_tot[0]), (label, mode)
    return c.stats()


@pytest.mark.parametrize("label", ["rmat s22", "grid 256"])
def test_full_size_server_slot_path(pkg, label):
    """The path every server slot takes (one-level build, full sweep with
    the filtering policy, no head sweep) at full size."""
    with env_set(MSF_BUCKETED_BUILD="2", MSF_HEADS="0"):
        c = pkg.Context(0)
    st = check_full(c, label, "one-level build, full sweep")
    assert st["head_sweeps"] == 0 and st["runs"] == 0
    c.close()


@pytest.mark.parametrize("label", ["rmat s22", "grid 256"])
def test_full_size_device_atomic_build(pkg, label):
    """The device-atomic adjacency build at full size."""
    with env_set(MSF_BUCKETED_BUILD="0"):
        c = pkg.Context(0)
    check_full(c, label, "device-atomic build")
    c.close()


def test_one_pass_scan_of_many_vertices(pkg):
    """Scans of more than 16K tiles of 2048 items take the one-pass
    look-back scan instead of the three launches: the device-atomic build's
    row-pointer scan over 36M vertices (2M edges, most vertices isolated)."""
    n = 36 << 20
    e, w = gen.er(n, 2_000_000, seed=41)
    with env_set(MSF_BUCKETED_BUILD="0"):
        c = pkg.Context(0)
    try:
        check_solve(c, pkg, n, e, w, U32, "36M vertices, device-atomic build")
    finally:
        c.close()


@pytest.mark.usefixtures("wide_path")
def test_column_slices_are_result_invariant(pkg):
    graphs = [
        ("er", 5000, *gen.er(5000, 40000, seed=12), U32),
        ("rmat13", *gen.rmat(13, 16, seed=2), F32),
        ("grid20", *gen.grid(20, 20, 20, 0.05, seed=3), U32),
        ("sparse", 3000, *gen.er(3000, 1500, seed=13), U32),
    ]
    old = {k: os.environ.get(k) for k in ("MSF_SLICES", "MSF_FILTER")}
    try:
        for slices in ("1", "2", "3", "8"):
            for filt in ("1", "2"):
                os.environ["MSF_SLICES"] = slices
                os.environ["MSF_FILTER"] = filt
                c = pkg.Context(0)
                for label, n, e, w, wt in graphs:
                    check_solve(c, pkg, n, e, w, wt, f"slices={slices} filter={filt} {label}",
                                device=(label != "sparse"))
                    ref = oracle.multilinear(n, e, w, wt, np.arange(n))
                    g = pkg.Graph(c, n, e, w, wtype=wt)
                    dr = torch.empty(n, dtype=torch.int64, device="cuda:0")
                    c.multilinear(g, dev(np.arange(n, dtype=np.uint32)), dr)
                    torch.cuda.synchronize()
                    assert np.array_equal(dr.cpu().numpy().view(np.uint64), ref), label
                    # pairwise, with a parent vector of stars
                    rng = np.random.default_rng(int(slices))
                    roots = rng.choice(n, size=max(1, n // 20), replace=False).astype(np.uint32)
                    star = roots[rng.integers(0, len(roots), n)]
                    star[roots] = roots
                    dr.fill_(0)
                    c.multilinear_pairwise(g, dev(star), dr)
                    torch.cuda.synchronize()
                    assert np.array_equal(dr.cpu().numpy().view(np.uint64),
                                          oracle.multilinear(n, e, w, wt, star)), label + " pair"
                    g.close()
                c.close()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.usefixtures("wide_path")
def test_first_round_modes_agree(pkg):
    """Round 1 from the generic sweep (0), the identity-parent sweep (1) and
    the minima kept by the adjacency build (2) give the same forest, with one
    and with eight column slices; the 8.5M-vertex grid under eight slices
    needs 8192-row blocks, whose build keeps 96 KB of LDS."""
    graphs = [
        ("er", 5000, *gen.er(5000, 40000, seed=21), U32),
        ("rmat14", *gen.rmat(14, 16, seed=22), F32),
        ("grid12", *gen.grid(12, 12, 12, 0.05, seed=23), U32),
    ]
    big = ("grid204", *gen.grid(204, 204, 204, 0.05, seed=24), U32)
    old = {k: os.environ.get(k) for k in ("MSF_SLICES", "MSF_FIRST_ROUND")}
    try:
        for slices in ("1", "8"):
            for first in ("0", "1", "2"):
                os.environ["MSF_SLICES"] = slices
                os.environ["MSF_FIRST_ROUND"] = first
                c = pkg.Context(0)
                cases = graphs + ([big] if (slices, first) in (("8", "2"), ("1", "2")) else [])
                for label, n, e, w, wt in cases:
                    check_solve(c, pkg, n, e, w, wt, f"slices={slices} first={first} {label}")
                    if first == "2":  # no sweep in round 1
                        assert c.stats()["sweep_bytes"][0] == 0, label
                c.close()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.usefixtures("wide_path")
def test_build_modes_agree(pkg):
    """The device-atomic (0), two-level bucketed (1, default) and one-level
    bucketed (2) adjacency builds give the same forest: skewed R-MAT rows far
    larger than a placement workgroup's LDS, the same kind of graph with ids
    sorted by degree (the first coarse bucket then holds over a million
    entries, more level-2 windows than a placement workgroup gathers at
    once), a grid, a multigraph with loops, and a graph with more vertices
    than edges.  The two-level build runs twice: with each level-2 entry's
    row inside its fine bucket in its column word (the default where the
    bits fit) and in the separate 2-byte array."""
    rng = np.random.default_rng(31)
    nm = 3000
    multi_e = rng.integers(0, nm, size=(20000, 2)).astype(np.int32)
    multi_w = rng.integers(0, 50, size=20000).astype(np.uint32)
    ns, es, ws = gen.rmat(16, 32, seed=35)
    deg = np.bincount(es.reshape(-1), minlength=ns)
    newid = np.empty(ns, dtype=np.int32)
    newid[np.argsort(-deg, kind="stable")] = np.arange(ns, dtype=np.int32)
    es = newid[es]
    graphs = [
        ("rmat15", *gen.rmat(15, 16, seed=32), F32),
        ("rmat16 degree-sorted", ns, es, ws, F32),
        ("grid24", *gen.grid(24, 24, 24, 0.05, seed=33), U32),
        ("multi", nm, multi_e, multi_w, U32),
        ("sparse", 50000, *gen.er(50000, 20000, seed=34), U32),
    ]
    keys = ("MSF_BUCKETED_BUILD", "MSF_TL_ROW_IN_COL")
    old = {k: os.environ.get(k) for k in keys}
    try:
        for mode, ric in (("0", "1"), ("1", "1"), ("1", "0"), ("2", "1")):
            os.environ["MSF_BUCKETED_BUILD"] = mode
            os.environ["MSF_TL_ROW_IN_COL"] = ric
            c = pkg.Context(0)
            for label, n, e, w, wt in graphs:
                check_solve(c, pkg, n, e, w, wt, f"build={mode} row_in_col={ric} {label}")
            c.close()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.usefixtures("wide_path")
def test_head_sweep_with_every_build_and_first_round(pkg):
    """The head sweep forced on after the device-atomic (0) and one-level (2)
    builds (runs set up from row_ptr by their own kernels) and with round 1
    swept instead of taken from the build (first round 0 and 1): the
    oracle's forest and per-round hooks."""
    graphs = [
        ("rmat14", *gen.rmat(14, 16, seed=51), F32),
        ("grid12", *gen.grid(12, 12, 12, 0.05, seed=52), U32),
    ]
    keys = ("MSF_HEADS", "MSF_BUCKETED_BUILD", "MSF_FIRST_ROUND")
    old = {k: os.environ.get(k) for k in keys}
    try:
        for build, first in (("0", "2"), ("2", "2"), ("1", "0"), ("1", "1")):
            os.environ["MSF_HEADS"] = "2"
            os.environ["MSF_BUCKETED_BUILD"] = build
            os.environ["MSF_FIRST_ROUND"] = first
            c = pkg.Context(0)
            for label, n, e, w, wt in graphs:
                st = check_solve(c, pkg, n, e, w, wt, f"heads build={build} first={first} {label}")
                ref = oracle.as_rounds(n, e, w, wt)
                hooks = [h for h in ref["hooks"] if h]
                assert st["hooks"][:len(hooks)] == hooks, (label, st["hooks"], hooks)
                assert st["runs"] > 0 and st["head_sweeps"] >= 1, (label, st["runs"])
            c.close()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
