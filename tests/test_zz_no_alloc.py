"""The allocation-free batched solve (msf_solve_batched_noalloc), called
through the C ABI, against msf_solve_batched: bit-identical forest ids,
counts and totals on two calls in a row (the second with a smaller batch,
on the same static scratch), and its checks reject bad input before
writing anything."""
import ctypes
import sys

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def noalloc(pkg, ctx, vo, eo, e, w, wt):
    """One call through the C ABI; returns (ids, counts, totals) on the host."""
    L = pkg.lib()
    G = len(vo) - 1
    N, M = int(vo[-1]), int(eo[-1])
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    dvo, deo = d(vo.astype(np.int64)), d(eo.astype(np.int64))
    de = d(e.reshape(-1).astype(np.int32))
    dw = d(w.view(np.int32))
    out = torch.full((max(N, 1),), -1, dtype=torch.int32, device="cuda:0")
    counts = torch.full((max(G, 1),), -1, dtype=torch.int64, device="cuda:0")
    totals = torch.zeros((max(G, 1), 2), dtype=torch.int64, device="cuda:0")
    P = ctypes.c_void_p
    rc = L.msf_solve_batched_noalloc(ctx._h, G, P(dvo.data_ptr()), P(deo.data_ptr()),
                                     P(de.data_ptr()), P(dw.data_ptr()), wt,
                                     P(out.data_ptr()), P(counts.data_ptr()),
                                     P(totals.data_ptr()))
    torch.cuda.synchronize()
    if rc != 0:
        raise pkg.MSFError(rc, L.msf_last_error().decode())
    t = totals.cpu().numpy()
    return (out.cpu().numpy(), counts.cpu().numpy()[:G],
            [(int(np.uint64(x[0])), float(x[1:2].view(np.float64)[0])) for x in t[:G]])


def compare(pkg, ctx, vo, eo, e, w, wt, label):
    G = len(vo) - 1
    ids, counts, totals = noalloc(pkg, ctx, vo, eo, e, w, wt)
    rid, rcounts, rtotals = ctx.solve_batched(vo, eo, e, w, wtype=wt)
    assert np.array_equal(counts, rcounts), label
    for g in range(G):
        a, c = int(vo[g]), int(counts[g])
        assert np.array_equal(ids[a:a + c], rid[a:a + c]), (label, g)
        assert totals[g][0] == rtotals[g][0], (label, g)
        assert totals[g][1] == rtotals[g][1], (label, g)
    # and a few against the oracle directly
    for g in range(0, G, max(1, G // 7)):
        n = int(vo[g + 1] - vo[g])
        wi, wc, wtot = oracle.msf(n, e[eo[g]:eo[g + 1]], w[eo[g]:eo[g + 1]], wt)
        assert counts[g] == wc and np.array_equal(ids[vo[g]:vo[g] + wc].astype(np.int64), wi)
    say(label, "ok", G, "graphs")


def test_noalloc_equals_batched_twice(pkg, ctx):
    vo, eo, e, w = gen.batch(400, seed=71, lo=16, hi=20000)
    compare(pkg, ctx, vo, eo, e, w, oracle.W_U32, "first call, 400 graphs")
    vo2, eo2, e2, _ = gen.batch(37, seed=72, lo=8, hi=3000)
    w2 = gen.weights(len(e2), gen.W_F32, seed=72)
    compare(pkg, ctx, vo2, eo2, e2, w2, oracle.W_F32, "second call, 37 smaller graphs")


def test_noalloc_rejects_before_writing(pkg, ctx):
    vo = np.array([0, 3, 6], np.int64)
    eo = np.array([0, 1, 2], np.int64)
    e = np.array([[0, 1], [2, 3]], np.int32)  # 3 is outside graph 1
    w = np.array([1, 2], np.uint32)
    with pytest.raises(pkg.MSFError) as ex:
        noalloc(pkg, ctx, vo, eo, e, w, oracle.W_U32)
    assert ex.value.status == 1
    # a graph above the size limits
    vo = np.array([0, (1 << 20) + 1], np.int64)
    eo = np.array([0, 1], np.int64)
    with pytest.raises(pkg.MSFError) as ex:
        noalloc(pkg, ctx, vo, eo, np.array([[0, 1]], np.int32), np.array([1], np.uint32),
                oracle.W_U32)
    assert ex.value.status == 1
    # the first call after the errors is exact again
    vo, eo, e, w = gen.batch(20, seed=73, lo=16, hi=500)
    compare(pkg, ctx, vo, eo, e, w, oracle.W_U32, "after errors")
