"""Serving loop: results in a mixed, overlapping stream equal solo results
and the oracle (tolerance 0); budget admission; error isolation."""
import sys
import threading
import time

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U32, F32 = oracle.W_U32, oracle.W_F32


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


def small_pool(count=16, seed=5):
    # the served mix in miniature: R-MAT (edge factor 16) and cubic grids
    return gen.serve_pool(count, seed=seed, log2_lo=8.0, log2_hi=15.0)


def test_mixed_stream_equals_solo_and_oracle(ctx, pkg):
    pool = small_pool()
    srv = pkg.Server(ctx, 8 << 30)
    say("server mixed stream", len(pool))
    tickets = []
    for i, (n, e, w, kind) in enumerate(pool * 2):
        tickets.append((srv.submit(n, e, w, wtype=F32), n, e, w))
        if i % 5 == 0:
            time.sleep(0.002)  # arrivals while others are in flight
    for t, n, e, w in tickets:
        ids, cnt, tot = srv.result(t, n)
        want_ids, want_cnt, want_tot = oracle.msf(n, e, w, F32)
        assert cnt == want_cnt and np.array_equal(ids.astype(np.int64), want_ids)
        assert tot[1] == want_tot[1]
        sids, scnt, stot = ctx.solve(n, e, w, wtype=F32)
        assert scnt == cnt and np.array_equal(sids, ids) and stot == tot
    srv.close()


def test_latency_and_poll(ctx, pkg):
    n, e, w = gen.rmat(12, 16, seed=9)
    srv = pkg.Server(ctx, 4 << 30)
    t = srv.submit(n, e, w, wtype=F32)
    deadline = time.time() + 60
    while not srv.poll(t):
        assert time.time() < deadline
        time.sleep(0.001)
    lat = srv.latency(t)
    assert 0 < lat < 60
    ids, cnt, tot = srv.result(t, n)
    assert cnt == oracle.msf(n, e, w, F32)[1]
    with pytest.raises(pkg.MSFError):
        srv.poll(t)  # released by result()
    srv.close()


def test_budget_admission_serialises_but_stays_exact(ctx, pkg):
    pool = small_pool(8, seed=7)
    biggest = max(pkg.footprint(n, len(e)) for n, e, w, k in pool)
    srv = pkg.Server(ctx, biggest + 1)  # at most about one request resident
    say("server tight budget", biggest)
    ts = [(srv.submit(n, e, w, wtype=F32), n, e, w) for n, e, w, k in pool]
    for t, n, e, w in ts:
        ids, cnt, tot = srv.result(t, n)
        want_ids, want_cnt, want_tot = oracle.msf(n, e, w, F32)
        assert cnt == want_cnt and np.array_equal(ids.astype(np.int64), want_ids)
    # a request that can never fit is refused up front
    m = 4 * 1024 * 1024
    assert pkg.footprint(1 << 20, m) > biggest + 1
    with pytest.raises(pkg.MSFError) as ex:
        srv.submit(1 << 20, np.zeros((m, 2), np.int32), np.ones(m, np.uint32), wtype=U32)
    assert ex.value.status == 4
    srv.close()


def test_bad_request_fails_alone(ctx, pkg):
    srv = pkg.Server(ctx, 4 << 30)
    good = [gen.rmat(10, 16, seed=s) for s in (1, 2, 3)]
    t0 = srv.submit(*good[0], wtype=F32)
    bad = srv.submit(10, np.array([[0, 1], [3, 99]], np.int32), np.array([1, 2], np.uint32),
                     wtype=U32)
    t1 = srv.submit(*good[1], wtype=F32)
    t2 = srv.submit(*good[2], wtype=F32)
    with pytest.raises(pkg.MSFError) as ex:
        srv.result(bad, 10)
    assert ex.value.status == 1
    for t, (n, e, w) in zip((t0, t1, t2), good):
        ids, cnt, tot = srv.result(t, n)
        assert np.array_equal(ids.astype(np.int64), oracle.msf(n, e, w, F32)[0])
    with pytest.raises(pkg.MSFError) as ex:
        srv.result(123456789, 10)
    assert ex.value.status == 5
    srv.close()


def test_concurrent_submitters(ctx, pkg):
    pool = small_pool(12, seed=11)
    srv = pkg.Server(ctx, 8 << 30)
    out = {}

    def client(k):
        n, e, w, kind = pool[k]
        t = srv.submit(n, e, w, wtype=F32)
        out[k] = srv.result(t, n)

    th = [threading.Thread(target=client, args=(k,)) for k in range(len(pool))]
    for x in th:
        x.start()
    for x in th:
        x.join(120)
    for k, (n, e, w, kind) in enumerate(pool):
        ids, cnt, tot = out[k]
        assert np.array_equal(ids.astype(np.int64), oracle.msf(n, e, w, F32)[0])
    srv.close()


def test_full_pool_at_real_sizes(ctx, pkg):
    """The whole served pool at its real sizes (R-MAT up to scale 21 with
    edge factor 16, grids up to about 148^3), submitted with overlapping
    arrivals under a 32 GiB budget: every result equals the oracle's forest
    (ids, count, totals) and the solo msf_solve of the same request."""
    t0 = time.time()
    pool = gen.serve_pool(64, seed=5)
    say("full served pool generated", len(pool), f"{time.time() - t0:.1f}s",
        sum(len(p[1]) for p in pool), "edges")
    srv = pkg.Server(ctx, 32 << 30)
    order = list(range(len(pool)))
    np.random.default_rng(3).shuffle(order)
    tickets = []
    for i, k in enumerate(order):
        n, e, w, kind = pool[k]
        tickets.append((srv.submit(n, e, w, wtype=F32), k))
        if i % 4 == 3:
            time.sleep(0.003)  # later requests arrive while earlier ones run
    for t, k in tickets:
        n, e, w, kind = pool[k]
        ids, cnt, tot = srv.result(t, n)
        want_ids, want_cnt, want_tot = oracle.msf(n, e, w, F32)
        assert cnt == want_cnt, (k, kind, n)
        assert np.array_equal(ids.astype(np.int64), want_ids), (k, kind, n)
        assert tot[1] == want_tot[1], (k, kind, n)
        sids, scnt, stot = ctx.solve(n, e, w, wtype=F32)
        assert scnt == cnt and np.array_equal(sids, ids) and stot == tot, (k, kind, n)
    say("full served pool checked", f"{time.time() - t0:.1f}s")
    srv.close()


def test_shared_launches_equal_slots(ctx, pkg):
    """Small requests solved together in shared persistent launches give the
    same forests as with every request in its own slot (MSF_SERVER_BATCH=0),
    and both equal solo msf_solve; a failing small request fails alone."""
    import os
    pool = gen.serve_pool(24, seed=13, log2_lo=6.0, log2_hi=13.5)
    bad = (10, np.array([[0, 1], [3, 99]], np.int32), np.array([1.0, 2.0], np.float32), "bad")
    results = {}
    for mode in ("1", "0"):
        old = os.environ.get("MSF_SERVER_BATCH")
        os.environ["MSF_SERVER_BATCH"] = mode
        try:
            srv = pkg.Server(ctx, 8 << 30)
        finally:
            if old is None:
                os.environ.pop("MSF_SERVER_BATCH", None)
            else:
                os.environ["MSF_SERVER_BATCH"] = old
        reqs = pool * 3
        reqs.insert(17, bad)
        tickets = [(srv.submit(n, e, w, wtype=F32), n, kind) for n, e, w, kind in reqs]
        out = []
        for t, n, kind in tickets:
            if kind == "bad":
                with pytest.raises(pkg.MSFError) as ex:
                    srv.result(t, n)
                assert ex.value.status == 1
                continue
            out.append(srv.result(t, n))
        srv.close()
        results[mode] = out
    good = [p for p in pool * 3]
    for (a, b, (n, e, w, kind)) in zip(results["1"], results["0"], good):
        assert a[1] == b[1] and np.array_equal(a[0], b[0]) and a[2] == b[2], (kind, n)
    for n, e, w, kind in pool:
        si, sc, st = ctx.solve(n, e, w, wtype=F32)
        wi, wc, wt = oracle.msf(n, e, w, F32)
        assert sc == wc and np.array_equal(si.astype(np.int64), wi) and st[1] == wt[1]
    k = 0
    for n, e, w, kind in good:
        ids, cnt, tot = results["1"][k]
        k += 1
        wi, wc, wt = oracle.msf(n, e, w, F32)
        assert cnt == wc and np.array_equal(ids.astype(np.int64), wi) and tot[1] == wt[1]
