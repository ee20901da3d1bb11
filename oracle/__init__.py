"""CPU oracle for the algebraic Awerbuch-Shiloach minimum spanning forest.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP library (``paper_2110_04865_amd``) and never imports it.

Functions and what each follows
-------------------------------
``edge_keys``        the total edge order: key(e) = (wkey(w_e) << 32) | e.
                     The paper assumes distinct weights (section 2); ties are
                     broken by edge id, which makes the forest unique and keeps
                     the no-long-cycle argument of the tie-breaking step
                     (section 2.3) valid.  float32 weights map to an
                     order-preserving unsigned key; -0.0 is +0.0; NaN is an
                     error.
``msf``              the minimum spanning forest under that order (section 2,
                     problem statement).  Plain Kruskal: a library sort of the
                     keys, then union-find in C (``oracle.c``).
``multilinear``      the all-at-once multilinear kernel of section 3.1 with
                     the projection step of Algorithm 2:
                     r[k] = min{key(e) : stored direction i->j of e,
                     p[i] == k, p[i] != p[j]}, UINT64_MAX where none.
``find_roots``       complete shortcutting (section 4.2): every vertex ends at
                     the root of its tree; error on a cycle.
``as_rounds``        Algorithm 2 step by step with complete shortcutting
                     (section 4.2), numpy vectorised, for per-round
                     statistics: multilinear kernel, projection, hooking,
                     tie-breaking, shortcutting until every tree is a star.
``components``       connected components (section 2.4, the result of the
                     connectivity variant): union-find over every edge in C
                     (``oracle.c``); each vertex is labelled with the
                     smallest vertex id of its component.
``total``            forest weight: exact integer sum for uint32 weights; the
                     exact real sum rounded once to float64 for float32
                     weights (``math.fsum``), so it is independent of
                     summation order.

Parity pins for all of the above live in ``tests/test_oracle.py``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

W_U32 = 0
W_F32 = 1
INF = np.uint64(0xFFFFFFFFFFFFFFFF)


def build(verbose: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (plain gcc, no OpenMP)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-o", _SO + ".tmp", os.path.join(_HERE, "oracle.c")]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    P = ctypes.c_void_p
    lib.oracle_kruskal.restype = ctypes.c_int64
    lib.oracle_kruskal.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P]
    lib.oracle_multilinear.restype = None
    lib.oracle_multilinear.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, P]
    lib.oracle_multilinear_rows.restype = None
    lib.oracle_multilinear_rows.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, P, P]
    lib.oracle_find_roots.restype = ctypes.c_int
    lib.oracle_find_roots.argtypes = [ctypes.c_int32, P, P]
    lib.oracle_components.restype = ctypes.c_int64
    lib.oracle_components.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _edges2(edges) -> np.ndarray:
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32))
    return e.reshape(-1, 2) if e.size else np.zeros((0, 2), dtype=np.int32)


# ------------------------------------------------------------------ keys --

def weight_keys(w, wtype: int) -> np.ndarray:
    """Order-preserving 32-bit unsigned key of each weight (uint64 array)."""
    if wtype == W_U32:
        return np.asarray(w, dtype=np.uint32).astype(np.uint64)
    wf = np.asarray(w, dtype=np.float32)
    if np.isnan(wf).any():
        raise ValueError("NaN weight")
    bits = wf.view(np.uint32).astype(np.uint64)
    bits = np.where(bits == 0x80000000, np.uint64(0), bits)  # -0.0 -> +0.0
    neg = (bits >> np.uint64(31)) != 0
    # negative floats: flip every bit; non-negative: set the sign bit
    return np.where(neg, bits ^ np.uint64(0xFFFFFFFF), bits | np.uint64(0x80000000))


def edge_keys(w, wtype: int) -> np.ndarray:
    """key(e) = (wkey(w_e) << 32) | e as uint64."""
    wk = weight_keys(w, wtype)
    return (wk << np.uint64(32)) | np.arange(len(wk), dtype=np.uint64)


def validate(n: int, edges, w, wtype: int):
    e = _edges2(edges)
    if n < 0 or n > 2**31 - 1 or len(e) > 2**31 - 1:
        raise ValueError("size out of range")
    if len(w) != len(e):
        raise ValueError("weights/edges length mismatch")
    if len(e) and (e.min() < 0 or e.max() >= n):
        raise ValueError("endpoint out of range")
    if wtype == W_F32 and np.isnan(np.asarray(w, dtype=np.float32)).any():
        raise ValueError("NaN weight")
    return e


# -------------------------------------------------------------- results --

def total(w, ids, wtype: int):
    """(u64, f64) forest weight.  u64 is exact for uint32 weights (0 for
    float32); f64 is the exact sum rounded once to float64."""
    ids = np.asarray(ids, dtype=np.int64)
    if wtype == W_U32:
        s = int(np.asarray(w, dtype=np.uint32)[ids].astype(np.uint64).sum(dtype=np.uint64))
        return s, float(s)
    vals = np.asarray(w, dtype=np.float32)[ids].astype(np.float64)
    vals = np.where(vals == 0.0, 0.0, vals)  # -0.0 counts as +0.0
    return 0, math.fsum(vals.tolist())


def msf(n: int, edges, w, wtype: int):
    """Minimum spanning forest under key(e).

    Returns (ids int64 ascending, count, (total_u64, total_f64))."""
    e = validate(n, edges, w, wtype)
    m = len(e)
    keys = edge_keys(w, wtype)
    keys = keys[e[:, 0] != e[:, 1]] if m else keys
    keys = np.sort(keys)  # library sort as a step; keys are distinct
    flags = np.zeros(max(m, 1), dtype=np.uint8)
    cnt = _load().oracle_kruskal(n, len(keys), _ptr(keys), _ptr(e), _ptr(flags))
    if cnt < 0:
        raise MemoryError("oracle_kruskal")
    ids = np.nonzero(flags[:m])[0].astype(np.int64)
    assert len(ids) == cnt
    return ids, int(cnt), total(w, ids, wtype)


def multilinear(n: int, edges, w, wtype: int, p, rows=None) -> np.ndarray:
    """r[k] = min key over stored directions i->j with p[i]==k != p[j].

    rows (optional): the row subset, as vertex ids or a boolean mask of
    length n; only stored directions i->j with i in it count (one owner's
    share when the rows of A are split, section 5)."""
    e = validate(n, edges, w, wtype)
    keys = np.ascontiguousarray(edge_keys(w, wtype))
    p = np.ascontiguousarray(np.asarray(p, dtype=np.uint32))
    if len(p) != n or (n and p.max() >= n):
        raise ValueError("bad parent vector")
    r = np.empty(max(n, 1), dtype=np.uint64)
    if rows is None:
        _load().oracle_multilinear(n, len(e), _ptr(e), _ptr(keys), _ptr(p), _ptr(r))
        return r[:n]
    rows = np.asarray(rows)
    mask = np.zeros(max(n, 1), dtype=np.uint8)
    if rows.dtype == np.bool_:
        if len(rows) != n:
            raise ValueError("row mask must have length n")
        mask[:n] = rows
    else:
        rows = rows.astype(np.int64)
        if len(rows) and (rows.min() < 0 or rows.max() >= n):
            raise ValueError("row id out of range")
        mask[rows] = 1
    _load().oracle_multilinear_rows(n, len(e), _ptr(e), _ptr(keys), _ptr(p), _ptr(mask),
                                    _ptr(r))
    return r[:n]


def find_roots(p) -> np.ndarray:
    """Root of every vertex in the parent forest p; ValueError on a cycle."""
    p = np.ascontiguousarray(np.asarray(p, dtype=np.uint32))
    n = len(p)
    root = np.empty(max(n, 1), dtype=np.uint32)
    rc = _load().oracle_find_roots(n, _ptr(p), _ptr(root))
    if rc == -1:
        raise ValueError("parent vector has a cycle")
    if rc == -2:
        raise ValueError("parent out of range")
    if rc != 0:
        raise MemoryError("oracle_find_roots")
    return root[:n]


def components(n: int, edges):
    """(labels int32[n], count): labels[i] is the smallest vertex id of the
    connected component of i (section 2.4 computes this partition)."""
    e = _edges2(edges)
    lab = np.empty(max(n, 1), dtype=np.int32)
    c = _load().oracle_components(n, len(e), _ptr(e), _ptr(lab))
    if c == -1:
        raise ValueError("endpoint out of range")
    if c < 0:
        raise MemoryError("oracle_components")
    return lab[:n], int(c)


# ------------------------------------------------- Algorithm 2, by rounds --

def as_rounds(n: int, edges, w, wtype: int, max_rounds: int = 1000):
    """Algorithm 2 with complete shortcutting, one vectorised operation per step.

    Readings: vertices are 0-indexed and the empty EDGE is UINT64_MAX; the
    EDGE pair carries the edge id in place of the parent and the hook target
    is recovered from the edge's endpoints; the smaller id of a mutual pair
    reverts to root; only kept hooks add weight; the loop stops after a
    round in which nothing hooks (the parent vector is then unchanged).

    Returns dict(ids, count, total, hooks=[per round], roots=[per round,
    before hooking], sub_iters=[per round, synchronous pointer jumping]).
    """
    e = validate(n, edges, w, wtype)
    m = len(e)
    keys = edge_keys(w, wtype)
    u = e[:, 0].astype(np.int64)
    v = e[:, 1].astype(np.int64)
    p = np.arange(n, dtype=np.int64)
    forest = np.zeros(m, dtype=bool)
    hooks, roots_before, subs = [], [], []
    for _ in range(max_rounds):
        pu, pv = p[u], p[v]
        out = pu != pv
        # multilinear kernel + projection (every tree is a star here)
        r = np.full(n, INF, dtype=np.uint64)
        np.minimum.at(r, pu[out], keys[out])
        np.minimum.at(r, pv[out], keys[out])
        is_root = p == np.arange(n)
        roots_before.append(int(is_root.sum()))
        hooked = np.nonzero(r != INF)[0]
        if len(hooked) == 0:
            hooks.append(0)
            subs.append(0)
            break
        eid = (r[hooked] & np.uint64(0xFFFFFFFF)).astype(np.int64)
        a, b = p[u[eid]], p[v[eid]]
        h = np.arange(n, dtype=np.int64)
        h[hooked] = np.where(a == hooked, b, a)  # hook: p_i <- r_i's parent
        # tie-breaking: t_i = i < p_i and p_{p_i} = i
        t = (hooked < h[hooked]) & (h[h[hooked]] == hooked)
        h[hooked[t]] = hooked[t]
        forest[eid[~t]] = True
        hooks.append(int((~t).sum()))
        # complete shortcutting: p <- p_p until every tree is a star
        s = 0
        while True:
            hh = h[h]
            if np.array_equal(hh, h):
                break
            h = hh
            s += 1
        subs.append(s)
        p = h[p]
    ids = np.nonzero(forest)[0].astype(np.int64)
    return dict(ids=ids, count=len(ids), total=total(w, ids, wtype), hooks=hooks,
                roots=roots_before, sub_iters=subs)
