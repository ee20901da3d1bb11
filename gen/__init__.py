"""Seeded synthetic graph generators (shared test/benchmark input module).

Holds no minimum-spanning-forest arithmetic: it produces undirected edge
lists (``int32[m, 2]``) and weights (``uint32[m]`` or ``float32[m]``) only.
Both the CPU oracle and the HIP path consume these arrays.

The workload families stand in for the paper's evaluation graphs (section 7,
Table 1): R-MAT for the skewed social networks, a 3D 7-point grid with a
fraction of edges dropped for the high-diameter road networks, and
Erdos-Renyi graphs for the uniform random graphs of the weak-scaling study.
The datasets themselves are not used.

The C source ``gen.c`` is compiled by :func:`build` into ``libmsfgen.so``
next to this file.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libmsfgen.so")
_lib = None

W_U32 = 0
W_F32 = 1

# Default seeds of the five named workloads.
SEED_ER = 1
SEED_RMAT = 2
SEED_GRID = 3
SEED_BATCH = 4
SEED_SERVE = 5


def build(verbose: bool = False) -> str:
    """Compile ``gen.c`` into ``libmsfgen.so`` (gcc, OpenMP)."""
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", _SO + ".tmp",
           os.path.join(_HERE, "gen.c"), "-lm"]
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
    lib.gen_draw.restype = ctypes.c_uint64
    lib.gen_draw.argtypes = [ctypes.c_uint64] * 3
    lib.gen_weights.restype = None
    lib.gen_weights.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, P]
    lib.gen_er.restype = ctypes.c_int
    lib.gen_er.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, P]
    lib.gen_rmat.restype = ctypes.c_int64
    lib.gen_rmat.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64, P, ctypes.c_int64]
    lib.gen_grid_full_edges.restype = ctypes.c_int64
    lib.gen_grid_full_edges.argtypes = [ctypes.c_int32] * 3
    lib.gen_grid.restype = ctypes.c_int64
    lib.gen_grid.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                             ctypes.c_uint64, ctypes.c_uint64, P]
    lib.gen_batch_sizes.restype = None
    lib.gen_batch_sizes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_uint64, P]
    lib.gen_batch_fill.restype = ctypes.c_int
    lib.gen_batch_fill.argtypes = [ctypes.c_int32, P, P, ctypes.c_uint64, ctypes.c_int, P, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def draw(seed: int, stream: int, index: int) -> int:
    """The counter-based 64-bit draw every generator uses."""
    return int(_load().gen_draw(seed, stream, index))


def weights(m: int, wtype: int, seed: int, stream: int = 2) -> np.ndarray:
    """Edge weights: uint32 (top 32 bits of a draw) or float32 k*2^-24, k in [1, 2^24-1]."""
    lib = _load()
    out = np.empty(m, dtype=np.uint32 if wtype == W_U32 else np.float32)
    lib.gen_weights(seed, stream, m, wtype, _ptr(out))
    return out


def er(n: int, m: int, seed: int = SEED_ER, wtype: int = W_U32, stream_base: int = 0):
    """Erdos-Renyi G(n, m) without self-loops or duplicates; returns (edges, w)."""
    lib = _load()
    edges = np.empty((m, 2), dtype=np.int32)
    if lib.gen_er(n, m, seed, stream_base + 1, _ptr(edges)) != 0:
        raise ValueError(f"cannot draw {m} distinct edges on {n} vertices")
    return edges, weights(m, wtype, seed, stream_base + 2)


def rmat(scale: int, ef: int = 16, seed: int = SEED_RMAT, wtype: int = W_F32,
         a: float = 0.57, b: float = 0.19, c: float = 0.19, stream_base: int = 0):
    """R-MAT graph with 2^scale vertices, ef*2^scale draws, permuted ids,
    self-loops and duplicates removed; returns (n, edges, w)."""
    lib = _load()
    cap = ef << scale
    edges = np.empty((cap, 2), dtype=np.int32)
    m = lib.gen_rmat(scale, ef, a, b, c, seed, stream_base, _ptr(edges), cap)
    if m < 0:
        raise MemoryError("R-MAT generation failed")
    edges = edges[:m]
    return 1 << scale, edges, weights(m, wtype, seed, stream_base + 2)


def grid_full_edges(sx: int, sy: int, sz: int) -> int:
    return int(_load().gen_grid_full_edges(sx, sy, sz))


def grid(sx: int, sy: int | None = None, sz: int | None = None, drop_frac: float = 0.05,
         seed: int = SEED_GRID, wtype: int = W_U32, stream_base: int = 0):
    """3D 7-point grid with exactly floor(drop_frac * M) edges removed;
    returns (n, edges, w)."""
    sy = sx if sy is None else sy
    sz = sx if sz is None else sz
    lib = _load()
    M = grid_full_edges(sx, sy, sz)
    drop = int(math.floor(drop_frac * M + 1e-9))
    edges = np.empty((M - drop, 2), dtype=np.int32)
    m = lib.gen_grid(sx, sy, sz, drop, seed, stream_base, _ptr(edges))
    if m != M - drop:
        raise RuntimeError("grid generation failed")
    return sx * sy * sz, edges, weights(m, wtype, seed, stream_base + 2)


def batch(G: int, seed: int = SEED_BATCH, lo: int = 64, hi: int = 65536, edge_ratio: int = 4,
          wtype: int = W_U32):
    """G independent Erdos-Renyi graphs, n_g log-uniform in [lo, hi), m_g = edge_ratio*n_g.

    Returns (vtx_off int64[G+1], edge_off int64[G+1], edges int32[sum m, 2] with
    local vertex ids, w)."""
    lib = _load()
    n = np.empty(G, dtype=np.int32)
    lib.gen_batch_sizes(G, lo, hi, seed, _ptr(n))
    vtx_off = np.zeros(G + 1, dtype=np.int64)
    vtx_off[1:] = np.cumsum(n, dtype=np.int64)
    edge_off = np.zeros(G + 1, dtype=np.int64)
    edge_off[1:] = np.cumsum(n.astype(np.int64) * edge_ratio)
    M = int(edge_off[-1])
    edges = np.empty((M, 2), dtype=np.int32)
    w = np.empty(M, dtype=np.uint32 if wtype == W_U32 else np.float32)
    bad = lib.gen_batch_fill(G, _ptr(vtx_off), _ptr(edge_off), seed, wtype, _ptr(edges), _ptr(w))
    if bad:
        raise RuntimeError(f"batch graph {bad - 1} failed")
    return vtx_off, edge_off, edges, w


def serve_pool(count: int = 64, seed: int = SEED_SERVE, log2_lo: float = 10.0,
               log2_hi: float = 22.0, wtype: int = W_F32, max_log2: float | None = None):
    """Pool of mixed request graphs: log2(n) uniform in [log2_lo, log2_hi];
    the first half R-MAT with scale round(log2 n) and edge factor 16, the
    second half cubic grids with side round(n^(1/3)) and 5% of edges dropped.

    ``max_log2`` optionally caps the drawn size (smaller pools for tests).
    Returns a list of (n, edges, w, kind)."""
    pool = []
    for g in range(count):
        x = draw(seed, 5, g)
        u = (x >> 11) * 2.0 ** -53
        l2 = log2_lo + (log2_hi - log2_lo) * u
        if max_log2 is not None:
            l2 = min(l2, max_log2)
        sb = 16 + 4 * g
        if g < count // 2:
            s = int(round(l2))
            n, e, w = rmat(s, 16, seed, wtype, stream_base=sb)
            pool.append((n, e, w, "rmat"))
        else:
            side = max(2, int(round(2.0 ** (l2 / 3.0))))
            n, e, w = grid(side, side, side, 0.05, seed, wtype, stream_base=sb)
            pool.append((n, e, w, "grid"))
    return pool


# --- the five named workloads -------------------------------------------

def workload_er_4096():
    """Erdos-Renyi n=4096, m=32768, uint32 weights."""
    e, w = er(4096, 32768, SEED_ER, W_U32)
    return 4096, e, w


def workload_rmat_s22():
    """R-MAT scale 22, edge factor 16, a/b/c/d = .57/.19/.19/.05, float32 weights."""
    return rmat(22, 16, SEED_RMAT, W_F32)


def workload_grid_256():
    """256^3 7-point grid, 5% of edges dropped, uint32 weights."""
    return grid(256, 256, 256, 0.05, SEED_GRID, W_U32)


def workload_batch_10k(G: int = 10000):
    """10^4 Erdos-Renyi graphs, n log-uniform in [64, 65536), average degree 8."""
    return batch(G, SEED_BATCH, 64, 65536, 4, W_U32)
