"""Python binding of ``libmsf.so``, the gfx950 minimum spanning forest library.

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in ``include/msf.h``.  Host inputs are
numpy arrays; device inputs are torch CUDA (ROCm) tensors, whose
``data_ptr()`` is passed through together with the current torch stream.

There is no fallback: importing works without the library, but any call
raises :class:`MSFError` if ``libmsf.so`` has not been built.
"""
from __future__ import annotations

import atexit
from collections.abc import Sequence
import ctypes
import os
import weakref

import numpy as np

__all__ = ["MSFError", "Context", "Graph", "Server", "lib", "W_U32", "W_F32",
           "STATUS_NAMES", "footprint"]

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "libmsf.so")

W_U32 = 0
W_F32 = 1
MEM_HOST = 0
MEM_DEVICE = 1
# shortcut strategies (msf_shortcut_strategy)
SHORTCUT_FRONTIER, SHORTCUT_FULL, SHORTCUT_SWITCH = 0, 1, 2
STATUS_NAMES = {0: "MSF_OK", 1: "MSF_EINVAL", 2: "MSF_ENOMEM", 3: "MSF_EDEVICE",
                4: "MSF_EBUDGET", 5: "MSF_ENOTFOUND"}

EXPORTS = [
    "msf_ctx_create", "msf_ctx_destroy", "msf_last_error", "msf_version", "msf_solve",
    "msf_get_stats", "msf_graph_create", "msf_graph_destroy", "msf_multilinear",
    "msf_multilinear_pairwise", "msf_shortcut_strategy", "msf_components",
    "msf_solve_starcheck",
    "msf_shortcut", "msf_solve_batched", "msf_server_create", "msf_server_destroy",
    "msf_server_submit", "msf_server_poll", "msf_server_latency", "msf_server_result",
    "msf_request_footprint", "msf_batch_configs", "msf_solve_batched_noalloc",
    "msf_multilinear_rows", "msf_graph_order",
]


class MSFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Total(ctypes.Structure):
    _fields_ = [("u64", ctypes.c_uint64), ("f64", ctypes.c_double)]


class BatchTotals(Sequence):
    """Per-graph totals of a batched solve as (u64, f64) pairs, read from the
    library's output array on access (no per-graph conversion up front)."""

    def __init__(self, arr, n: int):
        self._a = np.frombuffer(arr, dtype=np.dtype([("u64", "<u8"), ("f64", "<f8")]),
                                count=n)

    def __len__(self) -> int:
        return len(self._a)

    def __getitem__(self, g):
        if isinstance(g, slice):
            return [self[i] for i in range(*g.indices(len(self)))]
        x = self._a[g]
        return (int(x["u64"]), float(x["f64"]))


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("hook_rounds", ctypes.c_int32),
                ("max_chase", ctypes.c_int32), ("filtered", ctypes.c_int32),
                ("hooks", ctypes.c_int64 * 64), ("active_nnz", ctypes.c_int64 * 64),
                ("build_ms", ctypes.c_double), ("rounds_ms", ctypes.c_double),
                ("sweep_ms", ctypes.c_double * 64), ("sweep_bytes", ctypes.c_double * 64),
                ("head_sweeps", ctypes.c_int32), ("path", ctypes.c_int32),
                ("runs", ctypes.c_int64), ("pass_ms", ctypes.c_double * 4),
                ("pass_bytes", ctypes.c_double * 4), ("batch_config", ctypes.c_int32),
                ("batch_grid", ctypes.c_int32), ("batch_graphs", ctypes.c_int64),
                ("batch_large", ctypes.c_int64), ("batch_ms", ctypes.c_double),
                ("roots", ctypes.c_int64 * 64), ("adjacency_ms", ctypes.c_double)]


_lib = None


def lib():
    """Load ``libmsf.so``; raise if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO_PATH):
        raise MSFError(3, f"{SO_PATH} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(SO_PATH)
    P, I32, I64, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    st = ctypes.c_int
    L.msf_ctx_create.argtypes = [ctypes.c_int, P, ctypes.POINTER(P)]
    L.msf_ctx_create.restype = st
    L.msf_ctx_destroy.argtypes = [P]
    L.msf_ctx_destroy.restype = None
    L.msf_last_error.restype = ctypes.c_char_p
    L.msf_version.restype = ctypes.c_char_p
    L.msf_solve.argtypes = [P, I32, I64, P, P, ctypes.c_int, ctypes.c_int, P,
                            ctypes.POINTER(I64), ctypes.POINTER(Total)]
    L.msf_solve.restype = st
    L.msf_get_stats.argtypes = [P, ctypes.POINTER(Stats)]
    L.msf_get_stats.restype = st
    L.msf_graph_create.argtypes = [P, I32, I64, P, P, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(P)]
    L.msf_graph_create.restype = st
    L.msf_graph_destroy.argtypes = [P]
    L.msf_graph_destroy.restype = None
    L.msf_multilinear.argtypes = [P, P, P, P]
    L.msf_multilinear.restype = st
    L.msf_multilinear_pairwise.argtypes = [P, P, P, P]
    L.msf_multilinear_pairwise.restype = st
    L.msf_multilinear_rows.argtypes = [P, P, P, P, I32, I32]
    L.msf_multilinear_rows.restype = st
    L.msf_graph_order.argtypes = [P, P, P]
    L.msf_graph_order.restype = st
    L.msf_shortcut.argtypes = [P, I32, P, ctypes.POINTER(I32)]
    L.msf_shortcut.restype = st
    L.msf_shortcut_strategy.argtypes = [P, I32, P, I32, ctypes.c_double, ctypes.POINTER(I32)]
    L.msf_shortcut_strategy.restype = st
    L.msf_components.argtypes = [P, P, P, ctypes.POINTER(I32)]
    L.msf_components.restype = st
    L.msf_solve_starcheck.argtypes = [P, P, P, ctypes.POINTER(I32)]
    L.msf_solve_starcheck.restype = st
    L.msf_solve_batched.argtypes = [P, I32, P, P, P, P, ctypes.c_int, ctypes.c_int, P, P, P]
    L.msf_solve_batched.restype = st
    L.msf_server_create.argtypes = [P, ctypes.c_size_t, ctypes.POINTER(P)]
    L.msf_server_create.restype = st
    L.msf_server_destroy.argtypes = [P]
    L.msf_server_destroy.restype = None
    L.msf_server_submit.argtypes = [P, I32, I64, P, P, ctypes.c_int, ctypes.POINTER(U64)]
    L.msf_server_submit.restype = st
    L.msf_server_poll.argtypes = [P, U64, ctypes.POINTER(ctypes.c_int)]
    L.msf_server_poll.restype = st
    L.msf_server_latency.argtypes = [P, U64, ctypes.POINTER(ctypes.c_double)]
    L.msf_server_latency.restype = st
    L.msf_server_result.argtypes = [P, U64, P, ctypes.POINTER(I64), ctypes.POINTER(Total)]
    L.msf_server_result.restype = st
    L.msf_request_footprint.argtypes = [I32, I64]
    L.msf_request_footprint.restype = ctypes.c_size_t
    L.msf_batch_configs.argtypes = [P, P, P, I32]
    L.msf_batch_configs.restype = ctypes.c_int
    L.msf_solve_batched_noalloc.argtypes = [P, I32, P, P, P, P, ctypes.c_int, P, P, P]
    L.msf_solve_batched_noalloc.restype = st
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        raise MSFError(rc, lib().msf_last_error().decode())


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _wtype_of(w) -> int:
    name = str(w.dtype)
    if "float32" in name:
        return W_F32
    if "uint32" in name or "int32" in name:
        return W_U32
    raise TypeError(f"weights must be uint32 or float32, got {w.dtype}")


def _dev(t, name: str, numel: int, elem: int):
    """Check a device tensor before its pointer reaches the library: on the
    GPU, contiguous, `elem`-byte elements, at least `numel` of them.  The
    kernels write every one of those elements, so anything smaller would be
    an out-of-bounds device write."""
    if not _is_torch(t):
        raise MSFError(1, f"{name} must be a device tensor")
    if not t.is_cuda:
        raise MSFError(1, f"{name} must be on the GPU")
    if not t.is_contiguous():
        raise MSFError(1, f"{name} must be contiguous")
    if t.element_size() != elem:
        raise MSFError(1, f"{name} must have {elem}-byte elements, got {t.dtype}")
    if t.numel() < numel:
        raise MSFError(1, f"{name} holds {t.numel()} elements, needs {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _host(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def batch_configs() -> list:
    """The batched solve's launch configurations: (threads per workgroup,
    edges per thread and step, dynamic LDS bytes), in index order."""
    L = lib()
    k = L.msf_batch_configs(None, None, None, 0)
    a = (ctypes.c_int32 * k)()
    b = (ctypes.c_int32 * k)()
    c = (ctypes.c_int32 * k)()
    L.msf_batch_configs(a, b, c, k)
    return [(a[i], b[i], c[i]) for i in range(k)]


def footprint(n: int, m: int) -> int:
    """Device bytes a served request of this size occupies while resident."""
    return int(lib().msf_request_footprint(n, m))


# Live contexts, released (with their graphs and servers) at interpreter
# exit, before module teardown: handles left open (by an exception, say)
# are not freed by finalisers running in an unspecified order.
_LIVE = weakref.WeakSet()


@atexit.register
def _release_all():
    for c in list(_LIVE):
        c.close()


class Context:
    """An ``msf_ctx`` on one HIP device, ordered on one stream."""

    def __init__(self, device: int = 0, stream=None):
        L = lib()
        if stream is None:
            try:
                import torch
                if torch.cuda.is_available():
                    torch.cuda.set_device(device)
                    stream = torch.cuda.current_stream().cuda_stream
            except ImportError:
                stream = None
        h = ctypes.c_void_p()
        _check(L.msf_ctx_create(device, ctypes.c_void_p(stream or 0), ctypes.byref(h)))
        self._h = h
        self.device = device
        # graphs and servers made on this context: released before it
        self._children = weakref.WeakSet()
        _LIVE.add(self)

    def close(self):
        for ch in list(getattr(self, "_children", ())):
            ch.close()
        if getattr(self, "_h", None) is not None and self._h.value and _lib is not None:
            _lib.msf_ctx_destroy(self._h)
        self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------ solve --
    def solve(self, n: int, edges, weights, wtype: int | None = None, out=None):
        """Minimum spanning forest.  Host (numpy) or device (torch) inputs.

        Returns (ids, count, (total_u64, total_f64)); ``ids`` is a numpy
        int32 array for host inputs, a torch int32 tensor (length count) for
        device inputs (``out`` may supply a device buffer of >= n-1)."""
        L = lib()
        wt = _wtype_of(weights) if wtype is None else wtype
        cnt = ctypes.c_int64()
        tot = Total()
        if _is_torch(edges):
            import torch
            m = edges.numel() // 2
            ids = out if out is not None else torch.empty(max(n - 1, 1), dtype=torch.int32,
                                                          device=edges.device)
            pe = _dev(edges, "edges", 2 * m, 4)
            pw = _dev(weights, "weights", m, 4)
            pi = _dev(ids, "out", max(n - 1, 1) if m > 0 else 0, 4)
            _check(L.msf_solve(self._h, n, m, pe, pw, wt, MEM_DEVICE, pi, ctypes.byref(cnt),
                               ctypes.byref(tot)))
            return ids[:cnt.value], cnt.value, (tot.u64, tot.f64)
        e = _host(edges, np.int32).reshape(-1)
        w = _host(weights, np.float32 if wt == W_F32 else np.uint32)
        m = len(w)
        if e.size != 2 * m:
            raise ValueError("edges must hold 2*m int32 values")
        ids = np.empty(max(n - 1, 1), dtype=np.int32)
        _check(L.msf_solve(self._h, n, m, ctypes.c_void_p(e.ctypes.data),
                           ctypes.c_void_p(w.ctypes.data), wt, MEM_HOST,
                           ctypes.c_void_p(ids.ctypes.data), ctypes.byref(cnt), ctypes.byref(tot)))
        return ids[:cnt.value].copy(), cnt.value, (tot.u64, tot.f64)

    def stats(self) -> dict:
        s = Stats()
        _check(lib().msf_get_stats(self._h, ctypes.byref(s)))
        k = min(s.rounds, 64)
        return dict(rounds=s.rounds, hook_rounds=s.hook_rounds, max_chase=s.max_chase,
                    filtered=s.filtered, hooks=list(s.hooks[:k]),
                    active_nnz=list(s.active_nnz[:k]), build_ms=s.build_ms,
                    rounds_ms=s.rounds_ms, sweep_ms=list(s.sweep_ms[:k]), path=s.path,
                    sweep_bytes=list(s.sweep_bytes[:k]), head_sweeps=s.head_sweeps,
                    runs=s.runs, pass_ms=list(s.pass_ms), pass_bytes=list(s.pass_bytes),
                    batch_config=s.batch_config, batch_grid=s.batch_grid,
                    batch_graphs=s.batch_graphs, batch_large=s.batch_large,
                    batch_ms=s.batch_ms, roots=list(s.roots[:k]),
                    adjacency_ms=s.adjacency_ms)

    # ------------------------------------------------------- primitives --
    def graph(self, n: int, edges, weights, wtype: int | None = None) -> "Graph":
        return Graph(self, n, edges, weights, wtype)

    def multilinear(self, g: "Graph", p, r):
        """r[k] = min key over stored directions i->j with p[i]==k != p[j].

        p: device int32/uint32 tensor [n]; r: device int64 tensor [n]
        (bit pattern of uint64 keys).  Stream-ordered."""
        _check(lib().msf_multilinear(self._h, g._h, _dev(p, "p", g.n, 4),
                                     _dev(r, "r", g.n, 8)))

    def multilinear_rows(self, g: "Graph", p, r, row_lo: int, row_hi: int):
        """multilinear() over the stored rows row_lo .. row_hi - 1 only (one
        owner's share when the rows are split); arguments as for
        multilinear, rows in the graph's stored order (graph_order)."""
        _check(lib().msf_multilinear_rows(self._h, g._h, _dev(p, "p", g.n, 4),
                                          _dev(r, "r", g.n, 8), int(row_lo), int(row_hi)))

    def graph_order(self, g: "Graph", order):
        """order[k] = caller id of the vertex stored as row k, into a device
        int32/uint32 tensor [n]."""
        _check(lib().msf_graph_order(self._h, g._h, _dev(order, "order", g.n, 4)))

    def multilinear_pairwise(self, g: "Graph", p, r):
        """The same r by the pairwise formulation (pairs (a_ij, p_j) stored
        first, then reduced).  Arguments as for multilinear."""
        _check(lib().msf_multilinear_pairwise(self._h, g._h, _dev(p, "p", g.n, 4),
                                              _dev(r, "r", g.n, 8)))

    def shortcut_strategy(self, p, strategy: int, switch_fraction: float = 0.0) -> int:
        """shortcut() by a chosen strategy (SHORTCUT_FRONTIER / _FULL / _SWITCH);
        returns the number of passes."""
        it = ctypes.c_int32()
        _check(lib().msf_shortcut_strategy(self._h, p.numel(), _dev(p, "p", p.numel(), 4),
                                           strategy, switch_fraction, ctypes.byref(it)))
        return it.value

    def components(self, g: "Graph", labels) -> int:
        """Connected-component labels of g into a device int32/uint32 tensor
        [n] (equal labels iff connected); returns the number of rounds."""
        it = ctypes.c_int32()
        _check(lib().msf_components(self._h, g._h, _dev(labels, "labels", g.n, 4),
                                    ctypes.byref(it)))
        return it.value

    def solve_starcheck(self, g: "Graph", in_forest) -> int:
        """Forest flags (device uint8 tensor [m]) by the original AS rounds
        with star check and one-step shortcut; returns the number of rounds."""
        it = ctypes.c_int32()
        _check(lib().msf_solve_starcheck(self._h, g._h, _dev(in_forest, "in_forest", g.m, 1),
                                         ctypes.byref(it)))
        return it.value

    def shortcut(self, p) -> int:
        """p <- root of each vertex (device int32/uint32 tensor, in place);
        returns the number of pointer-jumping passes."""
        it = ctypes.c_int32()
        _check(lib().msf_shortcut(self._h, p.numel(), _dev(p, "p", p.numel(), 4),
                                  ctypes.byref(it)))
        return it.value

    # ----------------------------------------------------------- batched --
    def solve_batched(self, vtx_off, edge_off, edges, weights, wtype: int | None = None,
                      out=None):
        """Solve G graphs at once.  Returns (ids, counts, totals) where graph
        g's local forest ids are ids[vtx_off[g] : vtx_off[g] + counts[g]] and
        totals is a list of (u64, f64)."""
        L = lib()
        vo = _host(vtx_off, np.int64)
        eo = _host(edge_off, np.int64)
        G = len(vo) - 1
        wt = _wtype_of(weights) if wtype is None else wtype
        counts = np.zeros(max(G, 1), dtype=np.int64)
        totals = (Total * max(G, 1))()
        N = int(vo[-1]) if G > 0 else 0
        if _is_torch(edges):
            import torch
            ids = out if out is not None else torch.empty(max(N, 1), dtype=torch.int32,
                                                          device=edges.device)
            M = int(eo[-1]) if G > 0 else 0
            _check(L.msf_solve_batched(self._h, G, ctypes.c_void_p(vo.ctypes.data),
                                       ctypes.c_void_p(eo.ctypes.data),
                                       _dev(edges, "edges", 2 * M, 4),
                                       _dev(weights, "weights", M, 4), wt, MEM_DEVICE,
                                       _dev(ids, "out", N, 4),
                                       ctypes.c_void_p(counts.ctypes.data), totals))
        else:
            e = _host(edges, np.int32).reshape(-1)
            w = _host(weights, np.float32 if wt == W_F32 else np.uint32)
            ids = np.empty(max(N, 1), dtype=np.int32)
            _check(L.msf_solve_batched(self._h, G, ctypes.c_void_p(vo.ctypes.data),
                                       ctypes.c_void_p(eo.ctypes.data),
                                       ctypes.c_void_p(e.ctypes.data),
                                       ctypes.c_void_p(w.ctypes.data), wt, MEM_HOST,
                                       ctypes.c_void_p(ids.ctypes.data),
                                       ctypes.c_void_p(counts.ctypes.data), totals))
        return ids, counts[:G], BatchTotals(totals, G)


def solve_batched_noalloc(ctx: "Context", vtx_off, edge_off, edges, weights, wtype: int,
                          out, counts, totals):
    """msf_solve_batched_noalloc: every argument a device tensor (offsets and
    counts int64, totals int64 [G, 2] holding msf_total's u64 and f64 bits);
    the library allocates nothing.  Stream-ordered after its checks."""
    G = vtx_off.numel() - 1
    N = int(vtx_off[-1].item()) if G > 0 else 0
    M = int(edge_off[-1].item()) if G > 0 else 0
    _check(lib().msf_solve_batched_noalloc(
        ctx._h, G, _dev(vtx_off, "vtx_off", G + 1, 8), _dev(edge_off, "edge_off", G + 1, 8),
        _dev(edges, "edges", 2 * M, 4), _dev(weights, "weights", M, 4), wtype,
        _dev(out, "out", N, 4), _dev(counts, "counts", G, 8), _dev(totals, "totals", 2 * G, 8)))


class Graph:
    """An ``msf_graph``: the device adjacency structure of one graph."""

    def __init__(self, ctx: Context, n: int, edges, weights, wtype: int | None = None):
        L = lib()
        wt = _wtype_of(weights) if wtype is None else wtype
        h = ctypes.c_void_p()
        if _is_torch(edges):
            m = edges.numel() // 2
            _check(L.msf_graph_create(ctx._h, n, m, _dev(edges, "edges", 2 * m, 4),
                                      _dev(weights, "weights", m, 4), wt, MEM_DEVICE,
                                      ctypes.byref(h)))
        else:
            e = _host(edges, np.int32).reshape(-1)
            w = _host(weights, np.float32 if wt == W_F32 else np.uint32)
            m = len(w)
            if e.size != 2 * m:
                raise ValueError("edges must hold 2*m int32 values")
            _check(L.msf_graph_create(ctx._h, n, m, ctypes.c_void_p(e.ctypes.data),
                                      ctypes.c_void_p(w.ctypes.data), wt, MEM_HOST,
                                      ctypes.byref(h)))
        self._h = h
        self.n = n
        self.m = m
        self.ctx = ctx
        ctx._children.add(self)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value and _lib is not None:
            _lib.msf_graph_destroy(self._h)
        self._h = None

    __del__ = close


class Server:
    """Continuous-batching request loop (``msf_server_*``)."""

    def __init__(self, ctx: Context, mem_budget_bytes: int):
        h = ctypes.c_void_p()
        _check(lib().msf_server_create(ctx._h, mem_budget_bytes, ctypes.byref(h)))
        self._h = h
        self.ctx = ctx
        ctx._children.add(self)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value and _lib is not None:
            _lib.msf_server_destroy(self._h)
        self._h = None

    __del__ = close

    def submit(self, n: int, edges, weights, wtype: int | None = None) -> int:
        wt = _wtype_of(weights) if wtype is None else wtype
        e = _host(edges, np.int32).reshape(-1)
        w = _host(weights, np.float32 if wt == W_F32 else np.uint32)
        t = ctypes.c_uint64()
        _check(lib().msf_server_submit(self._h, n, len(w), ctypes.c_void_p(e.ctypes.data),
                                       ctypes.c_void_p(w.ctypes.data), wt, ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int()
        _check(lib().msf_server_poll(self._h, ticket, ctypes.byref(d)))
        return bool(d.value)

    def latency(self, ticket: int) -> float:
        s = ctypes.c_double()
        _check(lib().msf_server_latency(self._h, ticket, ctypes.byref(s)))
        return s.value

    def result(self, ticket: int, n: int):
        ids = np.empty(max(n - 1, 1), dtype=np.int32)
        cnt = ctypes.c_int64()
        tot = Total()
        _check(lib().msf_server_result(self._h, ticket, ctypes.c_void_p(ids.ctypes.data),
                                       ctypes.byref(cnt), ctypes.byref(tot)))
        return ids[:cnt.value].copy(), cnt.value, (tot.u64, tot.f64)
