"""ORACLE — test infrastructure only.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of the
bench may import this package.  The product library never links, loads or
calls it.  It shares no code with the HIP path: the two meet only through the
seeded inputs of the ``synth`` package.

Functions (all host-side, written from the paper, arXiv 1906.12018):

* :func:`canonical_labels` -- Definition 2 written out, one BFS per vertex.
* :func:`pll_labels`       -- Algorithm 1 (PLL) with the small revision of
  Section 2.1.1.
* :func:`pll_labels_budget` -- the same PLL stopped after a host-time budget
  (the first roots in rank order; a timing sample of a long build).
* :func:`bvc_labels`       -- Algorithm 4 (BVC-PLL) run sequentially with
  batch size b; b = 1 is PLL and b = n is VC-PLL (Algorithm 3).
* :func:`query`            -- the 2-hop distance formula of Section 2.1.
* :func:`pll_labels_directed`, :func:`query_directed` -- the directed variant
  of Section 5.1 (L_in and L_out labels; the query merges L_out(s), L_in(t)).
* :func:`pll_labels_weighted` -- PLL with Dijkstra for positive integer edge
  weights (Section 5.1; the weighted baseline of Section 6).  The query is
  :func:`query` unchanged.
* :func:`pll_labels_bp`, :func:`query_bp` -- bit-parallel labels (Section 5.2,
  adopted from the original PLL) followed by PLL over the remaining vertices.
* :func:`bfs`              -- textbook BFS distances.

Label sets are returned as :class:`Labels` (CSR by vertex id, hubs as ranks in
ascending order, uint8 distances).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pll_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

DIST_INF = 0xFFFFFFFF
OK, EINVAL, ENOMEM, EDIST = 0, 1, 2, 4


class OracleError(RuntimeError):
    pass


def build_native(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _CLabels(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint32),
        ("total", ctypes.c_uint64),
        ("offsets", ctypes.POINTER(ctypes.c_uint64)),
        ("hub_rank", ctypes.POINTER(ctypes.c_uint32)),
        ("dist", ctypes.POINTER(ctypes.c_uint8)),
        ("counters", ctypes.c_uint64 * 8),
    ]


class _CBp(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_uint32),
        ("root", ctypes.POINTER(ctypes.c_uint32)),
        ("nbr", ctypes.POINTER(ctypes.c_uint32)),
        ("dist", ctypes.POINTER(ctypes.c_uint8)),
        ("sm1", ctypes.POINTER(ctypes.c_uint64)),
        ("s0", ctypes.POINTER(ctypes.c_uint64)),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_native(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_pll.argtypes = [ctypes.c_uint32, P, P, P, ctypes.POINTER(_CLabels)]
        lib.oracle_pll.restype = ctypes.c_int
        lib.oracle_pll_budget.argtypes = [ctypes.c_uint32, P, P, P, ctypes.c_double,
                                          ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(_CLabels)]
        lib.oracle_pll_budget.restype = ctypes.c_int
        lib.oracle_bvc.argtypes = [ctypes.c_uint32, P, P, P, ctypes.c_uint32, ctypes.POINTER(_CLabels)]
        lib.oracle_bvc.restype = ctypes.c_int
        lib.oracle_canonical.argtypes = [ctypes.c_uint32, P, P, P, ctypes.c_uint32, P, ctypes.c_uint32,
                                         ctypes.POINTER(_CLabels)]
        lib.oracle_canonical.restype = ctypes.c_int
        lib.oracle_labels_free.argtypes = [ctypes.POINTER(_CLabels)]
        lib.oracle_labels_free.restype = None
        lib.oracle_bfs.argtypes = [ctypes.c_uint32, P, P, ctypes.c_uint32, P]
        lib.oracle_bfs.restype = None
        lib.oracle_query.argtypes = [P, P, P, ctypes.c_uint64, P, P, P, P]
        lib.oracle_query.restype = None
        lib.oracle_pll_directed.argtypes = [ctypes.c_uint32, P, P, P, ctypes.POINTER(_CLabels),
                                            ctypes.POINTER(_CLabels)]
        lib.oracle_pll_directed.restype = ctypes.c_int
        lib.oracle_query_directed.argtypes = [P, P, P, P, P, P, ctypes.c_uint64, P, P, P]
        lib.oracle_query_directed.restype = None
        lib.oracle_pll_weighted.argtypes = [ctypes.c_uint32, P, P, P, P, ctypes.POINTER(_CLabels)]
        lib.oracle_pll_weighted.restype = ctypes.c_int
        lib.oracle_pll_bp.argtypes = [ctypes.c_uint32, P, P, P, ctypes.c_uint32, ctypes.POINTER(_CLabels),
                                      ctypes.POINTER(_CBp)]
        lib.oracle_pll_bp.restype = ctypes.c_int
        lib.oracle_bp_free.argtypes = [ctypes.POINTER(_CBp)]
        lib.oracle_bp_free.restype = None
        lib.oracle_query_bp.argtypes = [P, P, P, ctypes.POINTER(_CBp), ctypes.c_uint64, P, P, P]
        lib.oracle_query_bp.restype = None
        _lib = lib
    return _lib


@dataclass
class Labels:
    """Label lists in CSR form.  List i belongs to vertex ``owners[i]``
    (``owners`` is None when list i belongs to vertex i).  ``hub_rank`` holds
    hub ranks, ascending within each list."""
    offsets: np.ndarray   # uint64[len+1]
    hub_rank: np.ndarray  # uint32[total]
    dist: np.ndarray      # uint8[total]
    counters: dict = field(default_factory=dict)
    owners: np.ndarray | None = None

    @property
    def total(self) -> int:
        return int(self.offsets[-1])

    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.int64)

    def of(self, i: int):
        a, b = int(self.offsets[i]), int(self.offsets[i + 1])
        return self.hub_rank[a:b], self.dist[a:b]

    def hubs_as_ids(self, order: np.ndarray) -> np.ndarray:
        return np.asarray(order, dtype=np.uint32)[self.hub_rank]


_COUNTER_NAMES = ["checks", "added", "edge_accesses", "rounds", "batches", "scanned", "cost_pos", "cost_neg"]


def _take(c: _CLabels) -> Labels:
    n = c.n
    total = c.total
    off = np.ctypeslib.as_array(c.offsets, shape=(n + 1,)).copy()
    hub = np.ctypeslib.as_array(c.hub_rank, shape=(max(total, 1),))[:total].copy()
    dist = np.ctypeslib.as_array(c.dist, shape=(max(total, 1),))[:total].copy()
    counters = {name: int(c.counters[i]) for i, name in enumerate(_COUNTER_NAMES)}
    _load().oracle_labels_free(ctypes.byref(c))
    return Labels(off, hub, dist, counters)


def _graph_args(g, order):
    row_ptr = np.ascontiguousarray(g.row_ptr, dtype=np.uint64)
    col = np.ascontiguousarray(g.col, dtype=np.uint32)
    order = np.ascontiguousarray(order, dtype=np.uint32)
    if order.shape[0] != g.n:
        raise OracleError("order must have n entries")
    return row_ptr, col, order


def _check(rc: int, what: str):
    if rc != OK:
        raise OracleError(f"{what} failed with status {rc}")


def pll_labels(g, order) -> Labels:
    """Algorithm 1 (PLL) labels; lists by vertex id, hubs as ranks."""
    row_ptr, col, order = _graph_args(g, order)
    c = _CLabels()
    _check(_load().oracle_pll(g.n, row_ptr.ctypes.data, col.ctypes.data, order.ctypes.data, ctypes.byref(c)),
           "oracle_pll")
    return _take(c)


def pll_labels_budget(g, order, seconds: float):
    """The PLL of :func:`pll_labels` run over the first roots in rank order
    until ``seconds`` of host time are spent (the root running then is
    finished).  Returns ``(labels, roots_done)``; the lists hold only hubs of
    rank below roots_done."""
    row_ptr, col, order = _graph_args(g, order)
    c = _CLabels()
    done = ctypes.c_uint32(0)
    _check(_load().oracle_pll_budget(g.n, row_ptr.ctypes.data, col.ctypes.data, order.ctypes.data, float(seconds),
                                     ctypes.byref(done), ctypes.byref(c)), "oracle_pll_budget")
    return _take(c), int(done.value)


def bvc_labels(g, order, b: int) -> Labels:
    """Algorithm 4 (BVC-PLL) labels with batch size b, run sequentially."""
    row_ptr, col, order = _graph_args(g, order)
    c = _CLabels()
    _check(_load().oracle_bvc(g.n, row_ptr.ctypes.data, col.ctypes.data, order.ctypes.data, b, ctypes.byref(c)),
           "oracle_bvc")
    return _take(c)


def canonical_labels(g, order, verts=None, threads: int = 1) -> Labels:
    """Definition 2 labels of ``verts`` (default: every vertex), one BFS each.
    List i of the result belongs to ``verts[i]``."""
    row_ptr, col, order = _graph_args(g, order)
    all_v = verts is None
    verts = np.arange(g.n, dtype=np.uint32) if all_v else np.ascontiguousarray(verts, dtype=np.uint32)
    c = _CLabels()
    _check(_load().oracle_canonical(g.n, row_ptr.ctypes.data, col.ctypes.data, order.ctypes.data, len(verts),
                                    verts.ctypes.data, threads, ctypes.byref(c)), "oracle_canonical")
    lab = _take(c)
    if not all_v:
        lab.owners = verts
    return lab


def bfs(g, src: int) -> np.ndarray:
    row_ptr = np.ascontiguousarray(g.row_ptr, dtype=np.uint64)
    col = np.ascontiguousarray(g.col, dtype=np.uint32)
    out = np.empty(g.n, dtype=np.uint32)
    _load().oracle_bfs(g.n, row_ptr.ctypes.data, col.ctypes.data, src, out.ctypes.data)
    return out


def query(labels: Labels, u, v, with_consumed: bool = False):
    """Dis(u,v) for each pair (uint32; DIST_INF when no common hub)."""
    if labels.owners is not None:
        raise OracleError("query needs lists indexed by vertex id")
    u = np.ascontiguousarray(u, dtype=np.uint32)
    v = np.ascontiguousarray(v, dtype=np.uint32)
    out = np.empty(u.shape[0], dtype=np.uint32)
    cons = np.empty(u.shape[0], dtype=np.uint64) if with_consumed else None
    off = np.ascontiguousarray(labels.offsets, dtype=np.uint64)
    hub = np.ascontiguousarray(labels.hub_rank, dtype=np.uint32)
    dist = np.ascontiguousarray(labels.dist, dtype=np.uint8)
    _load().oracle_query(off.ctypes.data, hub.ctypes.data if hub.size else None,
                         dist.ctypes.data if dist.size else None, u.shape[0], u.ctypes.data, v.ctypes.data,
                         out.ctypes.data, cons.ctypes.data if cons is not None else None)
    return (out, cons) if with_consumed else out


def pll_labels_directed(g, order):
    """Directed PLL (Section 5.1) on the arcs of ``g`` (row v lists the heads
    of the arcs leaving v).  Returns ``(L_in, L_out)``: L_in(v) holds
    (u, d(u,v)), L_out(v) holds (u, d(v,u)); lists by vertex id, hubs as
    ranks.  Counters: L_in's are the forward searches', L_out's the backward
    searches'."""
    row_ptr, col, order = _graph_args(g, order)
    cin, cout = _CLabels(), _CLabels()
    _check(_load().oracle_pll_directed(g.n, row_ptr.ctypes.data, col.ctypes.data, order.ctypes.data,
                                       ctypes.byref(cin), ctypes.byref(cout)), "oracle_pll_directed")
    return _take(cin), _take(cout)


def query_directed(lin: Labels, lout: Labels, s, t):
    """d(s, t) for each pair: min over hubs of L_out(s) and L_in(t) (uint32;
    DIST_INF when t is unreachable from s)."""
    s = np.ascontiguousarray(s, dtype=np.uint32)
    t = np.ascontiguousarray(t, dtype=np.uint32)
    out = np.empty(s.shape[0], dtype=np.uint32)
    arrs = []
    for lab in (lout, lin):
        arrs += [np.ascontiguousarray(lab.offsets, dtype=np.uint64), np.ascontiguousarray(lab.hub_rank, dtype=np.uint32),
                 np.ascontiguousarray(lab.dist, dtype=np.uint8)]
    ptr = [a.ctypes.data if a.size else None for a in arrs]
    _load().oracle_query_directed(*ptr, s.shape[0], s.ctypes.data, t.ctypes.data, out.ctypes.data)
    return out


def pll_labels_weighted(g, order) -> Labels:
    """PLL with Dijkstra on the weighted graph ``g`` (``g.w``: uint8 weight of
    each CSR entry, >= 1, equal on both arcs of an edge); lists by vertex id,
    hubs as ranks, distances uint8 (a kept distance of 255 or more raises)."""
    row_ptr, col, order = _graph_args(g, order)
    w = np.ascontiguousarray(g.w, dtype=np.uint8)
    if w.shape[0] != col.shape[0]:
        raise OracleError("one weight per CSR entry")
    c = _CLabels()
    _check(_load().oracle_pll_weighted(g.n, row_ptr.ctypes.data, col.ctypes.data, w.ctypes.data,
                                       order.ctypes.data, ctypes.byref(c)), "oracle_pll_weighted")
    return _take(c)


@dataclass
class BPLabels:
    """Bit-parallel labels: BP root i is vertex ``root[i]`` with neighbour set
    ``nbr[i]`` (vertex ids, bit j = nbr[i][j]; DIST_INF past the set);
    ``dist[v, i]`` = d(root_i, v) (255: unreachable), ``sm1[v, i]`` and
    ``s0[v, i]`` the S^-1 and S^0 bit sets."""
    root: np.ndarray  # uint32[t]
    nbr: np.ndarray   # uint32[t, 64]
    dist: np.ndarray  # uint8[n, t]
    sm1: np.ndarray   # uint64[n, t]
    s0: np.ndarray    # uint64[n, t]

    @property
    def t(self) -> int:
        return int(self.root.shape[0])


def pll_labels_bp(g, order, t: int):
    """Up to t BP roots (each with up to 64 neighbours), then PLL over the
    vertices they did not use, pruning by the BP bound first.  Returns
    (Labels, BPLabels); the labels' counter "bp_pruned" counts the checks the
    BP bound decided."""
    row_ptr, col, order = _graph_args(g, order)
    c, b = _CLabels(), _CBp()
    lib = _load()
    _check(lib.oracle_pll_bp(g.n, row_ptr.ctypes.data, col.ctypes.data, order.ctypes.data, t, ctypes.byref(c),
                             ctypes.byref(b)), "oracle_pll_bp")
    tt, n = b.t, g.n
    bp = BPLabels(
        root=np.ctypeslib.as_array(b.root, shape=(max(tt, 1),))[:tt].copy(),
        nbr=np.ctypeslib.as_array(b.nbr, shape=(max(tt, 1) * 64,))[:tt * 64].copy().reshape(tt, 64),
        dist=np.ctypeslib.as_array(b.dist, shape=(n * tt + 1,))[:n * tt].copy().reshape(n, tt),
        sm1=np.ctypeslib.as_array(b.sm1, shape=(n * tt + 1,))[:n * tt].copy().reshape(n, tt),
        s0=np.ctypeslib.as_array(b.s0, shape=(n * tt + 1,))[:n * tt].copy().reshape(n, tt))
    lib.oracle_bp_free(ctypes.byref(b))
    lab = _take(c)
    lab.counters["bp_pruned"] = lab.counters.pop("cost_pos")
    lab.counters.pop("cost_neg", None)
    return lab, bp


def query_bp(labels: Labels, bp: BPLabels, u, v):
    """min(BP bound, 2-hop merge) for each pair (uint32; DIST_INF when none)."""
    u = np.ascontiguousarray(u, dtype=np.uint32)
    v = np.ascontiguousarray(v, dtype=np.uint32)
    out = np.empty(u.shape[0], dtype=np.uint32)
    off = np.ascontiguousarray(labels.offsets, dtype=np.uint64)
    hub = np.ascontiguousarray(labels.hub_rank, dtype=np.uint32)
    dist = np.ascontiguousarray(labels.dist, dtype=np.uint8)
    keep = [np.ascontiguousarray(bp.root, dtype=np.uint32), np.ascontiguousarray(bp.nbr, dtype=np.uint32),
            np.ascontiguousarray(bp.dist, dtype=np.uint8), np.ascontiguousarray(bp.sm1, dtype=np.uint64),
            np.ascontiguousarray(bp.s0, dtype=np.uint64)]
    cb = _CBp(bp.t, *(a.ctypes.data_as(ctypes.POINTER(ct)) for a, ct in
                      zip(keep, (ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint8, ctypes.c_uint64, ctypes.c_uint64))))
    _load().oracle_query_bp(off.ctypes.data, hub.ctypes.data if hub.size else None,
                            dist.ctypes.data if dist.size else None, ctypes.byref(cb), u.shape[0], u.ctypes.data,
                            v.ctypes.data, out.ctypes.data)
    return out
