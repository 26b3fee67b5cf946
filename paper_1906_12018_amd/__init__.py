"""MI355X (gfx950) pruned landmark labeling: Python binding of libpll.

Argument marshalling only: every step of label construction and querying runs
in the HIP kernels of ``libpll.so`` (declared in ``include/pll.h``).  PyTorch
supplies device memory and the current stream.  There is no CPU fallback; if
the library is not built, or no GPU is present, calls raise :class:`PllError`.

Paper: Jin et al., "Pruned Landmark Labeling Meets Vertex Centric
Computation" (arXiv 1906.12018): BVC-PLL (Section 4.2, Algorithm 4) builds the
canonical 2-hop labeling (Definition 2) for a vertex order; the 2-hop query
(Section 2.1) merges two hub-sorted lists.  Directed graphs (Section 5.1) get
L_in and L_out labels, and the query merges L_out(u) with L_in(v); weighted
graphs (Section 5.1) run the rounds as Bellman-Ford iterations with a
batch-end recheck.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpll.so")

PLL_OK, PLL_EINVAL, PLL_ENOMEM, PLL_ENOSPC, PLL_EDIST, PLL_EDEVICE, PLL_ESCRATCH = 0, 1, 2, 3, 4, 5, 6
DIST_INF = 0xFFFFFFFF
FLAG_VALIDATE, FLAG_RECHECK, FLAG_RELAXED, FLAG_PROFILE, FLAG_PERSISTENT, FLAG_PACK4 = 0x1, 0x2, 0x4, 0x8, 0x10, 0x20
PHASES = ("prep", "init", "push", "check", "end", "final", "loop")
DEFAULT_BATCH = 1024
LABELS_IN, LABELS_OUT = 0, 1

EXPORTED_SYMBOLS = (
    "pll_build_labels", "pll_build_labels_directed", "pll_build_labels_weighted", "pll_query", "pll_index_info_get", "pll_export_labels",
    "pll_export_labels_side", "pll_export_bp", "pll_index_set_query_lanes",
    "pll_build_labels_batched", "pll_index_free", "pll_status_string",
    "pll_server_create", "pll_server_add_index", "pll_server_index", "pll_server_submit", "pll_server_poll",
    "pll_server_replay", "pll_server_destroy", "pll_bench_stream_read", "pll_build_labels_noalloc",
)
REQ_QUERY, REQ_BUILD = 0, 1


class PllError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        msg = status_string(status) if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} (status {status})")


class BuildOpts(ctypes.Structure):
    _fields_ = [
        ("batch_size", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("arena_entries", ctypes.c_uint64),
        ("query_lanes", ctypes.c_uint32),
        ("gang_scale", ctypes.c_uint32),
        ("max_gang", ctypes.c_uint32),
        ("max_workgroups", ctypes.c_uint32),
        ("bp_roots", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32 * 3),
    ]


class IndexInfo(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint32),
        ("batch_size", ctypes.c_uint32),
        ("total_entries", ctypes.c_uint64),
        ("label_bytes", ctypes.c_uint64),
        ("max_dist", ctypes.c_uint32),
        ("max_label", ctypes.c_uint32),
        ("batches", ctypes.c_uint64),
        ("rounds", ctypes.c_uint64),
        ("candidates", ctypes.c_uint64),
        ("accepted", ctypes.c_uint64),
        ("edges_scanned", ctypes.c_uint64),
        ("recheck_removed", ctypes.c_uint64),
        ("arena_entries", ctypes.c_uint64),
        ("build_attempts", ctypes.c_uint32),
        ("gang", ctypes.c_uint32),
        ("build_ms", ctypes.c_double),
        ("check_entries_read", ctypes.c_uint64),
        ("check_table_reads", ctypes.c_uint64),
        ("check_cost_pos", ctypes.c_uint64),
        ("check_cost_neg", ctypes.c_uint64),
        ("phase_ms", ctypes.c_double * 7),
        ("phase_launches", ctypes.c_uint64 * 7),
        ("directed", ctypes.c_uint32),
        ("weighted", ctypes.c_uint32),
        ("in_entries", ctypes.c_uint64),
        ("out_entries", ctypes.c_uint64),
        ("bp_roots", ctypes.c_uint32),
        ("bp_vertices", ctypes.c_uint32),
        ("bp_pruned", ctypes.c_uint64),
        ("check_push_edges", ctypes.c_uint64),
        ("query_lanes", ctypes.c_uint32),
    ]

    def as_dict(self) -> dict:
        d = {}
        for name, _ in self._fields_:
            if name.startswith("reserved"):
                continue
            val = getattr(self, name)
            if name.startswith("phase_"):
                val = dict(zip(PHASES, list(val)))
            d[name] = val
        return d


class GraphDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint32),
        ("nnz", ctypes.c_uint64),
        ("d_row_ptr", ctypes.c_void_p),
        ("d_col", ctypes.c_void_p),
        ("d_order", ctypes.c_void_p),
    ]


class ServerOpts(ctypes.Structure):
    _fields_ = [
        ("slots", ctypes.c_uint32),
        ("build_batch_size", ctypes.c_uint32),
        ("max_batch_pairs", ctypes.c_uint64),
        ("mem_reserve", ctypes.c_uint64),
        ("build_workgroups", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32 * 3),
    ]


class Request(ctypes.Structure):
    _fields_ = [
        ("at", ctypes.c_double),
        ("kind", ctypes.c_uint32),
        ("index_id", ctypes.c_uint32),
        ("count", ctypes.c_uint64),
        ("h_u", ctypes.c_void_p),
        ("h_v", ctypes.c_void_p),
        ("h_out", ctypes.c_void_p),
        ("n", ctypes.c_uint32),
        ("reserved0", ctypes.c_uint32),
        ("nnz", ctypes.c_uint64),
        ("h_row_ptr", ctypes.c_void_p),
        ("h_col", ctypes.c_void_p),
        ("h_order", ctypes.c_void_p),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_uint64),
        ("status", ctypes.c_int32),
        ("kind", ctypes.c_uint32),
        ("index_id", ctypes.c_uint32),
        ("batch_requests", ctypes.c_uint32),
        ("t_arrival", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
        ("t_dev_start", ctypes.c_double),
        ("t_dev_end", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpll.so; raises if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise PllError(PLL_EDEVICE, f"{path} is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    P, U32, U64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
    lib.pll_build_labels.argtypes = [U32, U64, P, P, P, ctypes.POINTER(BuildOpts), P, ctypes.POINTER(P)]
    lib.pll_build_labels.restype = ctypes.c_int
    lib.pll_query.argtypes = [P, U64, P, P, P, P]
    lib.pll_query.restype = ctypes.c_int
    lib.pll_index_info_get.argtypes = [P, ctypes.POINTER(IndexInfo)]
    lib.pll_index_info_get.restype = ctypes.c_int
    lib.pll_export_labels.argtypes = [P, P, P, P, P]
    lib.pll_export_labels.restype = ctypes.c_int
    lib.pll_export_labels_side.argtypes = [P, U32, P, P, P, P]
    lib.pll_export_labels_side.restype = ctypes.c_int
    lib.pll_export_bp.argtypes = [P, P, P, P, P, P, P]
    lib.pll_export_bp.restype = ctypes.c_int
    lib.pll_index_set_query_lanes.argtypes = [P, U32]
    lib.pll_index_set_query_lanes.restype = ctypes.c_int
    lib.pll_build_labels_directed.argtypes = [U32, U64, P, P, P, ctypes.POINTER(BuildOpts), P, ctypes.POINTER(P)]
    lib.pll_build_labels_directed.restype = ctypes.c_int
    lib.pll_build_labels_weighted.argtypes = [U32, U64, P, P, P, P, ctypes.POINTER(BuildOpts), P, ctypes.POINTER(P)]
    lib.pll_build_labels_weighted.restype = ctypes.c_int
    lib.pll_export_labels.restype = ctypes.c_int
    lib.pll_build_labels_batched.argtypes = [U32, ctypes.POINTER(GraphDesc), ctypes.POINTER(BuildOpts), P,
                                             ctypes.POINTER(P)]
    lib.pll_build_labels_batched.restype = ctypes.c_int
    lib.pll_index_free.argtypes = [P]
    lib.pll_index_free.restype = None
    lib.pll_status_string.argtypes = [ctypes.c_int]
    lib.pll_status_string.restype = ctypes.c_char_p
    lib.pll_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(P)]
    lib.pll_server_create.restype = ctypes.c_int
    lib.pll_server_add_index.argtypes = [P, P, ctypes.c_int, ctypes.POINTER(ctypes.c_uint32)]
    lib.pll_server_add_index.restype = ctypes.c_int
    lib.pll_server_index.argtypes = [P, ctypes.c_uint32, ctypes.POINTER(P)]
    lib.pll_server_index.restype = ctypes.c_int
    lib.pll_server_submit.argtypes = [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    lib.pll_server_submit.restype = ctypes.c_int
    lib.pll_server_poll.argtypes = [P, ctypes.POINTER(Result), ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32),
                                    ctypes.c_int]
    lib.pll_server_poll.restype = ctypes.c_int
    lib.pll_server_replay.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(Request), ctypes.POINTER(Result)]
    lib.pll_server_replay.restype = ctypes.c_int
    lib.pll_server_destroy.argtypes = [P]
    lib.pll_server_destroy.restype = None
    lib.pll_build_labels_noalloc.argtypes = [U32, U64, P, P, P, ctypes.POINTER(BuildOpts), P, P, P, P, U64,
                                             ctypes.POINTER(ctypes.c_uint64)]
    lib.pll_build_labels_noalloc.restype = ctypes.c_int
    lib.pll_bench_stream_read.argtypes = [P, U64, P, U32, P]
    lib.pll_bench_stream_read.restype = ctypes.c_int
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load_library().pll_status_string(status).decode()


def _stream_handle(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _dev(t: torch.Tensor, dtype: torch.dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise PllError(PLL_EINVAL, f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise PllError(PLL_EINVAL, f"{name} must be {dtype}")
    return t.contiguous()


def _opts(batch_size: int, flags: int, arena_entries: int, query_lanes: int, gang_scale: int = 0,
          max_gang: int = 0, max_workgroups: int = 0, bp_roots: int = 0) -> BuildOpts:
    o = BuildOpts()
    o.batch_size = batch_size
    o.flags = flags
    o.arena_entries = arena_entries
    o.query_lanes = query_lanes
    o.gang_scale = gang_scale
    o.max_gang = max_gang
    o.max_workgroups = max_workgroups
    o.bp_roots = bp_roots
    return o


@dataclass
class ExportedLabels:
    offsets: torch.Tensor  # uint64 as int64 [n+1], by vertex id
    hubs: torch.Tensor     # int32 view of uint32 vertex ids, ascending hub rank per list
    dists: torch.Tensor    # uint8


class Index:
    """A resident label index (owns its device memory until :meth:`free`)."""

    def __init__(self, handle: int, device: torch.device):
        self._h = ctypes.c_void_p(handle)
        self.device = device

    @property
    def handle(self) -> int:
        if not self._h:
            raise PllError(PLL_EINVAL, "index already freed")
        return self._h.value

    def info(self) -> dict:
        i = IndexInfo()
        rc = load_library().pll_index_info_get(self.handle, ctypes.byref(i))
        if rc:
            raise PllError(rc, "pll_index_info_get")
        return i.as_dict()

    def query(self, u: torch.Tensor, v: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Distances for pairs (u[i], v[i]); int32 tensors of vertex ids.
        Returns int32 (a uint32 bit pattern: DIST_INF reads as -1)."""
        u = _dev(u, torch.int32, "u")
        v = _dev(v, torch.int32, "v")
        if u.shape != v.shape or u.dim() != 1:
            raise PllError(PLL_EINVAL, "u and v must be 1-D and equal length")
        if out is None:
            out = torch.empty_like(u)
        else:
            out = _dev(out, torch.int32, "out")
            if out.shape != u.shape:
                raise PllError(PLL_EINVAL, "out has the wrong shape")
        rc = load_library().pll_query(self.handle, u.numel(), u.data_ptr(), v.data_ptr(), out.data_ptr(),
                                      _stream_handle(stream))
        if rc:
            raise PllError(rc, "pll_query")
        return out

    def export(self, side: int = 0, stream=None) -> ExportedLabels:
        """Labels in CSR form; ``side`` is LABELS_IN (L_in, the one label of an
        undirected index) or LABELS_OUT (L_out of a directed index)."""
        inf = self.info()
        n = inf["n"]
        total = inf["out_entries"] if side == LABELS_OUT else inf["in_entries"]
        off = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        hubs = torch.empty(max(total, 1), dtype=torch.int32, device=self.device)
        dists = torch.empty(max(total, 1), dtype=torch.uint8, device=self.device)
        rc = load_library().pll_export_labels_side(self.handle, side, off.data_ptr(), hubs.data_ptr(),
                                                   dists.data_ptr(), _stream_handle(stream))
        if rc:
            raise PllError(rc, "pll_export_labels_side")
        return ExportedLabels(off, hubs[:total], dists[:total])

    def set_query_lanes(self, lanes: int) -> None:
        """Lanes per pair of later queries (0 = automatic, 1, 4, ..., 64)."""
        rc = load_library().pll_index_set_query_lanes(self.handle, lanes)
        if rc:
            raise PllError(rc, "pll_index_set_query_lanes")

    def export_bp(self, stream=None) -> dict:
        """Bit-parallel part (vertex ids): roots [t], nbrs [t, 64] (-1 past a
        set), dist [n, t] uint8, sm1 / s0 [n, t] (int64 views of the uint64 sets)."""
        inf = self.info()
        n, t = inf["n"], inf["bp_roots"]
        dev = self.device
        roots = torch.empty(max(t, 1), dtype=torch.int32, device=dev)
        nbrs = torch.empty(max(t, 1) * 64, dtype=torch.int32, device=dev)
        dist = torch.empty(max(n * t, 1), dtype=torch.uint8, device=dev)
        sm1 = torch.empty(max(n * t, 1), dtype=torch.int64, device=dev)
        s0 = torch.empty(max(n * t, 1), dtype=torch.int64, device=dev)
        rc = load_library().pll_export_bp(self.handle, roots.data_ptr(), nbrs.data_ptr(), dist.data_ptr(),
                                          sm1.data_ptr(), s0.data_ptr(), _stream_handle(stream))
        if rc:
            raise PllError(rc, "pll_export_bp")
        return {"roots": roots[:t], "nbrs": nbrs[:t * 64].view(t, 64), "dist": dist[:n * t].view(n, t),
                "sm1": sm1[:n * t].view(n, t), "s0": s0[:n * t].view(n, t)}

    def free(self):
        if self._h:
            load_library().pll_index_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build_labels(row_ptr: torch.Tensor, col: torch.Tensor, order: torch.Tensor, batch_size: int = DEFAULT_BATCH,
                 flags: int = FLAG_VALIDATE, arena_entries: int = 0, query_lanes: int = 0, max_workgroups: int = 0,
                 bp_roots: int = 0, stream=None) -> Index:
    """Canonical 2-hop labels of the CSR graph (row_ptr int64 [n+1], col
    int32 [nnz], order int32 [n]: order[k] = vertex of rank k).  With
    bp_roots > 0, bit-parallel labels of that many roots come first and the
    stored labels cover only what they do not (Section 5.2)."""
    row_ptr = _dev(row_ptr, torch.int64, "row_ptr")
    col = _dev(col, torch.int32, "col")
    order = _dev(order, torch.int32, "order")
    n = order.numel()
    if row_ptr.numel() != n + 1:
        raise PllError(PLL_EINVAL, "row_ptr must have n+1 entries")
    h = ctypes.c_void_p()
    o = _opts(batch_size, flags, arena_entries, query_lanes, max_workgroups=max_workgroups, bp_roots=bp_roots)
    rc = load_library().pll_build_labels(n, col.numel(), row_ptr.data_ptr(), col.data_ptr(), order.data_ptr(),
                                         ctypes.byref(o), _stream_handle(stream), ctypes.byref(h))
    if rc:
        raise PllError(rc, "pll_build_labels")
    return Index(h.value, order.device)


def build_labels_noalloc(row_ptr: torch.Tensor, col: torch.Tensor, order: torch.Tensor, offsets: torch.Tensor,
                         hubs: torch.Tensor, dists: torch.Tensor, batch_size: int = DEFAULT_BATCH,
                         flags: int = FLAG_VALIDATE, stream=None) -> int:
    """pll_build_labels_noalloc: the labels of the graph written into the
    caller's device tensors (offsets int64 [n+1], hubs int32 [capacity],
    dists uint8 [capacity]) without any device allocation by the library.
    Returns the number of entries; raises PllError (its ``total`` attribute
    holds the entries needed when the status is PLL_ENOSPC)."""
    row_ptr = _dev(row_ptr, torch.int64, "row_ptr")
    col = _dev(col, torch.int32, "col")
    order = _dev(order, torch.int32, "order")
    offsets = _dev(offsets, torch.int64, "offsets")
    hubs = _dev(hubs, torch.int32, "hubs")
    dists = _dev(dists, torch.uint8, "dists")
    n = order.numel()
    if row_ptr.numel() != n + 1 or offsets.numel() != n + 1:
        raise PllError(PLL_EINVAL, "row_ptr and offsets must have n + 1 entries")
    cap = min(hubs.numel(), dists.numel())
    total = ctypes.c_uint64()
    o = _opts(batch_size, flags, 0, 0)
    rc = load_library().pll_build_labels_noalloc(n, col.numel(), row_ptr.data_ptr(), col.data_ptr(), order.data_ptr(),
                                                 ctypes.byref(o), _stream_handle(stream), offsets.data_ptr(),
                                                 hubs.data_ptr(), dists.data_ptr(), cap, ctypes.byref(total))
    if rc:
        err = PllError(rc, "pll_build_labels_noalloc")
        err.total = total.value
        raise err
    return total.value


def build_labels_directed(row_ptr: torch.Tensor, col: torch.Tensor, order: torch.Tensor,
                          batch_size: int = DEFAULT_BATCH, flags: int = FLAG_VALIDATE, arena_entries: int = 0,
                          query_lanes: int = 0, stream=None) -> Index:
    """L_in / L_out labels of the directed CSR graph (row v lists the heads of
    the arcs leaving v); the index's query gives the distance from u to v."""
    row_ptr = _dev(row_ptr, torch.int64, "row_ptr")
    col = _dev(col, torch.int32, "col")
    order = _dev(order, torch.int32, "order")
    n = order.numel()
    if row_ptr.numel() != n + 1:
        raise PllError(PLL_EINVAL, "row_ptr must have n+1 entries")
    h = ctypes.c_void_p()
    o = _opts(batch_size, flags, arena_entries, query_lanes)
    rc = load_library().pll_build_labels_directed(n, col.numel(), row_ptr.data_ptr(), col.data_ptr(),
                                                  order.data_ptr(), ctypes.byref(o), _stream_handle(stream),
                                                  ctypes.byref(h))
    if rc:
        raise PllError(rc, "pll_build_labels_directed")
    return Index(h.value, order.device)


def build_labels_weighted(row_ptr: torch.Tensor, col: torch.Tensor, weights: torch.Tensor, order: torch.Tensor,
                          batch_size: int = DEFAULT_BATCH, flags: int = FLAG_VALIDATE, arena_entries: int = 0,
                          query_lanes: int = 0, stream=None) -> Index:
    """Labels of the undirected graph with positive integer edge weights
    (weights uint8 [nnz], one per CSR entry, equal on both arcs of an edge);
    the index's query gives weighted distances."""
    row_ptr = _dev(row_ptr, torch.int64, "row_ptr")
    col = _dev(col, torch.int32, "col")
    weights = _dev(weights, torch.uint8, "weights")
    order = _dev(order, torch.int32, "order")
    n = order.numel()
    if row_ptr.numel() != n + 1:
        raise PllError(PLL_EINVAL, "row_ptr must have n+1 entries")
    if weights.numel() != col.numel():
        raise PllError(PLL_EINVAL, "one weight per CSR entry")
    h = ctypes.c_void_p()
    o = _opts(batch_size, flags, arena_entries, query_lanes)
    rc = load_library().pll_build_labels_weighted(n, col.numel(), row_ptr.data_ptr(), col.data_ptr(),
                                                  weights.data_ptr(), order.data_ptr(), ctypes.byref(o),
                                                  _stream_handle(stream), ctypes.byref(h))
    if rc:
        raise PllError(rc, "pll_build_labels_weighted")
    return Index(h.value, order.device)


def build_labels_batched(graphs, batch_size: int = DEFAULT_BATCH, flags: int = FLAG_VALIDATE,
                         arena_entries: int = 0, query_lanes: int = 0, gang_scale: int = 0, max_gang: int = 0,
                         max_workgroups: int = 0, stream=None) -> list:
    """Build many graphs in one persistent launch; ``graphs`` is a list of
    (row_ptr, col, order) device tensors.  Returns one :class:`Index` per
    graph."""
    descs = (GraphDesc * max(len(graphs), 1))()
    keep = []
    for i, (rp, cl, od) in enumerate(graphs):
        rp = _dev(rp, torch.int64, "row_ptr")
        cl = _dev(cl, torch.int32, "col")
        od = _dev(od, torch.int32, "order")
        keep.append((rp, cl, od))
        descs[i].n = od.numel()
        descs[i].nnz = cl.numel()
        descs[i].d_row_ptr = rp.data_ptr()
        descs[i].d_col = cl.data_ptr()
        descs[i].d_order = od.data_ptr()
    outs = (ctypes.c_void_p * max(len(graphs), 1))()
    o = _opts(batch_size, flags, arena_entries, query_lanes, gang_scale, max_gang, max_workgroups)
    rc = load_library().pll_build_labels_batched(len(graphs), descs, ctypes.byref(o), _stream_handle(stream), outs)
    if rc:
        raise PllError(rc, "pll_build_labels_batched")
    dev = keep[0][2].device if keep else torch.device("cuda")
    return [Index(outs[i], dev) for i in range(len(graphs))]


def stream_read(buf: torch.Tensor, sink: torch.Tensor, workgroups: int = 0, stream=None) -> None:
    """Enqueue pll_bench_stream_read over the bytes of ``buf`` (a contiguous
    device tensor, size a multiple of 16); ``sink`` is a device int64 tensor
    whose first element receives the XOR of the words."""
    if not buf.is_cuda or not sink.is_cuda or sink.dtype != torch.int64 or not buf.is_contiguous():
        raise PllError(PLL_EINVAL, "stream_read needs a contiguous device buffer and an int64 device sink")
    nbytes = buf.numel() * buf.element_size()
    rc = load_library().pll_bench_stream_read(buf.data_ptr(), nbytes, sink.data_ptr(), workgroups,
                                              _stream_handle(stream))
    if rc:
        raise PllError(rc, "pll_bench_stream_read")


def graph_to_device(g, device="cuda"):
    """(row_ptr, col) numpy CSR -> device tensors of the binding's dtypes."""
    import numpy as np
    rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr).view(np.int64)).to(device)
    cl = torch.from_numpy(np.ascontiguousarray(g.col).view(np.int32)).to(device)
    return rp, cl


class Server:
    """Continuous-batching query server over resident indexes (pll_server_*).

    Query requests carry host numpy arrays (uint32 ids in, uint32 distances
    out); the server keeps them alive until their results are polled."""

    def __init__(self, slots: int = 4, max_batch_pairs: int = 0, mem_reserve: int = 0, build_batch_size: int = 0,
                 build_workgroups: int = 0):
        o = ServerOpts()
        o.build_workgroups = build_workgroups
        o.slots = slots
        o.max_batch_pairs = max_batch_pairs
        o.mem_reserve = mem_reserve
        o.build_batch_size = build_batch_size
        h = ctypes.c_void_p()
        rc = load_library().pll_server_create(ctypes.byref(o), ctypes.byref(h))
        if rc:
            raise PllError(rc, "pll_server_create")
        self._h = h
        self._keep = {}

    def add_index(self, index: Index, take_ownership: bool = False) -> int:
        """Make `index` resident.  Without ownership the C server takes a
        reference of its own, so `index` may be freed (or collected) at any
        time: its labels stay resident until the server is closed.  With
        ownership the handle passes to the server."""
        iid = ctypes.c_uint32()
        rc = load_library().pll_server_add_index(self._h, index.handle, int(take_ownership), ctypes.byref(iid))
        if rc:
            raise PllError(rc, "pll_server_add_index")
        if take_ownership:
            index._h = ctypes.c_void_p(0)
        return iid.value

    def index(self, index_id: int) -> "Index":
        """A non-owning view of a resident index (valid while the server lives)."""
        h = ctypes.c_void_p()
        rc = load_library().pll_server_index(self._h, index_id, ctypes.byref(h))
        if rc:
            raise PllError(rc, "pll_server_index")
        view = Index(h.value, torch.device("cuda"))
        view.free = lambda: None
        return view

    @staticmethod
    def query_request(index_id: int, u, v, out, at: float = 0.0):
        import numpy as np
        u = np.ascontiguousarray(u, dtype=np.uint32)
        v = np.ascontiguousarray(v, dtype=np.uint32)
        assert out.dtype == np.uint32 and out.flags["C_CONTIGUOUS"] and out.shape == u.shape == v.shape
        r = Request()
        r.at = at
        r.kind = REQ_QUERY
        r.index_id = index_id
        r.count = u.shape[0]
        r.h_u, r.h_v, r.h_out = u.ctypes.data, v.ctypes.data, out.ctypes.data
        return r, (u, v, out)

    @staticmethod
    def build_request(row_ptr, col, order, at: float = 0.0):
        import numpy as np
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.uint64)
        col = np.ascontiguousarray(col, dtype=np.uint32)
        order = np.ascontiguousarray(order, dtype=np.uint32)
        r = Request()
        r.at = at
        r.kind = REQ_BUILD
        r.n = order.shape[0]
        r.nnz = col.shape[0]
        r.h_row_ptr, r.h_col, r.h_order = row_ptr.ctypes.data, col.ctypes.data if col.size else None, \
            order.ctypes.data if order.size else None
        return r, (row_ptr, col, order)

    def submit(self, req_and_arrays) -> int:
        r, arrays = req_and_arrays
        rid = ctypes.c_uint64()
        rc = load_library().pll_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid))
        if rc:
            raise PllError(rc, "pll_server_submit")
        self._keep[rid.value] = arrays
        return rid.value

    def poll(self, wait: bool = False, max_results: int = 1024) -> list:
        buf = (Result * max_results)()
        got = ctypes.c_uint32()
        rc = load_library().pll_server_poll(self._h, buf, max_results, ctypes.byref(got), int(wait))
        if rc:
            raise PllError(rc, "pll_server_poll")
        out = []
        for i in range(got.value):
            d = buf[i].as_dict()
            self._keep.pop(d["id"], None)
            out.append(d)
        return out

    def wait(self, rid: int) -> dict:
        while True:
            for d in self.poll(wait=True):
                if d["id"] == rid:
                    return d

    def replay(self, reqs_and_arrays) -> list:
        """Open-loop replay: request i is submitted reqs[i].at seconds after
        the call starts; returns the results in request order."""
        n = len(reqs_and_arrays)
        arr = (Request * max(n, 1))()
        keep = []
        for i, (r, arrays) in enumerate(reqs_and_arrays):
            arr[i] = r
            keep.append(arrays)
        res = (Result * max(n, 1))()
        rc = load_library().pll_server_replay(self._h, n, arr, res)
        if rc:
            raise PllError(rc, "pll_server_replay")
        return [res[i].as_dict() for i in range(n)]

    def close(self):
        if getattr(self, "_h", None):
            load_library().pll_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
