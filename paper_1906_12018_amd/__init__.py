"""MI355X (gfx950) pruned landmark labeling: Python binding of libpll.

Argument marshalling only: every step of label construction and querying runs
in the HIP kernels of ``libpll.so`` (declared in ``include/pll.h``).  PyTorch
supplies device memory and the current stream.  There is no CPU fallback; if
the library is not built, or no GPU is present, calls raise :class:`PllError`.

Paper: Jin et al., "Pruned Landmark Labeling Meets Vertex Centric
Computation" (arXiv 1906.12018): BVC-PLL (Section 4.2, Algorithm 4) builds the
canonical 2-hop labeling (Definition 2) for a vertex order; the 2-hop query
(Section 2.1) merges two hub-sorted lists.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpll.so")

PLL_OK, PLL_EINVAL, PLL_ENOMEM, PLL_ENOSPC, PLL_EDIST, PLL_EDEVICE = 0, 1, 2, 3, 4, 5
DIST_INF = 0xFFFFFFFF
FLAG_VALIDATE, FLAG_RECHECK, FLAG_RELAXED, FLAG_PROFILE = 0x1, 0x2, 0x4, 0x8
PHASES = ("prep", "init", "push", "check", "end", "final")
DEFAULT_BATCH = 1024

EXPORTED_SYMBOLS = (
    "pll_build_labels", "pll_query", "pll_index_info_get", "pll_export_labels",
    "pll_build_labels_batched", "pll_index_free", "pll_status_string",
)


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
        ("reserved", ctypes.c_uint32 * 5),
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
        ("phase_ms", ctypes.c_double * 6),
        ("phase_launches", ctypes.c_uint64 * 6),
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
    lib.pll_build_labels_batched.argtypes = [U32, ctypes.POINTER(GraphDesc), ctypes.POINTER(BuildOpts), P,
                                             ctypes.POINTER(P)]
    lib.pll_build_labels_batched.restype = ctypes.c_int
    lib.pll_index_free.argtypes = [P]
    lib.pll_index_free.restype = None
    lib.pll_status_string.argtypes = [ctypes.c_int]
    lib.pll_status_string.restype = ctypes.c_char_p
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
          max_gang: int = 0) -> BuildOpts:
    o = BuildOpts()
    o.batch_size = batch_size
    o.flags = flags
    o.arena_entries = arena_entries
    o.query_lanes = query_lanes
    o.gang_scale = gang_scale
    o.max_gang = max_gang
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

    def export(self, stream=None) -> ExportedLabels:
        inf = self.info()
        n, total = inf["n"], inf["total_entries"]
        off = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        hubs = torch.empty(max(total, 1), dtype=torch.int32, device=self.device)
        dists = torch.empty(max(total, 1), dtype=torch.uint8, device=self.device)
        rc = load_library().pll_export_labels(self.handle, off.data_ptr(), hubs.data_ptr(), dists.data_ptr(),
                                              _stream_handle(stream))
        if rc:
            raise PllError(rc, "pll_export_labels")
        return ExportedLabels(off, hubs[:total], dists[:total])

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
                 flags: int = FLAG_VALIDATE, arena_entries: int = 0, query_lanes: int = 0, stream=None) -> Index:
    """Canonical 2-hop labels of the CSR graph (row_ptr int64 [n+1], col
    int32 [nnz], order int32 [n]: order[k] = vertex of rank k)."""
    row_ptr = _dev(row_ptr, torch.int64, "row_ptr")
    col = _dev(col, torch.int32, "col")
    order = _dev(order, torch.int32, "order")
    n = order.numel()
    if row_ptr.numel() != n + 1:
        raise PllError(PLL_EINVAL, "row_ptr must have n+1 entries")
    h = ctypes.c_void_p()
    o = _opts(batch_size, flags, arena_entries, query_lanes)
    rc = load_library().pll_build_labels(n, col.numel(), row_ptr.data_ptr(), col.data_ptr(), order.data_ptr(),
                                         ctypes.byref(o), _stream_handle(stream), ctypes.byref(h))
    if rc:
        raise PllError(rc, "pll_build_labels")
    return Index(h.value, order.device)


def build_labels_batched(graphs, batch_size: int = DEFAULT_BATCH, flags: int = FLAG_VALIDATE,
                         arena_entries: int = 0, query_lanes: int = 0, gang_scale: int = 0, max_gang: int = 0,
                         stream=None) -> list:
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
    o = _opts(batch_size, flags, arena_entries, query_lanes, gang_scale, max_gang)
    rc = load_library().pll_build_labels_batched(len(graphs), descs, ctypes.byref(o), _stream_handle(stream), outs)
    if rc:
        raise PllError(rc, "pll_build_labels_batched")
    dev = keep[0][2].device if keep else torch.device("cuda")
    return [Index(outs[i], dev) for i in range(len(graphs))]


def graph_to_device(g, device="cuda"):
    """(row_ptr, col) numpy CSR -> device tensors of the binding's dtypes."""
    import numpy as np
    rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr).view(np.int64)).to(device)
    cl = torch.from_numpy(np.ascontiguousarray(g.col).view(np.int32)).to(device)
    return rp, cl
