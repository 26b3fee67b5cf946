"""Seeded synthetic inputs shared by the oracle side and the GPU side.

Holds graph generation and CSR assembly only, none of the labeling or query
arithmetic.  The generators stand in for the paper's real graphs (social and
web graphs with power-law degrees and small diameters; Section 6, Table of
datasets), which are not available here:

* Barabasi-Albert (BA) preferential attachment graphs.
* R-MAT graphs, edge factor 16, (a,b,c,d) = (0.57, 0.19, 0.19, 0.05).

The vertex order is the paper's degree order (Section 6, "Benchmarks"):
degree descending, ties broken by ascending vertex id.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None

GOLDEN = 0x9E3779B97F4A7C15


def build_native(force: bool = True) -> str:
    """Compile graphgen.c into libgraphgen.so (plain gcc, host only)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_native(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.synth_ba_edges.restype = ctypes.c_int64
        lib.synth_ba_edges.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p]
        lib.synth_rmat_edges.restype = None
        lib.synth_rmat_edges.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p]
        lib.synth_splitmix64_fill.restype = None
        lib.synth_splitmix64_fill.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclass
class Graph:
    """Undirected graph in CSR form: symmetric, no self-loops, no duplicate
    edges, each row sorted by vertex id."""
    n: int
    row_ptr: np.ndarray  # uint64[n+1]
    col: np.ndarray      # uint32[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def num_edges(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def neighbors(self, v: int) -> np.ndarray:
        return self.col[int(self.row_ptr[v]):int(self.row_ptr[v + 1])]


def splitmix64(seed: int, k0: int, count: int) -> np.ndarray:
    """Draws k0 .. k0+count-1 of the splitmix64 stream `seed` (uint64)."""
    out = np.empty(count, dtype=np.uint64)
    if count:
        _load().synth_splitmix64_fill(seed & 0xFFFFFFFFFFFFFFFF, k0, count, out.ctypes.data)
    return out


def bounded(x: np.ndarray, r: int) -> np.ndarray:
    """Lemire multiply-shift on the top 32 bits: values in [0, r), r < 2^32."""
    return (((x >> np.uint64(32)) * np.uint64(r)) >> np.uint64(32)).astype(np.uint32)


def uniform01(x: np.ndarray) -> np.ndarray:
    return (x >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray, name: str = "") -> Graph:
    """Symmetrise, drop self-loops, sort and dedup an edge list into CSR."""
    src = np.asarray(src, dtype=np.uint64)
    dst = np.asarray(dst, dtype=np.uint64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    keys = np.concatenate([(src << np.uint64(32)) | dst, (dst << np.uint64(32)) | src])
    keys = np.unique(keys)
    rows = (keys >> np.uint64(32)).astype(np.int64)
    col = (keys & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n=n, row_ptr=row_ptr, col=col, name=name)


def ba_graph(n: int, m: int, seed: int) -> Graph:
    """Barabasi-Albert graph (see graphgen.c for the exact process)."""
    if m < 1 or n < m + 1:
        raise ValueError("BA needs m >= 1 and n >= m + 1")
    ne = m * (n - m)
    edges = np.empty(2 * ne, dtype=np.uint32)
    got = _load().synth_ba_edges(n, m, seed, edges.ctypes.data)
    if got != ne:
        raise RuntimeError("BA generator failed")
    return csr_from_edges(n, edges[0::2], edges[1::2], name=f"ba_n{n}_m{m}_s{seed}")


def rmat_graph(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
               seed: int = 1) -> Graph:
    """R-MAT graph with 2^scale vertices and edge_factor * 2^scale samples,
    symmetrised, deduplicated, self-loops removed; isolated vertices kept."""
    n = 1 << scale
    ns = edge_factor * n
    edges = np.empty(2 * ns, dtype=np.uint32)
    _load().synth_rmat_edges(scale, ns, a, b, c, seed, edges.ctypes.data)
    return csr_from_edges(n, edges[0::2], edges[1::2], name=f"rmat{scale}_ef{edge_factor}_s{seed}")


def degree_order(g: Graph) -> np.ndarray:
    """order[k] = vertex of rank k; rank 0 is the highest.  Degree descending,
    ties by ascending vertex id."""
    deg = g.degrees()
    ids = np.arange(g.n, dtype=np.int64)
    return np.lexsort((ids, -deg)).astype(np.uint32)


def query_pairs(n: int, count: int, seed: int = 2):
    """Uniform pairs on [0,n)^2 with replacement: pair i uses draws 2i, 2i+1."""
    x = splitmix64(seed, 0, 2 * count)
    u = bounded(x[0::2], n)
    v = bounded(x[1::2], n)
    return u, v


def batching_specs(count: int = 256, n_lo: int = 500, n_hi: int = 20000, m_lo: int = 2, m_hi: int = 8,
                   seed: int = 3):
    """(n, m, seed) for the many-graph workload: n = round(exp(U[ln n_lo, ln n_hi])),
    m uniform in {m_lo..m_hi}, drawn from stream `seed` (draws 2g, 2g+1);
    graph g is generated with seed 1000 + g."""
    x = splitmix64(seed, 0, 2 * count)
    specs = []
    for g in range(count):
        uu = float(uniform01(x[2 * g:2 * g + 1])[0])
        n = int(round(math.exp(math.log(n_lo) + uu * (math.log(n_hi) - math.log(n_lo)))))
        m = m_lo + int(bounded(x[2 * g + 1:2 * g + 2], m_hi - m_lo + 1)[0])
        n = max(n, m + 1)
        specs.append((n, m, 1000 + g))
    return specs


# --- small deterministic families used by tests -------------------------------------------------

def path_graph(n: int) -> Graph:
    s = np.arange(n - 1)
    return csr_from_edges(n, s, s + 1, name=f"path{n}")


def star_graph(n: int) -> Graph:
    leaves = np.arange(1, n)
    return csr_from_edges(n, np.zeros(n - 1, dtype=np.int64), leaves, name=f"star{n}")


def complete_graph(n: int) -> Graph:
    iu = np.triu_indices(n, 1)
    return csr_from_edges(n, iu[0], iu[1], name=f"K{n}")


def gnp_graph(n: int, p: float, seed: int) -> Graph:
    """Erdos-Renyi G(n,p) from the splitmix64 stream (pair (i<j) in triu order)."""
    iu = np.triu_indices(n, 1)
    x = uniform01(splitmix64(seed, 0, len(iu[0])))
    keep = x < p
    return csr_from_edges(n, iu[0][keep], iu[1][keep], name=f"gnp{n}_{p}_s{seed}")


def random_tree(n: int, seed: int) -> Graph:
    """Random recursive tree: vertex t attaches to a uniform earlier vertex."""
    if n < 2:
        return csr_from_edges(n, np.zeros(0, np.int64), np.zeros(0, np.int64), name=f"tree{n}")
    x = splitmix64(seed, 0, n)
    par = np.array([int(bounded(x[t:t + 1], t)[0]) for t in range(1, n)], dtype=np.int64)
    return csr_from_edges(n, np.arange(1, n), par, name=f"tree{n}_s{seed}")


def disjoint_union(*graphs: Graph) -> Graph:
    n = sum(g.n for g in graphs)
    src, dst, base = [], [], 0
    for g in graphs:
        rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr).astype(np.int64))
        src.append(rows + base)
        dst.append(g.col.astype(np.int64) + base)
        base += g.n
    return csr_from_edges(n, np.concatenate(src) if src else np.zeros(0), np.concatenate(dst) if dst else np.zeros(0),
                          name="union")


# --- directed graphs (arcs) ---------------------------------------------------------------------

@dataclass
class DiGraph:
    """Directed graph in CSR form: row v lists the heads of the arcs leaving
    v, sorted by vertex id, with no self-loop and no duplicate arc."""
    n: int
    row_ptr: np.ndarray  # uint64[n+1]
    col: np.ndarray      # uint32[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def out_degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def in_degrees(self) -> np.ndarray:
        return np.bincount(self.col.astype(np.int64), minlength=self.n).astype(np.int64)


def digraph_from_arcs(n: int, src: np.ndarray, dst: np.ndarray, name: str = "") -> DiGraph:
    """Drop self-loops, sort and dedup an arc list into CSR (no symmetrisation)."""
    src = np.asarray(src, dtype=np.uint64)
    dst = np.asarray(dst, dtype=np.uint64)
    keep = src != dst
    keys = np.unique((src[keep] << np.uint64(32)) | dst[keep])
    rows = (keys >> np.uint64(32)).astype(np.int64)
    col = (keys & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    row_ptr = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    return DiGraph(n=n, row_ptr=row_ptr, col=col, name=name)


def rmat_digraph(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
                 seed: int = 1) -> DiGraph:
    """R-MAT arcs (same sampler as rmat_graph, sample i is the arc src -> dst),
    deduplicated, self-loops removed, not symmetrised."""
    n = 1 << scale
    ns = edge_factor * n
    edges = np.empty(2 * ns, dtype=np.uint32)
    _load().synth_rmat_edges(scale, ns, a, b, c, seed, edges.ctypes.data)
    return digraph_from_arcs(n, edges[0::2], edges[1::2], name=f"rmat{scale}_ef{edge_factor}_s{seed}_dir")


def gnp_digraph(n: int, p: float, seed: int) -> DiGraph:
    """Each ordered pair (i, j), i != j, is an arc with probability p (row-major order of the n*n grid)."""
    x = uniform01(splitmix64(seed, 0, n * n)).reshape(n, n)
    src, dst = np.nonzero(x < p)
    return digraph_from_arcs(n, src, dst, name=f"dgnp{n}_{p}_s{seed}")


def directed_path(n: int) -> DiGraph:
    s = np.arange(max(n - 1, 0))
    return digraph_from_arcs(n, s, s + 1, name=f"dpath{n}")


def directed_cycle(n: int) -> DiGraph:
    s = np.arange(n)
    return digraph_from_arcs(n, s, (s + 1) % n, name=f"dcycle{n}")


def as_digraph(g: Graph) -> DiGraph:
    """The symmetric digraph with both arcs of every edge of g."""
    return DiGraph(n=g.n, row_ptr=g.row_ptr.copy(), col=g.col.copy(), name=g.name + "_sym")


def reverse_digraph(g: DiGraph) -> DiGraph:
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr).astype(np.int64))
    return digraph_from_arcs(g.n, g.col.astype(np.int64), rows, name=g.name + "_rev")


def degree_order_directed(g: DiGraph) -> np.ndarray:
    """order[k] = vertex of rank k: total degree (in + out) descending, ties by ascending id."""
    deg = g.out_degrees() + g.in_degrees()
    ids = np.arange(g.n, dtype=np.int64)
    return np.lexsort((ids, -deg)).astype(np.uint32)


# --- weighted graphs ----------------------------------------------------------------------------

@dataclass
class WGraph:
    """Undirected graph with positive integer edge weights: the CSR of Graph
    plus w[e], the weight of CSR entry e (both arcs of an edge carry the same
    weight)."""
    n: int
    row_ptr: np.ndarray  # uint64[n+1]
    col: np.ndarray      # uint32[nnz]
    w: np.ndarray        # uint8[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def num_edges(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


def _mix64(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def splitmix64_at(seed: int, k: np.ndarray) -> np.ndarray:
    """Draw k of stream `seed` for any array of draw indices (graphgen.c's definition)."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (k + np.uint64(1)) * np.uint64(GOLDEN))


def with_weights(g: Graph, lo: int = 1, hi: int = 7, seed: int = 5) -> WGraph:
    """Weights uniform in [lo, hi] (the paper's recipe for its weighted runs
    is 1..7, Section 6): edge {a, b}, a < b, takes draw a * n + b of stream
    `seed`, so both arcs agree."""
    rows = np.repeat(np.arange(g.n, dtype=np.uint64), np.diff(g.row_ptr).astype(np.int64))
    cols = g.col.astype(np.uint64)
    a, b = np.minimum(rows, cols), np.maximum(rows, cols)
    x = splitmix64_at(seed, a * np.uint64(g.n) + b)
    w = (lo + bounded(x, hi - lo + 1)).astype(np.uint8)
    return WGraph(n=g.n, row_ptr=g.row_ptr, col=g.col, w=w, name=f"{g.name}_w{lo}-{hi}_s{seed}")


def constant_weights(g: Graph, c: int) -> WGraph:
    return WGraph(n=g.n, row_ptr=g.row_ptr, col=g.col, w=np.full(g.nnz, c, dtype=np.uint8), name=f"{g.name}_c{c}")
