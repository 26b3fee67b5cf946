"""Pins of the directed oracle (Section 5.1: L_in / L_out labels, forward
and backward pruned searches, query over L_out(s) and L_in(t)) against
what does not come from the oracle: the directed form of Definition 2 by
brute force on scipy's all-pairs directed distances, hand-derived labels,
closed forms for directed paths and cycles, the reduction of a symmetric
digraph to the undirected labels, and the swap of L_in and L_out under
arc reversal."""
import os

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_labels_directed.txt")


def _apsp(g):
    a = csr_matrix((np.ones(g.nnz), g.col.astype(np.int64), g.row_ptr.astype(np.int64)), shape=(g.n, g.n))
    return shortest_path(a, method="D", unweighted=True, directed=True)


def brute_directed(g, order):
    """Directed Definition 2: on-path set P = {w : d(u,w) + d(w,v) = d(u,v)};
    u is in L_in(v) iff u is the highest-ranked vertex of P for the pair
    (u, v), and u is in L_out(v) iff it is for the pair (v, u)."""
    rank = np.empty(g.n, dtype=np.int64)
    rank[np.asarray(order, dtype=np.int64)] = np.arange(g.n)
    D = _apsp(g)
    lin = {v: [] for v in range(g.n)}
    lout = {v: [] for v in range(g.n)}
    for s in range(g.n):
        for t in range(g.n):
            if not np.isfinite(D[s, t]):
                continue
            on = np.isfinite(D[s]) & np.isfinite(D[:, t]) & (D[s] + D[:, t] == D[s, t])
            top = int(np.argmin(np.where(on, rank, g.n)))
            if top == s:
                lin[t].append((int(rank[s]), int(D[s, t])))
            if top == t:
                lout[s].append((int(rank[t]), int(D[s, t])))
    return {v: sorted(x) for v, x in lin.items()}, {v: sorted(x) for v, x in lout.items()}, D


def as_dict(lab):
    return {v: list(zip(*(a.tolist() for a in lab.of(v)))) for v in range(len(lab.offsets) - 1)}


def random_order(n, seed):
    return np.argsort(synth.splitmix64(seed, 0, n), kind="stable").astype(np.uint32)


def small_digraphs():
    gs = []
    for n in (1, 2, 3, 5, 8, 12, 16):
        for p, s in ((0.1, 1), (0.25, 2), (0.5, 3)):
            gs.append(synth.gnp_digraph(n, p, 300 * n + s))
    gs += [synth.directed_path(7), synth.directed_cycle(9), synth.rmat_digraph(5, 3, seed=4),
           synth.rmat_digraph(6, 2, seed=5)]
    return gs


@pytest.mark.parametrize("gi", range(len(small_digraphs())))
def test_directed_matches_bruteforce_def2(gi):
    g = small_digraphs()[gi]
    for order in (synth.degree_order_directed(g), random_order(g.n, 21 + gi), random_order(g.n, 733 + gi)):
        want_in, want_out, D = brute_directed(g, order)
        lin, lout = oracle.pll_labels_directed(g, order)
        assert as_dict(lin) == want_in, g.name
        assert as_dict(lout) == want_out, g.name
        s, t = np.divmod(np.arange(g.n * g.n), g.n)
        got = oracle.query_directed(lin, lout, s, t).astype(np.float64)
        want = D[s, t].copy()
        want[~np.isfinite(want)] = oracle.DIST_INF
        np.testing.assert_array_equal(got, want)


def _parse_golden():
    graphs, cur = [], None
    for line in open(GOLDEN):
        tok = line.split()
        if not tok or tok[0].startswith("#"):
            continue
        if tok[0] == "graph":
            cur = {"name": tok[1], "n": int(tok[2]), "in": {}, "out": {}}
        elif tok[0] == "arcs":
            cur["arcs"] = [tuple(int(x) for x in a.split(">")) for a in tok[1:]]
        elif tok[0] in ("in", "out"):
            cur[tok[0]][int(tok[1])] = [tuple(int(x) for x in e.split(":")) for e in tok[2:]]
        elif tok[0] == "end":
            graphs.append(cur)
    return graphs


@pytest.mark.parametrize("case", _parse_golden(), ids=lambda c: c["name"])
def test_hand_derived_directed_labels(case):
    src, dst = zip(*case["arcs"])
    g = synth.digraph_from_arcs(case["n"], np.array(src), np.array(dst))
    lin, lout = oracle.pll_labels_directed(g, np.arange(case["n"], dtype=np.uint32))
    assert as_dict(lin) == case["in"]
    assert as_dict(lout) == case["out"]


@pytest.mark.parametrize("n", [2, 3, 6, 17, 40])
def test_closed_forms_path_and_cycle(n):
    ident = np.arange(n, dtype=np.uint32)
    # directed path 0 > 1 > ... > n-1, rank = id: every u <= v is the top of the
    # only u-v path, and nothing reaches back
    lin, lout = oracle.pll_labels_directed(synth.directed_path(n), ident)
    for v in range(n):
        assert as_dict(lin)[v] == [(u, v - u) for u in range(v + 1)]
        assert as_dict(lout)[v] == [(v, 0)]
    # the reversed order swaps the roles
    lin, lout = oracle.pll_labels_directed(synth.directed_path(n), ident[::-1].copy())
    for v in range(n):
        assert as_dict(lin)[v] == [(n - 1 - v, 0)]
        assert as_dict(lout)[v] == sorted((n - 1 - u, u - v) for u in range(v, n))
    # directed cycle, rank = id: L_in(v) = {(u, v-u) : u <= v}; a path from v
    # back round to u < v passes 0, so L_out(v) = {(0, n-v), (v, 0)}
    lin, lout = oracle.pll_labels_directed(synth.directed_cycle(n), ident)
    for v in range(n):
        assert as_dict(lin)[v] == [(u, v - u) for u in range(v + 1)]
        assert as_dict(lout)[v] == ([(0, n - v)] if v else []) + [(v, 0)]


@pytest.mark.parametrize("seed", [1, 2])
def test_symmetric_digraph_reduces_to_undirected(seed):
    g = synth.ba_graph(300, 3, seed)
    order = synth.degree_order(g)
    und = as_dict(oracle.pll_labels(g, order))
    lin, lout = oracle.pll_labels_directed(synth.as_digraph(g), order)
    assert as_dict(lin) == und
    assert as_dict(lout) == und


def test_reversal_swaps_in_and_out():
    g = synth.rmat_digraph(9, 4, seed=7)
    order = synth.degree_order_directed(g)
    lin, lout = oracle.pll_labels_directed(g, order)
    rin, rout = oracle.pll_labels_directed(synth.reverse_digraph(g), order)
    assert as_dict(lin) == as_dict(rout)
    assert as_dict(lout) == as_dict(rin)


def test_query_matches_bfs_rmat_digraph():
    g = synth.rmat_digraph(10, 8, seed=3)
    order = synth.degree_order_directed(g)
    lin, lout = oracle.pll_labels_directed(g, order)
    for src in (0, 1, 5, 77, 1023):
        t = np.arange(g.n, dtype=np.uint32)
        got = oracle.query_directed(lin, lout, np.full(g.n, src, dtype=np.uint32), t)
        np.testing.assert_array_equal(got, oracle.bfs(g, src))


def test_directed_edist_and_bad_order():
    with pytest.raises(oracle.OracleError):
        oracle.pll_labels_directed(synth.directed_path(256), np.arange(256, dtype=np.uint32))
    lin, _ = oracle.pll_labels_directed(synth.directed_path(255), np.arange(255, dtype=np.uint32))
    assert int(lin.dist.max()) == 254
    with pytest.raises(oracle.OracleError):
        oracle.pll_labels_directed(synth.directed_path(4), np.array([0, 1, 1, 3], dtype=np.uint32))
