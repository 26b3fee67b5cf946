"""Pins of the weighted oracle (PLL with Dijkstra, Section 5.1's weighted
graphs) against what does not come from the oracle: Definition 2 with
weighted distances by brute force on scipy's Dijkstra all-pairs distances,
hand-derived labels, the reduction to the unweighted labels for unit and
constant weights, a closed form on weighted paths, and scipy distances for
the query."""
import os

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_labels_weighted.txt")


def _apsp(g):
    a = csr_matrix((g.w.astype(np.float64), g.col.astype(np.int64), g.row_ptr.astype(np.int64)), shape=(g.n, g.n))
    return shortest_path(a, method="D", directed=False)


def brute_def2(g, order):
    rank = np.empty(g.n, dtype=np.int64)
    rank[np.asarray(order, dtype=np.int64)] = np.arange(g.n)
    D = _apsp(g)
    out = {}
    for v in range(g.n):
        lst = []
        for u in range(g.n):
            if not np.isfinite(D[u, v]):
                continue
            on = np.isfinite(D[u]) & np.isfinite(D[:, v]) & (D[u] + D[:, v] == D[u, v])
            if rank[on].min() == rank[u]:
                lst.append((int(rank[u]), int(D[u, v])))
        out[v] = sorted(lst)
    return out, D


def as_dict(lab):
    return {v: list(zip(*(a.tolist() for a in lab.of(v)))) for v in range(len(lab.offsets) - 1)}


def random_order(n, seed):
    return np.argsort(synth.splitmix64(seed, 0, n), kind="stable").astype(np.uint32)


def small_wgraphs():
    gs = []
    for n in (1, 2, 4, 7, 11, 16):
        for p, s in ((0.25, 1), (0.5, 2)):
            gs.append(synth.with_weights(synth.gnp_graph(n, p, 500 * n + s), seed=n + s))
    gs += [synth.with_weights(synth.random_tree(20, 3), seed=4), synth.with_weights(synth.ba_graph(40, 2, 5), seed=6),
           synth.with_weights(synth.ba_graph(30, 3, 7), 1, 20, seed=8),
           synth.with_weights(synth.disjoint_union(synth.path_graph(5), synth.complete_graph(5)), seed=9)]
    return gs


def test_weights_are_symmetric_and_in_range():
    g = synth.with_weights(synth.ba_graph(500, 4, 1))
    assert g.w.min() >= 1 and g.w.max() <= 7
    a = csr_matrix((g.w.astype(np.int64), g.col.astype(np.int64), g.row_ptr.astype(np.int64)), shape=(g.n, g.n))
    assert (a != a.T).nnz == 0


@pytest.mark.parametrize("gi", range(len(small_wgraphs())))
def test_weighted_matches_bruteforce_def2(gi):
    g = small_wgraphs()[gi]
    for order in (synth.degree_order(g), random_order(g.n, 31 + gi), random_order(g.n, 811 + gi)):
        want, D = brute_def2(g, order)
        lab = oracle.pll_labels_weighted(g, order)
        assert as_dict(lab) == want, g.name
        s, t = np.divmod(np.arange(g.n * g.n), g.n)
        got = oracle.query(lab, s, t).astype(np.float64)
        exp = D[s, t].copy()
        exp[~np.isfinite(exp)] = oracle.DIST_INF
        np.testing.assert_array_equal(got, exp)


def _parse_golden():
    out, cur = [], None
    for line in open(GOLDEN):
        tok = line.split()
        if not tok or tok[0].startswith("#"):
            continue
        if tok[0] == "graph":
            cur = {"name": tok[1], "n": int(tok[2]), "labels": {}}
        elif tok[0] == "order":
            cur["order"] = [int(x) for x in tok[1:]]
        elif tok[0] == "edges":
            cur["edges"] = [(int(e.split(":")[0].split("-")[0]), int(e.split(":")[0].split("-")[1]), int(e.split(":")[1]))
                            for e in tok[1:]]
        elif tok[0] == "label":
            cur["labels"][int(tok[1])] = [tuple(int(x) for x in e.split(":")) for e in tok[2:]]
        elif tok[0] == "end":
            out.append(cur)
    return out


@pytest.mark.parametrize("case", _parse_golden(), ids=lambda c: c["name"])
def test_hand_derived_weighted_labels(case):
    n = case["n"]
    a = np.array([e[0] for e in case["edges"]])
    b = np.array([e[1] for e in case["edges"]])
    g = synth.csr_from_edges(n, a, b)
    wmap = {}
    for x, y, w in case["edges"]:
        wmap[(x, y)] = wmap[(y, x)] = w
    rows = np.repeat(np.arange(n), np.diff(g.row_ptr).astype(np.int64))
    wg = synth.WGraph(n=n, row_ptr=g.row_ptr, col=g.col,
                      w=np.array([wmap[(int(r), int(c))] for r, c in zip(rows, g.col)], dtype=np.uint8))
    lab = oracle.pll_labels_weighted(wg, np.array(case["order"], dtype=np.uint32))
    assert as_dict(lab) == case["labels"]


@pytest.mark.parametrize("seed", [1, 2])
def test_unit_and_constant_weights_reduce_to_unweighted(seed):
    g = synth.ba_graph(400, 3, seed)
    order = synth.degree_order(g)
    und = as_dict(oracle.pll_labels(g, order))
    assert as_dict(oracle.pll_labels_weighted(synth.constant_weights(g, 1), order)) == und
    for c in (2, 5):
        got = as_dict(oracle.pll_labels_weighted(synth.constant_weights(g, c), order))
        assert got == {v: [(h, c * d) for h, d in lst] for v, lst in und.items()}


@pytest.mark.parametrize("n", [2, 5, 30])
def test_weighted_path_closed_form(n):
    # path 0-1-...-(n-1), rank = id: every u <= v is the top of the only u-v path
    g = synth.with_weights(synth.path_graph(n), 1, 7, seed=n)
    rows = np.repeat(np.arange(n), np.diff(g.row_ptr).astype(np.int64))
    step = {int(min(r, c)): int(w) for r, c, w in zip(rows, g.col, g.w)}
    pre = np.concatenate([[0], np.cumsum([step[i] for i in range(n - 1)])])
    lab = as_dict(oracle.pll_labels_weighted(g, np.arange(n, dtype=np.uint32)))
    for v in range(n):
        assert lab[v] == [(u, int(pre[v] - pre[u])) for u in range(v + 1)]


def test_query_matches_scipy_ba_weighted():
    g = synth.with_weights(synth.ba_graph(1500, 4, 3))
    order = synth.degree_order(g)
    lab = oracle.pll_labels_weighted(g, order)
    D = _apsp(g)
    u, v = synth.query_pairs(g.n, 20000, seed=4)
    np.testing.assert_array_equal(oracle.query(lab, u, v), D[u, v].astype(np.uint32))


def test_weighted_errors():
    g = synth.constant_weights(synth.path_graph(60), 5)  # distances up to 295
    with pytest.raises(oracle.OracleError):
        oracle.pll_labels_weighted(g, np.arange(60, dtype=np.uint32))
    ok = synth.constant_weights(synth.path_graph(52), 5)  # 51 * 5 = 255 does not fit
    with pytest.raises(oracle.OracleError):
        oracle.pll_labels_weighted(ok, np.arange(52, dtype=np.uint32))
    ok = synth.constant_weights(synth.path_graph(51), 5)  # 50 * 5 = 250 fits
    assert int(oracle.pll_labels_weighted(ok, np.arange(51, dtype=np.uint32)).dist.max()) == 250
    z = synth.constant_weights(synth.path_graph(4), 0)
    with pytest.raises(oracle.OracleError):
        oracle.pll_labels_weighted(z, np.arange(4, dtype=np.uint32))
