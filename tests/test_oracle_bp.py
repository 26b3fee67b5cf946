"""Pins of the bit-parallel oracle (Section 5.2's bit-parallel labels,
adopted from the original PLL, followed by PLL over the other vertices)
against what does not come from the oracle:

* the BP quantities against scipy's distances from each BP root and each
  of its chosen neighbours (d_r(v); S^-1 and S^0 by their definitions);
* the choice of roots and neighbour sets, re-derived from the rule;
* the normal labels against a brute-force definition: (u, d(u,v)) is in
  L(v) iff u is not a BP vertex, no BP vertex lies on a shortest u-v path,
  and u has the highest rank on every shortest u-v path (pruning by the BP
  bound removes exactly the pairs some BP vertex lies between);
* every pair's query against scipy; t = 0 reduces to plain PLL.
"""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

import oracle
import synth


def _apsp(g):
    a = csr_matrix((np.ones(g.nnz), g.col.astype(np.int64), g.row_ptr.astype(np.int64)), shape=(g.n, g.n))
    return shortest_path(a, method="D", unweighted=True, directed=False)


def as_dict(lab):
    return {v: list(zip(*(a.tolist() for a in lab.of(v)))) for v in range(len(lab.offsets) - 1)}


def expected_selection(g, order, t):
    rank = np.empty(g.n, dtype=np.int64)
    rank[order.astype(np.int64)] = np.arange(g.n)
    used = np.zeros(g.n, dtype=bool)
    roots, sets = [], []
    for r in order:
        if len(roots) == t:
            break
        if used[r]:
            continue
        used[r] = True
        nb = [int(w) for w in g.neighbors(int(r)) if not used[w]]
        nb = sorted(nb, key=lambda w: rank[w])[:64]
        used[nb] = True
        roots.append(int(r))
        sets.append(nb)
    return roots, sets, used


def brute_normal_labels(g, order, used, D):
    rank = np.empty(g.n, dtype=np.int64)
    rank[order.astype(np.int64)] = np.arange(g.n)
    out = {}
    for v in range(g.n):
        lst = []
        for u in range(g.n):
            if used[u] or not np.isfinite(D[u, v]):
                continue
            on = np.isfinite(D[u]) & np.isfinite(D[:, v]) & (D[u] + D[:, v] == D[u, v])
            if on[used].any():
                continue
            if rank[on].min() == rank[u]:
                lst.append((int(rank[u]), int(D[u, v])))
        out[v] = sorted(lst)
    return out


def graphs():
    gs = [synth.gnp_graph(n, p, 700 * n + s) for n, p, s in ((6, 0.5, 1), (12, 0.3, 2), (20, 0.2, 3), (30, 0.1, 4))]
    gs += [synth.random_tree(40, 5), synth.ba_graph(60, 2, 6), synth.ba_graph(150, 3, 7), synth.star_graph(70),
           synth.disjoint_union(synth.ba_graph(50, 2, 8), synth.path_graph(6), synth.complete_graph(5)),
           synth.rmat_graph(7, 4, seed=9)]
    return gs


@pytest.mark.parametrize("gi", range(len(graphs())))
@pytest.mark.parametrize("t", [1, 2, 4, 16])
def test_bp_matches_definitions(gi, t):
    g = graphs()[gi]
    for order in (synth.degree_order(g), np.argsort(synth.splitmix64(40 + gi, 0, g.n), kind="stable").astype(np.uint32)):
        lab, bp = oracle.pll_labels_bp(g, order, t)
        roots, sets, used = expected_selection(g, order, t)
        assert bp.root.tolist() == roots
        D = _apsp(g)
        for i, (r, S) in enumerate(zip(roots, sets)):
            assert bp.nbr[i].tolist() == S + [oracle.DIST_INF] * (64 - len(S))
            dr = D[r]
            want = np.where(np.isfinite(dr), dr, 255).astype(np.uint8)
            assert np.array_equal(bp.dist[:, i], want)
            sm1 = np.zeros(g.n, dtype=np.uint64)
            s0 = np.zeros(g.n, dtype=np.uint64)
            for j, s in enumerate(S):
                ds = D[s]
                fin = np.isfinite(dr)
                sm1 |= np.where(fin & (ds == dr - 1), np.uint64(1) << np.uint64(j), np.uint64(0))
                s0 |= np.where(fin & (ds == dr), np.uint64(1) << np.uint64(j), np.uint64(0))
            assert np.array_equal(bp.sm1[:, i], sm1)
            assert np.array_equal(bp.s0[:, i], s0)
        assert as_dict(lab) == brute_normal_labels(g, order, used, D)
        s, tt = np.divmod(np.arange(g.n * g.n), g.n)
        got = oracle.query_bp(lab, bp, s, tt).astype(np.float64)
        exp = D[s, tt].copy()
        exp[~np.isfinite(exp)] = oracle.DIST_INF
        np.testing.assert_array_equal(got, exp)


def test_no_bp_roots_is_plain_pll():
    g = synth.ba_graph(500, 3, 11)
    order = synth.degree_order(g)
    lab, bp = oracle.pll_labels_bp(g, order, 0)
    assert bp.t == 0
    assert as_dict(lab) == as_dict(oracle.pll_labels(g, order))


def test_bp_query_ba2000_against_bfs_and_fewer_entries():
    g = synth.ba_graph(2000, 4, 1)
    order = synth.degree_order(g)
    lab, bp = oracle.pll_labels_bp(g, order, 16)
    assert bp.t == 16 and lab.total < oracle.pll_labels(g, order).total
    for src in (0, 1, 17, 999, 1999):
        got = oracle.query_bp(lab, bp, np.full(g.n, src, dtype=np.uint32), np.arange(g.n, dtype=np.uint32))
        np.testing.assert_array_equal(got, oracle.bfs(g, src))


def test_more_roots_than_vertices_and_bad_t():
    g = synth.path_graph(5)
    lab, bp = oracle.pll_labels_bp(g, np.arange(5, dtype=np.uint32), 64)
    assert bp.t == 3 and lab.total == 0  # roots 0, 2, 4 (with 1 and 3) use every vertex
    with pytest.raises(oracle.OracleError):
        oracle.pll_labels_bp(g, np.arange(5, dtype=np.uint32), 65)
