"""Pins for the oracle (CPU only).

Each test checks the oracle against something other than itself: a brute
force of Definition 2 built on scipy's all-pairs shortest paths, hand-derived
labelings, closed forms for graph families, BFS distances from scipy, the
minimality of canonical labels, and the counting identities of the paper's
cost analysis (Lemma 3 / Corollary 2).
"""
import os

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_labels.txt")


def _apsp(g):
    a = csr_matrix((np.ones(g.nnz), g.col.astype(np.int64), g.row_ptr.astype(np.int64)), shape=(g.n, g.n))
    return shortest_path(a, method="D", unweighted=True, directed=False)


def brute_def2(g, order):
    """Definition 2 by brute force: P_uv = {w : d(u,w) + d(w,v) = d(u,v)};
    u is a hub of v iff the highest-ranked member of P_uv is u."""
    rank = np.empty(g.n, dtype=np.int64)
    rank[np.asarray(order, dtype=np.int64)] = np.arange(g.n)
    D = _apsp(g)
    out = {}
    for v in range(g.n):
        lst = []
        for u in range(g.n):
            if not np.isfinite(D[u, v]):
                continue
            on_path = np.isfinite(D[u]) & np.isfinite(D[:, v]) & (D[u] + D[:, v] == D[u, v])
            if rank[on_path].min() == rank[u]:
                lst.append((int(rank[u]), int(D[u, v])))
        out[v] = sorted(lst)
    return out


def as_dict(lab: oracle.Labels):
    out = {}
    owners = lab.owners if lab.owners is not None else range(len(lab.offsets) - 1)
    for i, v in enumerate(owners):
        h, d = lab.of(i)
        out[int(v)] = list(zip(h.tolist(), d.tolist()))
    return out


def random_order(n, seed):
    x = synth.splitmix64(seed, 0, n)
    return np.argsort(x, kind="stable").astype(np.uint32)


def small_graphs():
    gs = []
    for n in (1, 2, 3, 5, 8, 11, 14):
        for p, s in ((0.2, 1), (0.35, 2), (0.6, 3)):
            gs.append(synth.gnp_graph(n, p, 100 * n + s))
    gs += [synth.random_tree(12, 7), synth.random_tree(17, 8), synth.path_graph(9), synth.star_graph(7),
           synth.complete_graph(6), synth.disjoint_union(synth.path_graph(4), synth.complete_graph(4)),
           synth.ba_graph(30, 2, 5), synth.ba_graph(25, 3, 6)]
    return gs


@pytest.mark.parametrize("gi", range(len(small_graphs())))
def test_all_oracles_match_bruteforce_def2(gi):
    g = small_graphs()[gi]
    orders = [synth.degree_order(g), random_order(g.n, 11 + gi), random_order(g.n, 977 + gi)]
    for order in orders:
        want = brute_def2(g, order)
        assert as_dict(oracle.canonical_labels(g, order)) == want
        assert as_dict(oracle.pll_labels(g, order)) == want
        for b in sorted({1, 2, 3, 5, max(1, g.n)}):
            assert as_dict(oracle.bvc_labels(g, order, b)) == want, (g.name, b)


def _parse_golden():
    graphs, cur = [], None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        if tok[0] == "graph":
            cur = {"name": tok[1], "n": int(tok[2]), "edges": [], "labels": {}}
        elif tok[0] == "edges":
            cur["edges"] = [tuple(int(x) for x in e.split("-")) for e in tok[1:]]
        elif tok[0] == "label":
            cur["labels"][int(tok[1])] = [tuple(int(x) for x in e.split(":")) for e in tok[2:]]
        elif tok[0] == "end":
            graphs.append(cur)
    return graphs


@pytest.mark.parametrize("case", _parse_golden(), ids=lambda c: c["name"])
def test_hand_derived_labels(case):
    e = np.array(case["edges"], dtype=np.int64)
    g = synth.csr_from_edges(case["n"], e[:, 0], e[:, 1])
    order = synth.degree_order(g)
    for lab in (oracle.canonical_labels(g, order), oracle.pll_labels(g, order), oracle.bvc_labels(g, order, 2)):
        got = as_dict(lab)
        for v, want in case["labels"].items():
            hubs_ids = [int(order[h]) for h, _ in got[v]]
            assert list(zip(hubs_ids, [d for _, d in got[v]])) == want, (case["name"], v)


@pytest.mark.parametrize("n", [3, 4, 5, 8, 13, 40])
def test_closed_forms(n):
    # complete graph: rank = id, L(v) = every u <= v
    g = synth.complete_graph(n)
    assert oracle.pll_labels(g, synth.degree_order(g)).total == n * (n + 1) // 2
    # star centred at 0: the centre plus itself for every leaf
    g = synth.star_graph(n)
    assert oracle.pll_labels(g, synth.degree_order(g)).total == 2 * n - 1
    # path: interior vertices first by id, then the two endpoints
    g = synth.path_graph(n)
    assert oracle.pll_labels(g, synth.degree_order(g)).total == (n - 2) * (n - 1) // 2 + n + 1


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tree_hub_is_top_of_unique_path(seed):
    g = synth.random_tree(60, seed)
    order = synth.degree_order(g)
    rank = np.empty(g.n, dtype=np.int64)
    rank[order.astype(np.int64)] = np.arange(g.n)
    # parent pointers from a BFS at vertex 0 give each unique path
    par = np.full(g.n, -1)
    depth = np.zeros(g.n, dtype=np.int64)
    seen = np.zeros(g.n, bool)
    seen[0] = True
    q = [0]
    for x in q:
        for y in g.neighbors(x):
            if not seen[y]:
                seen[y] = True
                par[y] = x
                depth[y] = depth[x] + 1
                q.append(int(y))

    def path(a, b):
        pa, pb = [a], [b]
        while pa[-1] != pb[-1]:
            if depth[pa[-1]] >= depth[pb[-1]]:
                pa.append(par[pa[-1]])
            else:
                pb.append(par[pb[-1]])
        return pa + pb[:-1][::-1]

    got = as_dict(oracle.pll_labels(g, order))
    for v in range(g.n):
        want = []
        for u in range(g.n):
            p = path(u, v)
            if min(rank[p]) == rank[u]:
                want.append((int(rank[u]), len(p) - 1))
        assert got[v] == sorted(want)


def test_disconnected_union_and_unreachable():
    a, b = synth.ba_graph(40, 2, 3), synth.complete_graph(5)
    g = synth.disjoint_union(a, b)
    order = synth.degree_order(g)
    lab = oracle.pll_labels(g, order)
    hubs = lab.hubs_as_ids(order)
    for v in range(g.n):
        lo, hi = int(lab.offsets[v]), int(lab.offsets[v + 1])
        comp = v < a.n
        assert all((h < a.n) == comp for h in hubs[lo:hi])
    u = np.array([0, 1, 41], dtype=np.uint32)
    v = np.array([42, 44, 2], dtype=np.uint32)
    assert (oracle.query(lab, u, v) == oracle.DIST_INF).all()


def test_query_matches_scipy_distances_ba():
    g = synth.ba_graph(400, 3, 9)
    order = synth.degree_order(g)
    lab = oracle.pll_labels(g, order)
    D = _apsp(g)
    uu, vv = np.meshgrid(np.arange(g.n), np.arange(g.n), indexing="ij")
    got = oracle.query(lab, uu.ravel(), vv.ravel()).reshape(g.n, g.n)
    assert (got == D.astype(np.int64)).all()


def test_query_matches_scipy_on_gnp_with_isolated():
    g = synth.gnp_graph(120, 0.02, 5)  # sparse: several components and isolated vertices
    order = synth.degree_order(g)
    lab = oracle.pll_labels(g, order)
    D = _apsp(g)
    uu, vv = np.meshgrid(np.arange(g.n), np.arange(g.n), indexing="ij")
    got = oracle.query(lab, uu.ravel(), vv.ravel()).reshape(g.n, g.n).astype(np.float64)
    want = np.where(np.isfinite(D), D, float(oracle.DIST_INF))
    assert (got == want).all()


def test_label_invariants_ba():
    """Self entry, hierarchy (hub ranks at or above the owner), exact
    distances (Corollary 1) and minimality (no entry can be dropped)."""
    g = synth.ba_graph(250, 3, 4)
    order = synth.degree_order(g)
    rank = np.empty(g.n, dtype=np.int64)
    rank[order.astype(np.int64)] = np.arange(g.n)
    lab = oracle.pll_labels(g, order)
    D = _apsp(g)
    d = as_dict(lab)
    for v in range(g.n):
        lst = d[v]
        assert lst[-1] == (rank[v], 0)
        assert all(h <= rank[v] for h, _ in lst)
        assert all(D[order[h], v] == dist for h, dist in lst)
    # minimality: without (u,d), L(u) and L(v) no longer certify d(u,v) = d
    for v in range(g.n):
        for h, dist in d[v]:
            u = int(order[h])
            if u == v:
                continue
            lu = dict(d[u])
            rest = [(x, y) for x, y in d[v] if x != h]
            best = min((lu[x] + y for x, y in rest if x in lu), default=10 ** 9)
            assert best > dist


def test_counters_corollary2_and_batch_invariance():
    """Corollary 2: PLL and BVC-PLL make the same distance checks; PLL also
    pops every root once.  Labels do not depend on the batch size."""
    g = synth.ba_graph(2000, 4, 1)
    order = synth.degree_order(g)
    p = oracle.pll_labels(g, order)
    for b in (1, 7, 64, 1024, g.n):
        bv = oracle.bvc_labels(g, order, b)
        assert np.array_equal(bv.offsets, p.offsets)
        assert np.array_equal(bv.hub_rank, p.hub_rank)
        assert np.array_equal(bv.dist, p.dist)
        assert bv.counters["checks"] + g.n == p.counters["checks"]
        assert bv.counters["added"] == p.total
    # VC-PLL (b = n) never sends more edge accesses than PLL (Section 3.3)
    assert oracle.bvc_labels(g, order, g.n).counters["edge_accesses"] <= p.counters["edge_accesses"]


def test_edist_on_long_path():
    g = synth.path_graph(300)
    with pytest.raises(oracle.OracleError):
        oracle.pll_labels(g, synth.degree_order(g))
    with pytest.raises(oracle.OracleError):
        oracle.bvc_labels(g, synth.degree_order(g), 16)
    # 256 vertices: largest distance 254 still fits
    g = synth.path_graph(256)
    lab = oracle.pll_labels(g, synth.degree_order(g))
    assert int(lab.dist.max()) == 254


def test_bad_order_rejected():
    g = synth.path_graph(5)
    with pytest.raises(oracle.OracleError):
        oracle.pll_labels(g, np.array([0, 1, 1, 2, 3], dtype=np.uint32))


def test_pll_matches_def2_sample_rmat16():
    """Full-size pin: Definition 2, vertex by vertex, on a sample of the
    R-MAT scale-16 graph against the PLL labels of the whole graph."""
    g = synth.rmat_graph(16)
    order = synth.degree_order(g)
    lab = oracle.pll_labels(g, order)
    x = synth.splitmix64(77, 0, 150)
    verts = np.unique(synth.bounded(x, g.n))
    verts = np.concatenate([verts, order[:10], order[-10:]]).astype(np.uint32)
    c = oracle.canonical_labels(g, order, verts=verts, threads=8)
    for i, v in enumerate(verts):
        h, d = c.of(i)
        ph, pd = lab.of(int(v))
        assert np.array_equal(h, ph) and np.array_equal(d, pd)


# ---- cost-model counters (Section 4.3, Theorem 3, Table 3) -------------------------------------------------------

def _lists_by_rank(lab: oracle.Labels, order):
    """(hub ranks, dists) of every list, indexed by the owner's rank."""
    n = len(order)
    out = [None] * n
    for vid in range(n):
        h, d = lab.of(vid)
        out[vid] = (h.astype(np.int64), d.astype(np.int64))
    rank = np.empty(n, dtype=np.int64)
    rank[order.astype(np.int64)] = np.arange(n)
    return [(rank[v], out[v][0], out[v][1]) for v in range(n)]


def pll_positive_cost(lab: oracle.Labels):
    """PLL adds the entries of L(v) in ascending hub rank, each after a check
    whose cost is the number of entries already there: 0 + 1 + ... + (l-1)."""
    sz = lab.sizes()
    return int((sz * (sz - 1) // 2).sum())


def bvc_positive_cost(lab: oracle.Labels, order, b):
    """BVC-PLL adds the entry (h, d) of L(v), h in batch i, after a check that
    sees every entry of earlier batches and the entries of batch i at a
    smaller distance (the groups g_1..g_{k-1} of Theorem 3's proof); the
    self entry (v, 0) is added without a check."""
    total = 0
    for rv, h, d in _lists_by_rank(lab, order):
        bt = h // b
        for i in range(len(h)):
            if h[i] == rv:
                continue
            earlier = int((bt < bt[i]).sum())
            same = int(((bt == bt[i]) & (d < d[i])).sum())
            total += earlier + same
    return total


@pytest.mark.parametrize("gi", range(len(small_graphs())))
def test_check_costs_match_closed_forms(gi):
    g = small_graphs()[gi]
    order = synth.degree_order(g)
    p = oracle.pll_labels(g, order)
    assert p.counters["cost_pos"] == pll_positive_cost(p)
    assert p.counters["cost_pos"] + p.counters["cost_neg"] == p.counters["scanned"]
    for b in (1, 2, 3, max(g.n, 1)):
        bv = oracle.bvc_labels(g, order, b)
        assert bv.counters["cost_pos"] == bvc_positive_cost(bv, order, b), b
        assert bv.counters["cost_pos"] + bv.counters["cost_neg"] == bv.counters["scanned"]
        # Theorem 3: the positive checks of BVC-PLL cost no more than PLL's
        assert bv.counters["cost_pos"] <= p.counters["cost_pos"]


def test_check_costs_ba_and_b1_reduces_to_pll():
    """With b = 1 every batch is one root: the negative checks and their costs
    are PLL's, and the positive ones differ only by PLL's n self checks,
    which see every other entry of L(v) (l_v - 1 each)."""
    g = synth.ba_graph(600, 3, 9)
    order = synth.degree_order(g)
    p = oracle.pll_labels(g, order)
    b1 = oracle.bvc_labels(g, order, 1)
    assert b1.counters["cost_neg"] == p.counters["cost_neg"]
    assert b1.counters["cost_pos"] == p.counters["cost_pos"] - int((p.sizes() - 1).sum())
    for b in (16, 100, 1024):
        bv = oracle.bvc_labels(g, order, b)
        assert bv.counters["cost_pos"] == bvc_positive_cost(bv, order, b)
        assert bv.counters["cost_pos"] <= p.counters["cost_pos"]


# ---- edge-access and round counters (Algorithm 4's rounds; Section 4.3's edge accesses) ---------------------------

def bvc_edge_accesses(lab: oracle.Labels, order, g, b):
    """Every vertex that accepts entries of batch i in a round sends them
    along all of its edges in the next round (the batch roots send their
    self entry in round 1), so v costs deg(v) edge accesses per distinct
    distance among its batch-i entries."""
    deg = g.degrees()
    total = 0
    for v in range(g.n):
        h, d = lab.of(v)
        bt = h.astype(np.int64) // b
        pairs = np.unique(bt * 256 + d.astype(np.int64))
        total += int(pairs.shape[0]) * int(deg[v])
    return total


def bvc_rounds(lab: oracle.Labels, n, b):
    """A batch runs one round per message distance 1 .. D+1, where D is the
    largest distance among its entries: the round carrying D+1 is the one in
    which nothing is accepted and the batch ends."""
    bt = lab.hub_rank.astype(np.int64) // b
    nb = (n + b - 1) // b
    dmax = np.full(nb, -1, dtype=np.int64)
    np.maximum.at(dmax, bt, lab.dist.astype(np.int64))
    assert (dmax >= 0).all()  # every batch has its roots' self entries
    return int((dmax + 1).sum())


@pytest.mark.parametrize("gi", range(len(small_graphs())))
def test_edge_and_round_counters_match_closed_forms(gi):
    g = small_graphs()[gi]
    if g.n == 0:
        return
    for order in (synth.degree_order(g), random_order(g.n, 5 + gi)):
        p = oracle.pll_labels(g, order)
        # PLL expands every vertex it labels: deg(v) per entry of L(v)
        assert p.counters["edge_accesses"] == int((p.sizes() * g.degrees()).sum())
        for b in sorted({1, 2, 3, 5, g.n}):
            bv = oracle.bvc_labels(g, order, b)
            assert bv.counters["edge_accesses"] == bvc_edge_accesses(bv, order, g, b), b
            assert bv.counters["rounds"] == bvc_rounds(bv, g.n, b), b
            assert bv.counters["batches"] == (g.n + b - 1) // b
            if b == 1:  # one root per batch: PLL's BFS expansions
                assert bv.counters["edge_accesses"] == p.counters["edge_accesses"]


def test_edge_and_round_counters_ba2000():
    g = synth.ba_graph(2000, 4, 1)
    order = synth.degree_order(g)
    for b in (64, 1024):
        bv = oracle.bvc_labels(g, order, b)
        assert bv.counters["edge_accesses"] == bvc_edge_accesses(bv, order, g, b)
        assert bv.counters["rounds"] == bvc_rounds(bv, g.n, b)


def test_budgeted_pll_is_a_prefix_of_pll():
    """The time-bounded PLL (the CPU baseline's sample of long builds) runs
    the first roots in rank order: its lists are exactly the full labels'
    entries whose hub ranks below the roots it ran, and with room for every
    root it is PLL."""
    g = synth.ba_graph(3000, 4, 3)
    order = synth.degree_order(g)
    full = oracle.pll_labels(g, order)
    part, k = oracle.pll_labels_budget(g, order, 1e-4)
    assert 1 <= k <= g.n
    keep = full.hub_rank < k
    owners = np.repeat(np.arange(g.n), full.sizes())
    want_sizes = np.bincount(owners[keep], minlength=g.n)
    assert np.array_equal(part.sizes(), want_sizes)
    assert np.array_equal(part.hub_rank, full.hub_rank[keep])
    assert np.array_equal(part.dist, full.dist[keep])
    whole, k = oracle.pll_labels_budget(g, order, 3600.0)
    assert k == g.n and np.array_equal(whole.offsets, full.offsets) and np.array_equal(whole.hub_rank, full.hub_rank)
