"""GPU parity of the weighted build (Section 5.1: rounds as Bellman-Ford
iterations with per-candidate distances, batch-end recheck) against the
weighted oracle (PLL with Dijkstra), through the C ABI, on seeded graphs
with weights uniform in 1..7 (the paper's recipe for its weighted runs).
Labels must match bit for bit and every query must be exact."""
import numpy as np
import pytest
import torch

import oracle
import paper_1906_12018_amd as pll
import synth
from gpu_util import DEV, assert_labels_equal, gpu_query, to_dev

pytestmark = pytest.mark.gpu


def build_w(g, order, **kw):
    rp, cl, od = to_dev(g, order)
    wt = torch.from_numpy(np.ascontiguousarray(g.w, dtype=np.uint8)).to(DEV)
    return pll.build_labels_weighted(rp, cl, wt, od, **kw)


def check_weighted(idx, g, order, pairs=3000, seed=2):
    want = oracle.pll_labels_weighted(g, order)
    assert_labels_equal(idx, want, order)
    info = idx.info()
    assert info["weighted"] == 1 and info["directed"] == 0
    assert info["total_entries"] == want.total
    assert info["max_dist"] == (int(want.dist.max()) if want.total else 0)
    # every kept entry was accepted once at its final distance; the rest of
    # the accepted entries were shorter-later duplicates or removed by the recheck
    assert info["accepted"] >= want.total - g.n
    if g.n:
        u, v = synth.query_pairs(g.n, pairs, seed=seed)
        assert np.array_equal(gpu_query(idx, u, v), oracle.query(want, u, v))
    return want, info


def small_wgraphs():
    return [
        synth.with_weights(synth.path_graph(2), seed=1), synth.with_weights(synth.path_graph(40), seed=2),
        synth.with_weights(synth.star_graph(9), seed=3), synth.with_weights(synth.complete_graph(12), seed=4),
        synth.with_weights(synth.random_tree(200, 3), seed=5), synth.with_weights(synth.gnp_graph(150, 0.05, 9), seed=6),
        synth.with_weights(synth.gnp_graph(90, 0.01, 4), seed=7),
        synth.with_weights(synth.ba_graph(700, 5, 12), seed=8),
        synth.with_weights(synth.ba_graph(500, 3, 13), 1, 30, seed=9),
    ]


@pytest.mark.parametrize("b", [1, 5, 64, 65, 512, 1024])
@pytest.mark.parametrize("gi", range(len(small_wgraphs())))
def test_small_weighted_labels_and_queries(gi, b):
    g = small_wgraphs()[gi]
    order = synth.degree_order(g)
    idx = build_w(g, order, batch_size=b)
    check_weighted(idx, g, order)
    idx.free()


def test_unit_weights_need_no_recheck():
    """With every weight 1 a round is a distance again: nothing non-canonical
    is accepted, the recheck removes nothing, and the labels are the
    unweighted ones."""
    g = synth.ba_graph(2000, 4, 1)
    order = synth.degree_order(g)
    idx = build_w(synth.constant_weights(g, 1), order)
    want = oracle.pll_labels(g, order)
    assert_labels_equal(idx, want, order)
    info = idx.info()
    assert info["recheck_removed"] == 0 and info["accepted"] == want.total - g.n


def test_ba2000_weighted_full_parity():
    g = synth.with_weights(synth.ba_graph(2000, 4, 1))
    order = synth.degree_order(g)
    idx = build_w(g, order, batch_size=512)
    _, info = check_weighted(idx, g, order, pairs=100_000)
    assert info["recheck_removed"] > 0  # the recheck is load-bearing on weighted graphs


@pytest.mark.parametrize("scale", [12, 14])
def test_rmat_weighted_parity(scale):
    """R-MAT, edge factor 16, weights uniform 1..7 (stream 5), degree order."""
    g = synth.with_weights(synth.rmat_graph(scale, 16, seed=1))
    order = synth.degree_order(g)
    for b in (512, 1024):
        idx = build_w(g, order, batch_size=b)
        check_weighted(idx, g, order, pairs=50_000)
        idx.free()


def test_random_orders_weighted():
    g = synth.with_weights(synth.ba_graph(1500, 3, 21), seed=11)
    for s in (5, 6):
        order = np.argsort(synth.splitmix64(s, 0, g.n), kind="stable").astype(np.uint32)
        idx = build_w(g, order, batch_size=256)
        check_weighted(idx, g, order)
        idx.free()


def test_weighted_errors_and_edge_cases():
    g = synth.with_weights(synth.ba_graph(300, 3, 14))
    order = synth.degree_order(g)
    rp, cl, od = to_dev(g, order)
    wt = torch.from_numpy(g.w.copy()).to(DEV)
    for flags in (pll.FLAG_RECHECK | pll.FLAG_RELAXED, pll.FLAG_PERSISTENT):
        with pytest.raises(pll.PllError) as e:
            pll.build_labels_weighted(rp, cl, wt, od, flags=flags)
        assert e.value.status == pll.PLL_EINVAL
    zero = wt.clone()
    zero[7] = 0
    with pytest.raises(pll.PllError) as e:
        pll.build_labels_weighted(rp, cl, zero, od, flags=0)
    assert e.value.status == pll.PLL_EINVAL
    # one arc of an edge with another weight: rejected under validation
    asym = wt.clone()
    asym[0] = int(asym[0]) % 7 + 1
    with pytest.raises(pll.PllError) as e:
        pll.build_labels_weighted(rp, cl, asym, od, flags=pll.FLAG_VALIDATE)
    assert e.value.status == pll.PLL_EINVAL
    idx = pll.build_labels_weighted(rp, cl, wt, od, flags=pll.FLAG_VALIDATE | pll.FLAG_PROFILE)
    check_weighted(idx, g, order)
    # distances of 255 or more do not fit
    p = synth.constant_weights(synth.path_graph(52), 5)
    with pytest.raises(pll.PllError) as e:
        build_w(p, np.arange(52, dtype=np.uint32))
    assert e.value.status == pll.PLL_EDIST
    p = synth.constant_weights(synth.path_graph(51), 5)
    idx = build_w(p, np.arange(51, dtype=np.uint32))
    check_weighted(idx, p, np.arange(51, dtype=np.uint32))
    assert idx.info()["max_dist"] == 250
    # no vertices; no edges
    e0 = synth.WGraph(n=0, row_ptr=np.zeros(1, dtype=np.uint64), col=np.zeros(0, dtype=np.uint32),
                      w=np.zeros(0, dtype=np.uint8))
    idx = build_w(e0, np.zeros(0, dtype=np.uint32))
    assert idx.info()["weighted"] == 1 and idx.info()["total_entries"] == 0
    iso = synth.WGraph(n=5, row_ptr=np.zeros(6, dtype=np.uint64), col=np.zeros(0, dtype=np.uint32),
                       w=np.zeros(0, dtype=np.uint8))
    idx = build_w(iso, np.arange(5, dtype=np.uint32))
    check_weighted(idx, iso, np.arange(5, dtype=np.uint32))
