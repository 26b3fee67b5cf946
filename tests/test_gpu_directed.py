"""GPU parity of the directed build (Section 5.1: L_in / L_out labels from
forward and backward searches in lockstep rounds) and of the directed query
(L_out(u) merged with L_in(v)) against the directed oracle, through the C
ABI, on seeded digraphs.  Labels must match bit for bit on both sides and
every query must be exact."""
import numpy as np
import pytest
import torch

import oracle
import paper_1906_12018_amd as pll
import synth
from gpu_util import DEV, gpu_query, to_dev

pytestmark = pytest.mark.gpu


def build_dir(g, order, **kw):
    rp, cl, od = to_dev(g, order)
    return pll.build_labels_directed(rp, cl, od, **kw)


def exported_side(idx, side):
    ex = idx.export(side=side)
    torch.cuda.synchronize()
    return ex.offsets.cpu().numpy().view(np.uint64), ex.hubs.cpu().numpy().view(np.uint32), ex.dists.cpu().numpy()


def assert_side_equal(idx, side, want: oracle.Labels, order, what):
    off, hubs, dists = exported_side(idx, side)
    assert np.array_equal(off, want.offsets), f"{what}: offsets differ"
    assert np.array_equal(hubs, want.hubs_as_ids(order)), f"{what}: hubs differ"
    assert np.array_equal(dists, want.dist), f"{what}: dists differ"


def check_directed(idx, g, order, pairs=3000, seed=2):
    lin, lout = oracle.pll_labels_directed(g, order)
    assert_side_equal(idx, pll.LABELS_IN, lin, order, "L_in")
    assert_side_equal(idx, pll.LABELS_OUT, lout, order, "L_out")
    info = idx.info()
    assert info["directed"] == 1
    assert info["in_entries"] == lin.total and info["out_entries"] == lout.total
    assert info["total_entries"] == lin.total + lout.total
    # every entry but the 2n self entries is accepted by a round check, and
    # each side's checks are the oracle search's pops minus its n roots
    assert info["accepted"] == lin.total + lout.total - 2 * g.n
    assert info["candidates"] + 2 * g.n == lin.counters["checks"] + lout.counters["checks"]
    if g.n:
        u, v = synth.query_pairs(g.n, pairs, seed=seed)
        assert np.array_equal(gpu_query(idx, u, v), oracle.query_directed(lin, lout, u, v))
    return lin, lout


def small_digraphs():
    return [
        synth.directed_path(2), synth.directed_path(70), synth.directed_cycle(50),
        synth.gnp_digraph(40, 0.05, 1), synth.gnp_digraph(120, 0.03, 2), synth.gnp_digraph(90, 0.008, 3),
        synth.rmat_digraph(8, 4, seed=4), synth.rmat_digraph(10, 6, seed=5),
        synth.as_digraph(synth.ba_graph(400, 3, 6)),
    ]


@pytest.mark.parametrize("b", [1, 5, 64, 65, 1024])
@pytest.mark.parametrize("gi", range(len(small_digraphs())))
def test_small_digraphs_labels_and_queries(gi, b):
    g = small_digraphs()[gi]
    order = synth.degree_order_directed(g)
    idx = build_dir(g, order, batch_size=b)
    check_directed(idx, g, order)
    idx.free()


def test_random_orders_and_recheck():
    g = synth.rmat_digraph(11, 6, seed=8)
    for s in (3, 4):
        order = np.argsort(synth.splitmix64(s, 0, g.n), kind="stable").astype(np.uint32)
        idx = build_dir(g, order, batch_size=256)
        check_directed(idx, g, order)
        idx.free()
    order = synth.degree_order_directed(g)
    idx = build_dir(g, order, flags=pll.FLAG_VALIDATE | pll.FLAG_RECHECK)
    check_directed(idx, g, order)
    assert idx.info()["recheck_removed"] == 0
    idx.free()


def test_symmetric_digraph_gives_the_undirected_labels():
    g = synth.ba_graph(1500, 4, 9)
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    idx = build_dir(synth.as_digraph(g), order)
    assert_side_equal(idx, pll.LABELS_IN, want, order, "L_in")
    assert_side_equal(idx, pll.LABELS_OUT, want, order, "L_out")
    u, v = synth.query_pairs(g.n, 20000, seed=3)
    assert np.array_equal(gpu_query(idx, u, v), oracle.query(want, u, v))


@pytest.mark.parametrize("lanes", [1, 4, 8, 16, 32, 64, 0])
def test_query_lanes_directed(lanes):
    g = synth.rmat_digraph(12, 8, seed=10)
    order = synth.degree_order_directed(g)
    lin, lout = oracle.pll_labels_directed(g, order)
    idx = build_dir(g, order, query_lanes=lanes)
    u, v = synth.query_pairs(g.n, 50000, seed=11)
    # out-of-range ids have no label
    u[:5] = g.n + np.arange(5)
    v[5:10] = 0xFFFFFFFF
    want = oracle.query_directed(lin, lout, np.minimum(u, g.n - 1), np.minimum(v, g.n - 1))
    want[:10] = oracle.DIST_INF
    assert np.array_equal(gpu_query(idx, u, v), want)


def test_rmat16_directed_parity():
    """Directed R-MAT, scale 16, edge factor 16 (arcs not symmetrised), total-degree order, b = 1024."""
    g = synth.rmat_digraph(16, 16, seed=1)
    order = synth.degree_order_directed(g)
    idx = build_dir(g, order)
    check_directed(idx, g, order, pairs=200_000, seed=2)


def test_directed_errors_and_edge_cases():
    g = synth.rmat_digraph(7, 4, seed=12)
    order = synth.degree_order_directed(g)
    rp, cl, od = to_dev(g, order)
    for flags in (pll.FLAG_RECHECK | pll.FLAG_RELAXED, pll.FLAG_PERSISTENT):
        with pytest.raises(pll.PllError) as e:
            pll.build_labels_directed(rp, cl, od, flags=flags)
        assert e.value.status == pll.PLL_EINVAL
    bad = od.clone()
    bad[1] = bad[0]
    with pytest.raises(pll.PllError) as e:
        pll.build_labels_directed(rp, cl, bad)
    assert e.value.status == pll.PLL_EINVAL
    # a self-loop fails validation; an asymmetric graph passes it
    loop = synth.DiGraph(n=3, row_ptr=np.array([0, 1, 2, 2], dtype=np.uint64), col=np.array([0, 2], dtype=np.uint32))
    lrp, lcl, lod = to_dev(loop, np.arange(3, dtype=np.uint32))
    with pytest.raises(pll.PllError) as e:
        pll.build_labels_directed(lrp, lcl, lod)
    assert e.value.status == pll.PLL_EINVAL
    idx = pll.build_labels_directed(rp, cl, od)
    check_directed(idx, g, order)
    # distances of 255 or more do not fit the labels
    p = synth.directed_path(256)
    prp, pcl, pod = to_dev(p, np.arange(256, dtype=np.uint32))
    with pytest.raises(pll.PllError) as e:
        pll.build_labels_directed(prp, pcl, pod)
    assert e.value.status == pll.PLL_EDIST
    p = synth.directed_path(255)
    idx = build_dir(p, np.arange(255, dtype=np.uint32))
    lin, lout = check_directed(idx, p, np.arange(255, dtype=np.uint32))
    assert idx.info()["max_dist"] == 254
    assert np.array_equal(gpu_query(idx, np.array([0, 254]), np.array([254, 0])),
                          np.array([254, oracle.DIST_INF], dtype=np.uint32))
    # no vertices
    e0 = synth.DiGraph(n=0, row_ptr=np.zeros(1, dtype=np.uint64), col=np.zeros(0, dtype=np.uint32))
    idx = build_dir(e0, np.zeros(0, dtype=np.uint32))
    info = idx.info()
    assert info["directed"] == 1 and info["total_entries"] == 0
    ex = idx.export(side=pll.LABELS_OUT)
    assert ex.offsets.numel() == 1
    # an undirected index exports the same label on both sides
    und = synth.ba_graph(200, 2, 13)
    from gpu_util import build
    ui = build(und, synth.degree_order(und))
    a, b = exported_side(ui, pll.LABELS_IN), exported_side(ui, pll.LABELS_OUT)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert ui.info()["in_entries"] == ui.info()["out_entries"] == ui.info()["total_entries"]
