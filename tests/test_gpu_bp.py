"""GPU parity of bit-parallel labels (Section 5.2): the BP roots, their
neighbour sets, d / S^-1 / S^0 of every vertex, the normal labels the
batches then build over the unused vertices, and the queries (BP bound and
2-hop merge), against the bit-parallel oracle through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import paper_1906_12018_amd as pll
import synth
from gpu_util import DEV, assert_labels_equal, build, gpu_query, to_dev

pytestmark = pytest.mark.gpu


def check_bp(idx, g, order, t, pairs=3000, seed=2):
    lab, bp = oracle.pll_labels_bp(g, order, t)
    assert_labels_equal(idx, lab, order)
    info = idx.info()
    assert info["bp_roots"] == bp.t
    nused = int(bp.t + (bp.nbr != oracle.DIST_INF).sum())
    assert info["bp_vertices"] == nused
    # Corollary 2 with BP: the rounds check the pairs the sequential searches
    # pop, minus the roots; the BP bound decides the same ones
    assert info["candidates"] + (g.n - nused) == lab.counters["checks"]
    assert info["bp_pruned"] == lab.counters["bp_pruned"]
    ex = idx.export_bp()
    torch.cuda.synchronize()
    assert np.array_equal(ex["roots"].cpu().numpy().view(np.uint32), bp.root)
    assert np.array_equal(ex["nbrs"].cpu().numpy().view(np.uint32), bp.nbr)
    assert np.array_equal(ex["dist"].cpu().numpy(), bp.dist)
    assert np.array_equal(ex["sm1"].cpu().numpy().view(np.uint64), bp.sm1)
    assert np.array_equal(ex["s0"].cpu().numpy().view(np.uint64), bp.s0)
    if g.n:
        u, v = synth.query_pairs(g.n, pairs, seed=seed)
        assert np.array_equal(gpu_query(idx, u, v), oracle.query_bp(lab, bp, u, v))
    return lab, bp


def cases():
    return [synth.path_graph(70), synth.star_graph(200), synth.random_tree(300, 3),
            synth.gnp_graph(150, 0.05, 9), synth.gnp_graph(90, 0.01, 4),
            synth.disjoint_union(synth.ba_graph(300, 2, 8), synth.complete_graph(7), synth.path_graph(5)),
            synth.ba_graph(700, 5, 12), synth.rmat_graph(10, 8, seed=3)]


@pytest.mark.parametrize("t", [1, 4, 16, 64])
@pytest.mark.parametrize("b", [1, 65, 1024])
@pytest.mark.parametrize("gi", range(len(cases())))
def test_bp_small_graphs(gi, b, t):
    g = cases()[gi]
    order = synth.degree_order(g)
    idx = build(g, order, batch_size=b, bp_roots=t)
    check_bp(idx, g, order, t)
    idx.free()


def test_bp_ba2000_and_random_order():
    g = synth.ba_graph(2000, 4, 1)
    order = synth.degree_order(g)
    idx = build(g, order, bp_roots=16)
    lab, _ = check_bp(idx, g, order, 16, pairs=100_000)
    assert lab.total < oracle.pll_labels(g, order).total
    order = np.argsort(synth.splitmix64(7, 0, g.n), kind="stable").astype(np.uint32)
    idx = build(g, order, batch_size=256, bp_roots=8)
    check_bp(idx, g, order, 8)


@pytest.mark.parametrize("lanes", [1, 4, 16, 64, 0])
def test_bp_query_lanes(lanes):
    g = synth.rmat_graph(12, 16, seed=1)
    order = synth.degree_order(g)
    lab, bp = oracle.pll_labels_bp(g, order, 16)
    idx = build(g, order, bp_roots=16, query_lanes=lanes)
    u, v = synth.query_pairs(g.n, 50_000, seed=5)
    u[:3] = g.n + np.arange(3)  # out of range: no label, no BP data
    want = oracle.query_bp(lab, bp, np.minimum(u, g.n - 1), v)
    want[:3] = oracle.DIST_INF
    assert np.array_equal(gpu_query(idx, u, v), want)


def test_bp_rmat16():
    """R-MAT-16 (the bench graph), degree order, b = 1024, 16 BP roots."""
    g = synth.rmat_graph(16, 16, seed=1)
    order = synth.degree_order(g)
    idx = build(g, order, bp_roots=16)
    check_bp(idx, g, order, 16, pairs=200_000)


def test_bp_edge_cases_and_errors():
    # every vertex used by BP: no normal labels at all, queries from BP alone
    p = synth.path_graph(5)
    idx = build(p, np.arange(5, dtype=np.uint32), bp_roots=64)
    check_bp(idx, p, np.arange(5, dtype=np.uint32), 64)
    assert idx.info()["total_entries"] == 0 and idx.info()["bp_roots"] == 3
    g = synth.ba_graph(300, 3, 4)
    order = synth.degree_order(g)
    rp, cl, od = to_dev(g, order)
    for kw in ({"bp_roots": 65}, {"bp_roots": 4, "flags": pll.FLAG_PERSISTENT}):
        with pytest.raises(pll.PllError) as e:
            pll.build_labels(rp, cl, od, **kw)
        assert e.value.status == pll.PLL_EINVAL
    with pytest.raises(pll.PllError) as e:
        o = pll._opts(1024, 0, 0, 0, bp_roots=4)
        import ctypes
        descs = (pll.GraphDesc * 1)()
        descs[0].n, descs[0].nnz = g.n, g.nnz
        descs[0].d_row_ptr, descs[0].d_col, descs[0].d_order = rp.data_ptr(), cl.data_ptr(), od.data_ptr()
        outs = (ctypes.c_void_p * 1)()
        rc = pll.load_library().pll_build_labels_batched(1, descs, ctypes.byref(o), None, outs)
        if rc:
            raise pll.PllError(rc, "batched")
    assert e.value.status == pll.PLL_EINVAL
    # no BP roots asked: no BP data, labels are the canonical ones
    idx = build(g, order, bp_roots=0)
    assert idx.info()["bp_roots"] == 0
    assert_labels_equal(idx, oracle.pll_labels(g, order), order)
