"""GPU parity of the many-graph build (pll_build_labels_batched): one
persistent-kernel launch captured in a hipGraph, one workgroup per graph at
a time.  Every graph's labels must equal the oracle's."""
import numpy as np
import pytest

import oracle
import paper_1906_12018_amd as pll
import synth
from gpu_util import (DEV, assert_answers_match_digests, assert_labels_equal, assert_labels_match_digests, golden,
                      gpu_query, to_dev)

pytestmark = pytest.mark.gpu


def mixed_graphs():
    return [
        synth.ba_graph(2000, 4, 1), synth.path_graph(40), synth.star_graph(30), synth.complete_graph(9),
        synth.random_tree(300, 2), synth.gnp_graph(200, 0.01, 3), synth.ba_graph(5000, 7, 11),
        synth.csr_from_edges(1, np.zeros(0), np.zeros(0)),
        synth.disjoint_union(synth.ba_graph(400, 3, 5), synth.path_graph(12)),
        synth.ba_graph(700, 2, 13), synth.csr_from_edges(5, np.zeros(0), np.zeros(0)),
    ]


@pytest.mark.parametrize("b", [64, 200, 1024])
def test_mixed_graphs_one_launch(b):
    gs = mixed_graphs()
    orders = [synth.degree_order(g) for g in gs]
    idxs = pll.build_labels_batched([to_dev(g, o) for g, o in zip(gs, orders)], batch_size=b)
    assert len(idxs) == len(gs)
    for g, o, idx in zip(gs, orders, idxs):
        want = oracle.pll_labels(g, o)
        assert_labels_equal(idx, want, o)
        info = idx.info()
        assert info["candidates"] + g.n == want.counters["checks"]
        assert info["accepted"] == want.total - g.n
        bvc = oracle.bvc_labels(g, o, b)
        assert (info["check_cost_pos"], info["check_cost_neg"]) == (bvc.counters["cost_pos"], bvc.counters["cost_neg"])
        u, v = synth.query_pairs(g.n, 2000, seed=2)
        assert np.array_equal(gpu_query(idx, u, v), oracle.query(want, u, v))
    # indexes share one output buffer: freeing some keeps the others valid
    for idx in idxs[::2]:
        idx.free()
    g, o, idx = gs[1], orders[1], idxs[1]
    assert_labels_equal(idx, oracle.pll_labels(g, o), o)


def test_batched_recheck_and_relaxed():
    gs = [synth.ba_graph(1500, 5, 21), synth.ba_graph(900, 3, 22)]
    orders = [synth.degree_order(g) for g in gs]
    idxs = pll.build_labels_batched([to_dev(g, o) for g, o in zip(gs, orders)], batch_size=128,
                                    flags=pll.FLAG_RECHECK | pll.FLAG_RELAXED)
    for g, o, idx in zip(gs, orders, idxs):
        assert_labels_equal(idx, oracle.pll_labels(g, o), o)
        assert idx.info()["recheck_removed"] > 0


def test_batched_rejects_invalid_graph():
    good = synth.ba_graph(300, 2, 1)
    bad = synth.ba_graph(300, 2, 2)
    bo = synth.degree_order(bad).copy()
    bo[3] = bo[4]
    with pytest.raises(pll.PllError) as e:
        pll.build_labels_batched([to_dev(good, synth.degree_order(good)), to_dev(bad, bo)])
    assert e.value.status == pll.PLL_EINVAL


def test_batching_workload_256_graphs():
    """The 256-graph workload (n log-uniform in [500, 20000], m in {2..8}) in
    one launch: every graph's labels hash to the oracle's stored digests
    (Definition 2 via PLL), and every graph answers its 2,000 seed-2 pairs as
    the oracle does; a sample is also compared entry by entry with the
    oracle run here."""
    want = golden("batch256")["graphs"]
    specs = synth.batching_specs()
    assert len(specs) == len(want) == 256
    gs = [synth.ba_graph(n, m, sd) for n, m, sd in specs]
    orders = [synth.degree_order(g) for g in gs]
    idxs = pll.build_labels_batched([to_dev(g, o) for g, o in zip(gs, orders)])
    for i, (g, idx) in enumerate(zip(gs, idxs)):
        assert (want[i]["n"], want[i]["m"], want[i]["seed"]) == (g.n, specs[i][1], specs[i][2])
        assert_labels_match_digests(idx, want[i], f"graph {i}")
        u, v = synth.query_pairs(g.n, 2000, seed=2)
        assert_answers_match_digests(gpu_query(idx, u, v), want[i]["pairs"], f"graph {i}")
    sizes = np.array([g.n for g in gs])
    for i in sorted({int(np.argmax(sizes)), int(np.argmin(sizes)), 17}):
        assert_labels_equal(idxs[i], oracle.pll_labels(gs[i], orders[i]), orders[i])
    for idx in idxs:
        idx.free()


@pytest.mark.parametrize("gang_scale,max_gang", [(100, 1), (100, 4), (300, 16), (50, 16)])
def test_gang_sizes_do_not_change_labels(gang_scale, max_gang):
    """Graphs built by gangs of 1..16 workgroups (barriers between phases)
    give the oracle's labels whatever the gang sizes."""
    gs = [synth.ba_graph(6000, 6, 31), synth.ba_graph(3000, 8, 32), synth.ba_graph(800, 3, 33),
          synth.gnp_graph(500, 0.02, 34)]
    orders = [synth.degree_order(g) for g in gs]
    idxs = pll.build_labels_batched([to_dev(g, o) for g, o in zip(gs, orders)], batch_size=512,
                                    gang_scale=gang_scale, max_gang=max_gang)
    gangs = [i.info()["gang"] for i in idxs]
    assert max(gangs) <= max_gang
    for g, o, idx in zip(gs, orders, idxs):
        want = oracle.pll_labels(g, o)
        assert_labels_equal(idx, want, o)
        assert idx.info()["candidates"] + g.n == want.counters["checks"]


def test_small_persistent_launch():
    """A launch capped at a few workgroups (max_workgroups) still builds
    every graph exactly: gangs shrink to fit and take graphs in turn."""
    gs = [synth.ba_graph(3000, 5, 61), synth.ba_graph(700, 2, 62), synth.star_graph(50), synth.ba_graph(1800, 7, 63)]
    orders = [synth.degree_order(g) for g in gs]
    for cap in (1, 3):
        idxs = pll.build_labels_batched([to_dev(g, o) for g, o in zip(gs, orders)], batch_size=256,
                                        max_workgroups=cap)
        for g, o, idx in zip(gs, orders, idxs):
            assert idx.info()["gang"] <= cap
            assert_labels_equal(idx, oracle.pll_labels(g, o), o)


def test_autotuner_picks_a_candidate_and_caches(tmp_path, monkeypatch):
    from paper_1906_12018_amd import autotune
    monkeypatch.setenv("PLL_TUNE_CACHE", str(tmp_path / "tune.json"))
    gs = [synth.ba_graph(n, 3, 40 + n) for n in (900, 1500, 2500)]
    orders = [synth.degree_order(g) for g in gs]
    dev = [to_dev(g, o) for g, o in zip(gs, orders)]
    cands = [dict(batch_size=256, gang_scale=100, max_gang=16), dict(batch_size=1024, gang_scale=200, max_gang=4)]
    res = autotune.tune_batched(dev, candidates=cands, reps=1)
    assert res["best"] in cands and len(res["results"]) == 2
    assert autotune.cached_config(dev) == res["best"]
    idxs = autotune.build_tuned(dev)
    for g, o, idx in zip(gs, orders, idxs):
        assert_labels_equal(idx, oracle.pll_labels(g, o), o)
