"""GPU parity of the four-receivers-per-wave check (rounds with many
receivers run it on their own; PLL_FLAG_PACK4 makes every fused round run it,
so the small graphs below cover it too) against the oracle: labels bit for
bit, Algorithm 4's counters and exact queries, as for the one-receiver check.
Cases: the small-graph set at several batch sizes (ragged last batches, one
candidate word and sixteen), relaxed rounds with the recheck, multi-batch
graphs with large rounds, pulled rounds, trailing isolated vertices, random
orders and the distance overflow."""
import numpy as np
import pytest

import oracle
import paper_1906_12018_amd as pll
import synth
from gpu_util import assert_labels_equal, build, check_counters, gpu_query
from test_gpu_build import small_cases
from test_gpu_bp import check_bp
from test_gpu_directed import build_dir, check_directed, small_digraphs
from test_gpu_weighted import build_w, check_weighted, small_wgraphs

pytestmark = pytest.mark.gpu

PACK = pll.FLAG_VALIDATE | pll.FLAG_PACK4


@pytest.mark.parametrize("b", [1, 5, 64, 65, 130, 1024])
@pytest.mark.parametrize("gi", range(len(small_cases())))
def test_small_graphs_packed(gi, b):
    g = small_cases()[gi]
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    idx = build(g, order, batch_size=b, flags=PACK)
    assert_labels_equal(idx, want, order)
    check_counters(idx, g, order, b, want)
    u, v = synth.query_pairs(g.n, 3000, seed=2)
    assert np.array_equal(gpu_query(idx, u, v), oracle.query(want, u, v))
    idx.free()


@pytest.mark.parametrize("b", [64, 1024])
def test_relaxed_rounds_packed(b):
    g = synth.ba_graph(2000, 4, 1)
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    idx = build(g, order, batch_size=b, flags=pll.FLAG_RECHECK | pll.FLAG_RELAXED | pll.FLAG_PACK4)
    assert_labels_equal(idx, want, order)
    info = idx.info()
    assert info["recheck_removed"] > 0
    assert info["accepted"] - info["recheck_removed"] == want.total - g.n
    idx.free()


@pytest.mark.parametrize("n,m,seed,b", [(4797, 3, 1001, 1024), (7051, 8, 1007, 300), (12000, 6, 77, 1024)])
def test_many_batches_large_rounds_packed(n, m, seed, b):
    g = synth.ba_graph(n, m, seed)
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    idx = build(g, order, batch_size=b, flags=PACK)
    assert_labels_equal(idx, want, order)
    check_counters(idx, g, order, b, want)
    u, v = synth.query_pairs(g.n, 20000, seed=3)
    assert np.array_equal(gpu_query(idx, u, v), oracle.query(want, u, v))
    idx.free()


def test_pulled_rounds_packed():
    """Rounds after one with at least n/2 receivers are pulled; the packed
    check then records where each receiver's delta L is."""
    g = synth.ba_graph(20000, 4, 3)
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    idx = build(g, order, flags=PACK | pll.FLAG_PROFILE)
    assert_labels_equal(idx, want, order)
    info = check_counters(idx, g, order, 1024, want)
    assert info["phase_launches"]["push"] > info["batches"]
    u, v = synth.query_pairs(g.n, 50_000, seed=4)
    assert np.array_equal(gpu_query(idx, u, v), oracle.query(want, u, v))
    idx.free()


@pytest.mark.parametrize("b", [64, 1024])
def test_trailing_isolated_and_random_orders_packed(b):
    core = synth.ba_graph(1200, 3, 31)
    g = synth.disjoint_union(core, synth.csr_from_edges(700, np.zeros(0), np.zeros(0)))
    for order in (synth.degree_order(g),
                  np.argsort(synth.splitmix64(5, 0, g.n), kind="stable").astype(np.uint32)):
        want = oracle.pll_labels(g, order)
        idx = build(g, order, batch_size=b, flags=PACK)
        assert_labels_equal(idx, want, order)
        check_counters(idx, g, order, b, want)
        idx.free()


def test_distance_overflow_packed():
    g = synth.path_graph(300)
    with pytest.raises(pll.PllError) as e:
        build(g, synth.degree_order(g), batch_size=32, flags=PACK)
    assert e.value.status == pll.PLL_EDIST
    g = synth.path_graph(256)
    order = synth.degree_order(g)
    idx = build(g, order, batch_size=32, flags=PACK)
    assert_labels_equal(idx, oracle.pll_labels(g, order), order)
    idx.free()


@pytest.mark.parametrize("b", [1, 64, 1024])
@pytest.mark.parametrize("gi", range(0, len(small_digraphs()), 3))
def test_directed_builds_ignore_the_flag(gi, b):
    """The directed build keeps one receiver per wave (packing measured
    slower there): with the flag its labels are still the oracle's."""
    g = small_digraphs()[gi]
    order = synth.degree_order_directed(g)
    idx = build_dir(g, order, batch_size=b, flags=PACK)
    check_directed(idx, g, order)
    idx.free()


@pytest.mark.parametrize("b", [64, 1024])
def test_weighted_and_bit_parallel_builds_ignore_the_flag(b):
    """Weighted and bit-parallel builds have checks of their own: with the
    flag their labels, counters and queries are still the oracles'."""
    for g in small_wgraphs()[-2:]:
        order = synth.degree_order(g)
        idx = build_w(g, order, batch_size=b, flags=PACK)
        check_weighted(idx, g, order)
        idx.free()
    g = synth.ba_graph(700, 5, 12)
    order = synth.degree_order(g)
    idx = build(g, order, batch_size=b, bp_roots=4, flags=PACK)
    check_bp(idx, g, order, 4)
    idx.free()
