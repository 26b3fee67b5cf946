"""GPU parity of the batched merge-join query for every lanes-per-pair
setting: the scalar merge (1 lane) and the windowed group merge (4..64 lanes,
windows of 4 entries per lane).  Distances are integers: compared exactly
with the oracle's query on the same labels."""
import numpy as np
import torch
import pytest

import oracle
import paper_1906_12018_amd as pll
import synth
from gpu_util import DEV, build, gpu_query, to_dev

pytestmark = pytest.mark.gpu

LANES = [1, 4, 8, 16, 32, 64]


@pytest.fixture(scope="module")
def ba5000():
    g = synth.ba_graph(5000, 5, 3)
    o = synth.degree_order(g)
    return g, o, oracle.pll_labels(g, o)


@pytest.mark.parametrize("lanes", LANES + [0])
def test_query_lanes_match_oracle(ba5000, lanes):
    g, o, want = ba5000
    idx = build(g, o, query_lanes=lanes)
    u, v = synth.query_pairs(g.n, 100_000, seed=21)
    assert np.array_equal(gpu_query(idx, u, v), oracle.query(want, u, v))
    # every vertex against itself and against the highest and lowest ranks
    ids = np.arange(g.n, dtype=np.uint32)
    for other in (ids, np.full(g.n, o[0], np.uint32), np.full(g.n, o[-1], np.uint32)):
        assert np.array_equal(gpu_query(idx, ids, other), oracle.query(want, ids, other))
    idx.free()


@pytest.mark.parametrize("lanes", LANES)
def test_query_lanes_disconnected_and_out_of_range(lanes):
    # two components plus isolated vertices: unreachable pairs and labels of
    # one entry; ids >= n answer "no common hub"
    g = synth.disjoint_union(synth.ba_graph(800, 3, 5), synth.path_graph(200),
                             synth.csr_from_edges(7, np.zeros(0), np.zeros(0)))
    o = synth.degree_order(g)
    want = oracle.pll_labels(g, o)
    idx = build(g, o, query_lanes=lanes)
    u, v = synth.query_pairs(g.n, 50_000, seed=4)
    assert np.array_equal(gpu_query(idx, u, v), oracle.query(want, u, v))
    bad_u = np.array([g.n, 0, g.n + 5, 0xFFFFFFFF, 3], dtype=np.uint32)
    bad_v = np.array([0, g.n, 1, 2, 0xFFFFFFFF], dtype=np.uint32)
    assert np.all(gpu_query(idx, bad_u, bad_v) == 0xFFFFFFFF)
    idx.free()


@pytest.mark.parametrize("lanes", [4, 16, 64])
def test_query_lanes_on_batched_indexes(lanes):
    """Indexes of the many-graph build share one store; each graph's labels
    start on a 4-entry boundary of it, so every window load is aligned."""
    gs = [synth.ba_graph(n, m, 50 + n) for n, m in ((777, 3), (1201, 5), (93, 2), (2500, 7), (5, 2))]
    orders = [synth.degree_order(g) for g in gs]
    idxs = pll.build_labels_batched([to_dev(g, o) for g, o in zip(gs, orders)], batch_size=256,
                                    query_lanes=lanes)
    for g, o, idx in zip(gs, orders, idxs):
        want = oracle.pll_labels(g, o)
        u, v = synth.query_pairs(g.n, 20_000, seed=6)
        assert np.array_equal(gpu_query(idx, u, v), oracle.query(want, u, v))


def test_query_lanes_rejects_other_values():
    g = synth.ba_graph(100, 2, 1)
    with pytest.raises(pll.PllError) as e:
        build(g, synth.degree_order(g), query_lanes=3)
    assert e.value.status == pll.PLL_EINVAL


def test_query_lane_autotuner_keeps_answers():
    """The query autotuner times every lanes value on the caller's pairs,
    refuses a value whose answers differ and sets the fastest; the answers
    afterwards are still the oracle's."""
    from paper_1906_12018_amd import autotune
    g = synth.rmat_graph(12, 16, seed=1)
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    idx = build(g, order)
    u, v = synth.query_pairs(g.n, 20000, seed=9)
    du = torch.from_numpy(u.view(np.int32)).to(DEV)
    dv = torch.from_numpy(v.view(np.int32)).to(DEV)
    res = autotune.tune_query(idx, du, dv, reps=1, save=False)
    assert res["best"] in autotune.QUERY_LANES and len(res["results"]) == len(autotune.QUERY_LANES)
    assert np.array_equal(gpu_query(idx, u, v), oracle.query(want, u, v))
    with pytest.raises(pll.PllError) as e:
        idx.set_query_lanes(3)
    assert e.value.status == pll.PLL_EINVAL
