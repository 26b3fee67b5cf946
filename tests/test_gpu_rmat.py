"""Full-size GPU parity on the R-MAT scale-16 graph, in the launch
configuration the bench times (b = 1024, profiling on): every label entry
against the oracle's PLL, and the 10^6 query pairs of seed 2."""
import numpy as np
import pytest

import oracle
import paper_1906_12018_amd as pll
import synth
from gpu_util import assert_labels_equal, build, check_counters, gpu_query

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rmat16():
    g = synth.rmat_graph(16)
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    return g, order, want


def test_rmat16_labels_bit_exact(rmat16):
    g, order, want = rmat16
    idx = build(g, order, batch_size=1024, flags=pll.FLAG_PROFILE)
    assert_labels_equal(idx, want, order)
    info = check_counters(idx, g, order, 1024, want)
    assert info["batches"] == 64
    u, v = synth.query_pairs(g.n, 1_000_000, seed=2)
    got = gpu_query(idx, u, v)
    assert np.array_equal(got, oracle.query(want, u, v))
    # isolated vertices: only their self entry, unreachable from everything else
    iso = np.flatnonzero(g.degrees() == 0)[:50].astype(np.uint32)
    assert np.all(gpu_query(idx, iso, np.full_like(iso, order[0])) == pll.DIST_INF)
    assert np.all(gpu_query(idx, iso, iso) == 0)


def test_rmat16_queries_match_bfs_sample(rmat16):
    """Independent of the oracle's labels: BFS distances from sampled sources."""
    g, order, _ = rmat16
    idx = build(g, order, batch_size=1024, flags=pll.FLAG_PROFILE)
    srcs = synth.bounded(synth.splitmix64(31, 0, 6), g.n)
    for s in srcs:
        d = oracle.bfs(g, int(s))
        got = gpu_query(idx, np.full(g.n, s, dtype=np.uint32), np.arange(g.n, dtype=np.uint32))
        assert np.array_equal(got, d)


def test_rmat16_persistent_loop(rmat16):
    """The persistent batch loop on the full graph, including its hand-backs
    to the host for label-arena compaction."""
    g, order, want = rmat16
    idx = build(g, order, batch_size=1024, flags=pll.FLAG_PROFILE | pll.FLAG_PERSISTENT)
    assert_labels_equal(idx, want, order)
    info = check_counters(idx, g, order, 1024, want)
    assert info["phase_launches"]["loop"] >= 1
