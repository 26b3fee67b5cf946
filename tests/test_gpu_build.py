"""GPU parity of the label build and the query (HIP path through the C ABI)
against the oracle on the same seeded inputs.  Labels must match bit for
bit; every query must be exact."""
import numpy as np
import pytest
import torch

import oracle
import paper_1906_12018_amd as pll
import synth
from gpu_util import DEV, assert_labels_equal, build, check_counters, gpu_query, to_dev

pytestmark = pytest.mark.gpu


def small_cases():
    cases = [
        synth.path_graph(2), synth.path_graph(3), synth.path_graph(70), synth.star_graph(9),
        synth.complete_graph(12), synth.random_tree(200, 3), synth.gnp_graph(150, 0.05, 9),
        synth.gnp_graph(90, 0.01, 4),  # many isolated vertices and small components
        synth.disjoint_union(synth.ba_graph(300, 2, 8), synth.complete_graph(7), synth.path_graph(5)),
        synth.ba_graph(700, 5, 12),
    ]
    return cases


@pytest.mark.parametrize("b", [1, 5, 64, 65, 130, 1024])
@pytest.mark.parametrize("gi", range(len(small_cases())))
def test_small_graphs_labels_and_queries(gi, b):
    g = small_cases()[gi]
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    idx = build(g, order, batch_size=b)
    assert_labels_equal(idx, want, order)
    check_counters(idx, g, order, b, want)
    u, v = synth.query_pairs(g.n, 3000, seed=2)
    assert np.array_equal(gpu_query(idx, u, v), oracle.query(want, u, v))
    idx.free()


def test_ba2000_full_parity():
    """Barabasi-Albert n=2000, m=4, seed 1, degree order, b=1024, and the
    100,000 uniform query pairs of seed 2."""
    g = synth.ba_graph(2000, 4, 1)
    assert g.num_edges == 7984
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    idx = build(g, order)
    assert_labels_equal(idx, want, order)
    info = check_counters(idx, g, order, 1024, want)
    assert info["batches"] == 2
    u, v = synth.query_pairs(g.n, 100_000, seed=2)
    assert np.array_equal(gpu_query(idx, u, v), oracle.query(want, u, v))


def test_random_orders_ba():
    g = synth.ba_graph(1500, 3, 21)
    for s in (5, 6):
        order = np.argsort(synth.splitmix64(s, 0, g.n), kind="stable").astype(np.uint32)
        want = oracle.pll_labels(g, order)
        idx = build(g, order, batch_size=256)
        assert_labels_equal(idx, want, order)


def test_batch_size_invariance_ba2000():
    g = synth.ba_graph(2000, 4, 1)
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    for b in (2, 63, 100, 512, 1000):
        idx = build(g, order, batch_size=b)
        assert_labels_equal(idx, want, order)
        idx.free()


def test_recheck_removes_nothing_in_exact_rounds():
    g = synth.ba_graph(2000, 4, 1)
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    idx = build(g, order, flags=pll.FLAG_VALIDATE | pll.FLAG_RECHECK)
    assert_labels_equal(idx, want, order)
    assert idx.info()["recheck_removed"] == 0


@pytest.mark.parametrize("b", [64, 1024])
def test_relaxed_rounds_then_recheck_restore_canonical(b):
    """Rounds that ignore current-batch hubs accept extra entries; the
    batch-end recheck removes exactly those."""
    g = synth.ba_graph(2000, 4, 1)
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    idx = build(g, order, batch_size=b, flags=pll.FLAG_RECHECK | pll.FLAG_RELAXED)
    assert_labels_equal(idx, want, order)
    info = idx.info()
    assert info["recheck_removed"] > 0
    assert info["accepted"] - info["recheck_removed"] == want.total - g.n


def test_empty_and_single_vertex():
    g0 = synth.csr_from_edges(0, np.zeros(0), np.zeros(0))
    idx = build(g0, np.zeros(0, dtype=np.uint32))
    assert idx.info()["total_entries"] == 0
    out = idx.query(torch.zeros(0, dtype=torch.int32, device=DEV), torch.zeros(0, dtype=torch.int32, device=DEV))
    assert out.numel() == 0
    g1 = synth.csr_from_edges(1, np.zeros(0), np.zeros(0))
    idx1 = build(g1, np.zeros(1, dtype=np.uint32))
    assert idx1.info()["total_entries"] == 1
    assert gpu_query(idx1, np.array([0]), np.array([0]))[0] == 0


def test_unreachable_pairs_are_inf():
    g = synth.disjoint_union(synth.path_graph(10), synth.path_graph(10))
    order = synth.degree_order(g)
    idx = build(g, order, batch_size=4)
    d = gpu_query(idx, np.array([0, 0, 15]), np.array([19, 9, 12]))
    assert d[0] == pll.DIST_INF and d[1] == 9 and d[2] == 3


def test_invalid_inputs_rejected():
    g = synth.ba_graph(100, 2, 3)
    order = synth.degree_order(g)
    bad = order.copy()
    bad[5] = bad[6]
    with pytest.raises(pll.PllError) as e:
        build(g, bad)
    assert e.value.status == pll.PLL_EINVAL
    bad = order.copy()
    bad[0] = g.n + 3
    with pytest.raises(pll.PllError):
        build(g, bad)
    # column id out of range
    g2 = synth.Graph(g.n, g.row_ptr.copy(), g.col.copy())
    g2.col[10] = g.n + 7
    with pytest.raises(pll.PllError):
        build(g2, order)
    # asymmetric, unsorted, self-loop: caught by the full check
    g3 = synth.Graph(g.n, g.row_ptr.copy(), g.col.copy())
    a, b = int(g3.row_ptr[4]), int(g3.row_ptr[5])
    g3.col[a] = (g3.col[a] + 1) % g.n if g3.col[a] + 1 != 4 else (g3.col[a] + 2) % g.n
    with pytest.raises(pll.PllError):
        build(g3, order, flags=pll.FLAG_VALIDATE)
    g4 = synth.Graph(g.n, g.row_ptr.copy(), g.col.copy())
    a = int(g4.row_ptr[0])
    g4.col[a], g4.col[a + 1] = g4.col[a + 1], g4.col[a]
    with pytest.raises(pll.PllError):
        build(g4, order, flags=pll.FLAG_VALIDATE)
    g5 = synth.Graph(g.n, g.row_ptr.copy(), g.col.copy())
    g5.col[int(g5.row_ptr[7])] = 7
    with pytest.raises(pll.PllError):
        build(g5, order, flags=pll.FLAG_VALIDATE)
    # bad options
    with pytest.raises(pll.PllError):
        build(g, order, batch_size=2048)
    with pytest.raises(pll.PllError):
        build(g, order, flags=pll.FLAG_RELAXED)


def test_distance_overflow_is_edist():
    g = synth.path_graph(300)
    with pytest.raises(pll.PllError) as e:
        build(g, synth.degree_order(g), batch_size=32)
    assert e.value.status == pll.PLL_EDIST
    g = synth.path_graph(256)  # longest distance 254 still fits
    order = synth.degree_order(g)
    idx = build(g, order, batch_size=32)
    assert_labels_equal(idx, oracle.pll_labels(g, order), order)
    # one batch, ids as ranks: the round-255 candidate of vertex 0 at vertex
    # 255 meets only empty table cells (255 + 0 must not count as <= 255)
    g = synth.path_graph(257)
    with pytest.raises(pll.PllError) as e:
        build(g, np.arange(257, dtype=np.uint32))
    assert e.value.status == pll.PLL_EDIST


def test_fixed_arena_too_small_is_enospc():
    g = synth.ba_graph(2000, 4, 1)
    order = synth.degree_order(g)
    with pytest.raises(pll.PllError) as e:
        build(g, order, arena_entries=20_000)
    assert e.value.status == pll.PLL_ENOSPC
    idx = build(g, order, arena_entries=4_000_000)
    assert_labels_equal(idx, oracle.pll_labels(g, order), order)


def test_many_indexes_resident_and_batched_api():
    gs = [synth.ba_graph(n, m, 1000 + i) for i, (n, m) in enumerate([(600, 2), (900, 5), (1300, 8)])]
    orders = [synth.degree_order(g) for g in gs]
    idxs = pll.build_labels_batched([to_dev(g, o) for g, o in zip(gs, orders)])
    for g, o, idx in zip(gs, orders, idxs):
        want = oracle.pll_labels(g, o)
        assert_labels_equal(idx, want, o)
        u, v = synth.query_pairs(g.n, 2000, seed=2)
        assert np.array_equal(gpu_query(idx, u, v), oracle.query(want, u, v))


def test_query_on_side_stream():
    g = synth.ba_graph(2000, 4, 1)
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    idx = build(g, order)
    u, v = synth.query_pairs(g.n, 50_000, seed=5)
    du = torch.from_numpy(u.view(np.int32)).to(DEV)
    dv = torch.from_numpy(v.view(np.int32)).to(DEV)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        out = idx.query(du, dv, stream=s)
    s.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint32), oracle.query(want, u, v))


@pytest.mark.parametrize("b", [5, 130])
@pytest.mark.parametrize("gi", range(len(small_cases())))
def test_persistent_rounds_match(gi, b):
    """The persistent batch loop (PLL_FLAG_PERSISTENT: one launch, grid
    barriers between phases) gives the oracle's labels and the same counters
    as the per-phase launches."""
    g = small_cases()[gi]
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    idx = build(g, order, batch_size=b, flags=pll.FLAG_VALIDATE | pll.FLAG_PERSISTENT)
    assert_labels_equal(idx, want, order)
    check_counters(idx, g, order, b, want)
    idx.free()


@pytest.mark.parametrize("cap", [1, 2, 7])
def test_persistent_loop_with_few_workgroups(cap):
    """The grid barrier with fewer workgroups than barrier shards, and a
    single workgroup doing every phase."""
    g = synth.ba_graph(2000, 4, 1)
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    idx = build(g, order, batch_size=300, max_workgroups=cap, flags=pll.FLAG_VALIDATE | pll.FLAG_PERSISTENT)
    assert idx.info()["gang"] == cap
    assert_labels_equal(idx, want, order)
    check_counters(idx, g, order, 300, want)


def test_persistent_flag_is_accepted_and_unknown_flags_are_not():
    g = synth.ba_graph(100, 2, 1)
    order = synth.degree_order(g)
    build(g, order, flags=pll.FLAG_PERSISTENT).free()
    with pytest.raises(pll.PllError) as e:
        build(g, order, flags=0x400)
    assert e.value.status == pll.PLL_EINVAL


@pytest.mark.parametrize("n,m,seed", [(4797, 3, 1001), (6575, 8, 1005), (7051, 8, 1007), (12000, 6, 77)])
def test_many_batches_large_rounds(n, m, seed):
    """Graphs of several batches whose rounds have thousands of receivers:
    the check of a round and the push of the next share a launch, so the two
    rounds' receiver lists and messages must not share storage."""
    g = synth.ba_graph(n, m, seed)
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    idx = build(g, order)
    assert_labels_equal(idx, want, order)
    check_counters(idx, g, order, 1024, want)
    u, v = synth.query_pairs(g.n, 20000, seed=3)
    assert np.array_equal(gpu_query(idx, u, v), oracle.query(want, u, v))


def test_size_limits_rejected_before_any_work():
    """n at the 24-bit hub-rank limit and nnz beyond 2^33 are PLL_EINVAL
    (checked on the host before anything is read)."""
    import ctypes
    g = synth.ba_graph(50, 2, 1)
    rp, cl, od = to_dev(g, synth.degree_order(g))
    lib = pll.load_library()
    o = pll._opts(1024, 0, 0, 0)
    h = ctypes.c_void_p()
    for n, nnz in (((1 << 24), g.nnz), (g.n, 0xFFFFFFFF * 2 + 1)):
        rc = lib.pll_build_labels(n, nnz, rp.data_ptr(), cl.data_ptr(), od.data_ptr(), ctypes.byref(o), None,
                                  ctypes.byref(h))
        assert rc == pll.PLL_EINVAL and not h.value
    for bad in (dict(batch_size=1025), dict(query_lanes=3)):
        with pytest.raises(pll.PllError) as e:
            build(g, synth.degree_order(g), **bad)
        assert e.value.status == pll.PLL_EINVAL


@pytest.mark.parametrize("b", [64, 1024])
def test_pulled_rounds_match_oracle(b):
    """Graphs of 16,384 vertices or more gather the rounds that follow a round
    with at least n/2 receivers instead of pushing them: labels and every
    counter of Algorithm 4 (edge accesses included) stay as with pushes."""
    g = synth.ba_graph(20000, 4, 3)
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    idx = build(g, order, batch_size=b, flags=pll.FLAG_PROFILE)
    assert_labels_equal(idx, want, order)
    info = check_counters(idx, g, order, b, want)
    assert int(g.degrees().max()) <= 1024  # no heavy-row pushes: every extra push launch is a pull
    assert info["phase_launches"]["push"] > info["batches"]
    u, v = synth.query_pairs(g.n, 100_000, seed=4)
    assert np.array_equal(gpu_query(idx, u, v), oracle.query(want, u, v))


@pytest.mark.parametrize("b", [64, 300, 1024])
@pytest.mark.parametrize("isolated", [0, 1, 700, 5000])
def test_trailing_isolated_vertices(b, isolated):
    """Isolated vertices ranked last: the batches that hold only them are not
    run, and finalize writes their self entries.  Labels, counters (one batch
    of one round per such batch, as the oracle counts them) and queries equal
    the oracle's, also when the boundary falls inside a batch."""
    g0 = synth.ba_graph(1200, 3, 31)
    g = synth.disjoint_union(g0, synth.csr_from_edges(isolated, np.zeros(0), np.zeros(0))) if isolated else g0
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    idx = build(g, order, batch_size=b)
    assert_labels_equal(idx, want, order)
    check_counters(idx, g, order, b, want)
    u, v = synth.query_pairs(g.n, 20_000, seed=3)
    assert np.array_equal(gpu_query(idx, u, v), oracle.query(want, u, v))
    idx.free()


@pytest.mark.parametrize("b", [1, 64, 1024])
def test_edgeless_graph_of_several_batches(b):
    """No edges at all: only the first batch runs; every label is its self
    entry and every pair but (v, v) is unreachable."""
    n = 3000
    g = synth.csr_from_edges(n, np.zeros(0), np.zeros(0))
    order = synth.degree_order(g)
    want = oracle.pll_labels(g, order)
    assert want.total == n
    idx = build(g, order, batch_size=b)
    assert_labels_equal(idx, want, order)
    check_counters(idx, g, order, b, want)
    u, v = synth.query_pairs(n, 5000, seed=4)
    got = gpu_query(idx, u, v)
    assert np.array_equal(got, np.where(u == v, 0, pll.DIST_INF).astype(got.dtype))
    idx.free()
