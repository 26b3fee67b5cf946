"""The allocation-free build (pll_build_labels_noalloc) against the
allocating one (pll_build_labels, then pll_export_labels) on the same
graphs: two calls in a row, the second with a smaller graph, so the fixed
scratch holds the first call's contents when the second starts.  Labels are
integers: they must be equal byte for byte, and equal to the oracle's."""
import numpy as np
import pytest
import torch

import oracle
import paper_1906_12018_amd as pll
import synth
from gpu_util import DEV, build, exported, to_dev

pytestmark = pytest.mark.gpu


def outputs(n, cap):
    return (torch.empty(n + 1, dtype=torch.int64, device=DEV), torch.empty(max(cap, 1), dtype=torch.int32, device=DEV),
            torch.empty(max(cap, 1), dtype=torch.uint8, device=DEV))


def as_numpy(off, hubs, dists, total):
    return (off.cpu().numpy().view(np.uint64), hubs[:total].cpu().numpy().view(np.uint32),
            dists[:total].cpu().numpy())


def test_noalloc_equals_allocating_build_on_two_calls():
    cases = [(synth.ba_graph(12000, 6, 21), 1024), (synth.ba_graph(3000, 3, 22), 256)]
    prepared = []
    for g, b in cases:
        order = synth.degree_order(g)
        idx = build(g, order, batch_size=b)
        want = exported(idx)
        idx.free()
        dev_in = to_dev(g, order)
        prepared.append((g, order, b, dev_in, want, outputs(g.n, len(want[1]) + 64)))
    torch.cuda.synchronize()
    free_before = torch.cuda.mem_get_info()[0]
    totals = []
    for g, order, b, (rp, cl, od), want, (off, hubs, dists) in prepared:
        totals.append(pll.build_labels_noalloc(rp, cl, od, off, hubs, dists, batch_size=b))
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free_before  # no device memory taken
    for (g, order, b, _, want, (off, hubs, dists)), total in zip(prepared, totals):
        got = as_numpy(off, hubs, dists, total)
        assert total == len(want[1])
        for a, w in zip(got, want):
            assert np.array_equal(a, w), g.name
        lab = oracle.pll_labels(g, order)
        assert np.array_equal(got[0], lab.offsets) and np.array_equal(got[1], lab.hubs_as_ids(order))
        assert np.array_equal(got[2], lab.dist)


def test_noalloc_capacity_and_size_limits():
    g = synth.ba_graph(2000, 4, 1)
    order = synth.degree_order(g)
    rp, cl, od = to_dev(g, order)
    off, hubs, dists = outputs(g.n, 100)
    with pytest.raises(pll.PllError) as e:
        pll.build_labels_noalloc(rp, cl, od, off, hubs, dists)
    assert e.value.status == pll.PLL_ENOSPC and e.value.total == oracle.pll_labels(g, order).total
    off, hubs, dists = outputs(g.n, e.value.total)
    assert pll.build_labels_noalloc(rp, cl, od, off, hubs, dists) == e.value.total
    big = synth.rmat_graph(16)
    rp, cl, od = to_dev(big, synth.degree_order(big))
    off, hubs, dists = outputs(big.n, 16)
    with pytest.raises(pll.PllError) as e:
        pll.build_labels_noalloc(rp, cl, od, off, hubs, dists, batch_size=1024)
    assert e.value.status == pll.PLL_ESCRATCH
