"""Full-size GPU checks on the R-MAT scale-20 graph (1,048,576 vertices,
edge factor 16), b = 1024, in the launch configuration the bench times.

* The whole exported labeling hashes to the oracle's stored digests
  (tests/golden/rmat20_oracle.json, the sequential PLL of Algorithm 1 run
  offline; Definition 2 and Theorem 1 make the labels unique), block by
  block on a mismatch.
* All 10^7 configured pairs (seed 2) answer as the oracle's merge over its
  own labels (Section 2.1).
* Independently of the stored digests: sampled vertices against Definition 2
  (one BFS each) and sampled sources against BFS distances."""
import numpy as np
import pytest
import torch

import oracle
import paper_1906_12018_amd as pll
import synth
from gpu_util import (DEV, assert_answers_match_digests, assert_labels_equal, assert_labels_match_digests, build,
                      exported, golden, gpu_query)


def overlapping(a, b):
    """Device intervals (t_dev_start, t_dev_end) that share some time."""
    return a[0] < b[1] and b[0] < a[1]

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rmat20():
    g = synth.rmat_graph(20)
    order = synth.degree_order(g)
    idx = build(g, order, batch_size=1024, flags=0)
    yield g, order, idx
    idx.free()


def test_rmat20_labels_equal_oracle_digests(rmat20):
    g, order, idx = rmat20
    want = golden("rmat20")
    info = idx.info()
    assert info["batches"] == 1024
    assert info["accepted"] + g.n == info["total_entries"]
    assert info["candidates"] + g.n == want["counters"]["checks"]  # Corollary 2
    assert info["max_dist"] == want["max_dist"]
    assert_labels_match_digests(idx, want, "R-MAT-20")


def test_rmat20_configured_pairs_equal_oracle(rmat20):
    g, order, idx = rmat20
    want = golden("rmat20")["pairs"]
    u, v = synth.query_pairs(g.n, 10_000_000, seed=2)
    assert_answers_match_digests(gpu_query(idx, u, v), want, "R-MAT-20 10^7 pairs")
    # the reversed pairs give the same distances (the graph is undirected)
    du = torch.from_numpy(v.view(np.int32)).to(DEV)
    dv = torch.from_numpy(u.view(np.int32)).to(DEV)
    back = idx.query(du, dv)
    torch.cuda.synchronize()
    assert_answers_match_digests(back.cpu().numpy().view(np.uint32), want, "R-MAT-20 reversed pairs")


def test_rmat20_sampled_labels_match_definition2(rmat20):
    g, order, idx = rmat20
    off, hubs, dists = exported(idx)
    verts = np.unique(synth.bounded(synth.splitmix64(77, 0, 60), g.n))
    iso = np.flatnonzero(g.degrees() == 0)[:3]
    verts = np.concatenate([verts, order[:8], order[-8:], iso]).astype(np.uint32)
    want = oracle.canonical_labels(g, order, verts=verts, threads=16)
    for i, v in enumerate(verts):
        h, d = want.of(i)
        a, b = int(off[v]), int(off[v + 1])
        assert np.array_equal(order[h], hubs[a:b]), int(v)
        assert np.array_equal(d, dists[a:b]), int(v)


def test_rmat20_queries_exact_from_sampled_sources(rmat20):
    g, order, idx = rmat20
    for s in synth.bounded(synth.splitmix64(91, 0, 3), g.n):
        want = oracle.bfs(g, int(s))
        got = gpu_query(idx, np.full(g.n, s, dtype=np.uint32), np.arange(g.n, dtype=np.uint32))
        assert np.array_equal(got, want)


def test_rmat20_serving_alone_equals_mix(rmat20):
    """The serving configuration: the R-MAT-20 index resident, the 10^7
    configured pairs arriving as requests of log-uniform sizes in [1, 65536]
    (a burst, then one every 100 us), and Barabasi-Albert labeling jobs
    (n in [1000, 50000]) among them.  Every request equals the same pairs
    asked alone (one pll_query), all answers together equal the oracle's
    stored digest, some query batches ran on the device beside other query
    batches and beside a labeling launch, and the built indexes equal the
    oracle's labels."""
    g, order, idx = rmat20
    want = golden("rmat20")["pairs"]
    u, v = synth.query_pairs(g.n, 10_000_000, seed=2)
    alone = gpu_query(idx, u, v)
    x = synth.uniform01(synth.splitmix64(12, 0, 4000))
    sizes = np.maximum(1, np.round(np.exp(x * np.log(65536)))).astype(np.int64)
    cuts = np.concatenate([[0], np.cumsum(sizes)])
    cuts = cuts[cuts < len(u)]
    cuts = np.append(cuts, len(u))
    jobs = []
    jx = synth.splitmix64(13, 0, 12)
    for i in range(6):
        n = int(round(np.exp(np.log(1000) + synth.uniform01(jx[2 * i:2 * i + 1])[0] * np.log(50))))
        m = 2 + int(synth.bounded(jx[2 * i + 1:2 * i + 2], 7)[0])
        bg = synth.ba_graph(n, m, 6000 + i)
        jobs.append((bg, synth.degree_order(bg)))
    srv = pll.Server(slots=4)
    iid = srv.add_index(idx)
    out = np.zeros(len(u), dtype=np.uint32)
    reqs, job_at = [], {}
    nreq = len(cuts) - 1
    for k in range(nreq):
        a, b = int(cuts[k]), int(cuts[k + 1])
        at = 1e-4 * max(k - 64, 0)
        reqs.append(pll.Server.query_request(iid, u[a:b], v[a:b], out[a:b], at=at))
        if k % (nreq // 6) == 5 and len(job_at) < len(jobs):
            j = len(job_at)
            job_at[j] = len(reqs)
            reqs.append(pll.Server.build_request(jobs[j][0].row_ptr, jobs[j][0].col, jobs[j][1], at=at))
    res = srv.replay(reqs)
    assert all(r["status"] == pll.PLL_OK for r in res)
    assert np.array_equal(out, alone)
    assert_answers_match_digests(out, want, "R-MAT-20 pairs served in the mix")
    q = [(r["t_dev_start"], r["t_dev_end"]) for r in res if r["kind"] == pll.REQ_QUERY]
    bl = [(r["t_dev_start"], r["t_dev_end"]) for r in res if r["kind"] == pll.REQ_BUILD]
    assert all(0 <= a <= b for a, b in q + bl)
    batches = sorted(set(q))
    assert any(overlapping(batches[i], batches[j]) for i in range(len(batches))
               for j in range(i + 1, min(len(batches), i + 8))), "no two query batches overlapped"
    assert any(overlapping(a, b) for a in batches for b in bl), "no query batch ran beside a labeling launch"
    for j, (bg, bo) in enumerate(jobs):
        r = res[job_at[j]]
        assert r["kind"] == pll.REQ_BUILD
        assert_labels_equal(srv.index(r["index_id"]), oracle.pll_labels(bg, bo), bo)
    srv.close()
