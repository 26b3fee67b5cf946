"""Write the stored expected values of the full-size parity tests.

Every value here comes from the oracle (``oracle/``) run on the seeded inputs
of ``synth/``; nothing is read from the HIP path.  The labels are the
canonical labeling of Definition 2 (Section 2.1), which PLL (Algorithm 1)
computes and which BVC-PLL reaches for every batch size (Theorem 1 and the
batch argument of Section 4.2), so the GPU export must hash to the same
digests.  The query answers are the 2-hop formula of Section 2.1 evaluated
by the oracle's merge over its own labels.

Digest layout (both sides compute it the same way from the exported CSR):

* labels are exported by vertex id: ``offsets`` uint64[n+1], ``hubs``
  uint32 (vertex ids, ascending hub rank within a list), ``dists`` uint8;
* ``sha_offsets``/``sha_hubs``/``sha_dists`` hash the three arrays whole;
* block k covers vertices [k*B, (k+1)*B): its digest hashes the block's list
  lengths (uint32), then its hubs, then its dists;
* query answers are uint32 (0xFFFFFFFF for no common hub); chunk c covers
  pairs [c*C, (c+1)*C).

Usage: ``python tests/golden/make_goldens.py [rmat20] [batch256]`` (both by
default).  The R-MAT scale-20 oracle build takes tens of minutes on one core.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

RMAT20_FILE = os.path.join(HERE, "rmat20_oracle.json")
BATCH256_FILE = os.path.join(HERE, "batch256_oracle.json")
LABEL_BLOCK = 1 << 16
PAIR_CHUNK = 1_000_000


def sha(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def label_digests(offsets, hubs, dists, block=LABEL_BLOCK) -> dict:
    """Whole-array and per-block SHA-256 of an exported labeling."""
    offsets = np.asarray(offsets, dtype=np.uint64)
    n = offsets.shape[0] - 1
    lens = np.diff(offsets).astype(np.uint32)
    blocks = []
    for lo in range(0, n, block):
        hi = min(n, lo + block)
        a, b = int(offsets[lo]), int(offsets[hi])
        blocks.append(sha(lens[lo:hi], hubs[a:b], dists[a:b]))
    return {
        "n": int(n),
        "total": int(offsets[-1]),
        "sha_offsets": sha(offsets),
        "sha_hubs": sha(np.asarray(hubs, dtype=np.uint32)),
        "sha_dists": sha(np.asarray(dists, dtype=np.uint8)),
        "block": int(block),
        "blocks": blocks,
    }


def answer_digests(ans, chunk=PAIR_CHUNK) -> dict:
    ans = np.asarray(ans, dtype=np.uint32)
    vals, counts = np.unique(ans, return_counts=True)
    return {
        "count": int(ans.shape[0]),
        "sha": sha(ans),
        "chunk": int(chunk),
        "chunks": [sha(ans[i:i + chunk]) for i in range(0, ans.shape[0], chunk)],
        "histogram": {str(int(v)): int(c) for v, c in zip(vals, counts)},
    }


def one_graph(g, order, pairs: int, pair_seed: int = 2) -> dict:
    t0 = time.perf_counter()
    lab = oracle.pll_labels(g, order)
    secs = time.perf_counter() - t0
    hubs = lab.hubs_as_ids(order)
    rec = label_digests(lab.offsets, hubs, lab.dist)
    rec["oracle_build_s"] = round(secs, 3)
    rec["counters"] = dict(lab.counters)
    rec["max_dist"] = int(lab.dist.max()) if lab.total else 0
    if pairs:
        u, v = synth.query_pairs(g.n, pairs, seed=pair_seed)
        ans, cons = oracle.query(lab, u, v, with_consumed=True)
        rec["pairs"] = answer_digests(ans)
        rec["pairs"]["seed"] = pair_seed
        rec["pairs"]["consumed_entries"] = int(cons.sum())
    return rec


def make_rmat20():
    g = synth.rmat_graph(20)
    order = synth.degree_order(g)
    rec = {"workload": "R-MAT scale 20, edge factor 16, (a,b,c)=(0.57,0.19,0.19), seed 1; degree-descending "
                       "order, ties by id; 10^7 query pairs of seed 2",
           "nnz": int(g.nnz)}
    rec.update(one_graph(g, order, 10_000_000))
    with open(RMAT20_FILE, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(f"rmat20: {rec['total']} entries, oracle build {rec['oracle_build_s']} s", flush=True)


def make_batch256():
    graphs = []
    for i, (n, m, sd) in enumerate(synth.batching_specs()):
        g = synth.ba_graph(n, m, sd)
        rec = {"index": i, "m": m, "seed": sd}
        rec.update(one_graph(g, synth.degree_order(g), 2000))
        del rec["block"]
        graphs.append(rec)
    out = {"workload": "256 Barabasi-Albert graphs, n log-uniform in [500, 20000], m in {2..8}, graph g of seed "
                       "1000+g, each with its own degree-descending order; 2,000 query pairs of seed 2 per graph",
           "block": LABEL_BLOCK, "graphs": graphs}
    with open(BATCH256_FILE, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"batch256: {sum(r['total'] for r in graphs)} entries", flush=True)


if __name__ == "__main__":
    what = sys.argv[1:] or ["batch256", "rmat20"]
    if "batch256" in what:
        make_batch256()
    if "rmat20" in what:
        make_rmat20()
