"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare it with the oracle on the same seeded inputs."""
import os
import sys

import numpy as np
import torch

import oracle
import paper_1906_12018_amd as pll
import synth

DEV = torch.device("cuda:0")


def to_dev(g, order):
    rp, cl = pll.graph_to_device(g, DEV)
    od = torch.from_numpy(np.ascontiguousarray(order, dtype=np.uint32).view(np.int32)).to(DEV)
    return rp, cl, od


def build(g, order, **kw):
    rp, cl, od = to_dev(g, order)
    return pll.build_labels(rp, cl, od, **kw)


def exported(idx):
    ex = idx.export()
    torch.cuda.synchronize()
    return (ex.offsets.cpu().numpy().view(np.uint64), ex.hubs.cpu().numpy().view(np.uint32), ex.dists.cpu().numpy())


def assert_labels_equal(idx, want: oracle.Labels, order):
    off, hubs, dists = exported(idx)
    assert np.array_equal(off, want.offsets), "offsets differ"
    assert np.array_equal(hubs, want.hubs_as_ids(order)), "hubs differ"
    assert np.array_equal(dists, want.dist), "dists differ"


def gpu_query(idx, u, v):
    du = torch.from_numpy(np.ascontiguousarray(u, dtype=np.uint32).view(np.int32)).to(DEV)
    dv = torch.from_numpy(np.ascontiguousarray(v, dtype=np.uint32).view(np.int32)).to(DEV)
    out = idx.query(du, dv)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


def check_counters(idx, g, order, b, want_pll: oracle.Labels):
    """Corollary 2: candidates + n = PLL distance checks; accepted = entries
    minus the n self entries; rounds, edge reads and checks equal the
    sequential Algorithm 4 run with the same batch size."""
    info = idx.info()
    bvc = oracle.bvc_labels(g, order, b)
    assert info["total_entries"] == want_pll.total
    assert info["candidates"] + g.n == want_pll.counters["checks"]
    assert info["candidates"] == bvc.counters["checks"]
    assert info["accepted"] == want_pll.total - g.n
    assert info["rounds"] == bvc.counters["rounds"]
    assert info["batches"] == bvc.counters["batches"]
    assert info["edges_scanned"] == bvc.counters["edge_accesses"]
    # cost of the positive and negative checks (sum of |L(v)| at each check)
    assert info["check_cost_pos"] == bvc.counters["cost_pos"]
    assert info["check_cost_neg"] == bvc.counters["cost_neg"]
    assert info["max_dist"] == (int(want_pll.dist.max()) if want_pll.total else 0)
    return info


GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
if GOLDEN_DIR not in sys.path:
    sys.path.insert(0, GOLDEN_DIR)
from make_goldens import label_digests  # noqa: E402  (hashing only: no labeling arithmetic)


def golden(name: str) -> dict:
    """Stored oracle digests (tests/golden/<name>_oracle.json, written by
    tests/golden/make_goldens.py from the oracle alone)."""
    import json
    path = os.path.join(GOLDEN_DIR, f"{name}_oracle.json")
    with open(path) as f:
        return json.load(f)


def assert_labels_match_digests(idx, want: dict, what: str = ""):
    """The exported labels hash to the oracle's stored digests; on a
    mismatch, name the first vertex block that differs."""
    off, hubs, dists = exported(idx)
    got = label_digests(off, hubs, dists, want.get("block", 1 << 16))
    assert got["n"] == want["n"], f"{what}: n {got['n']} != {want['n']}"
    assert got["total"] == want["total"], f"{what}: {got['total']} entries, the oracle has {want['total']}"
    if any(got[k] != want[k] for k in ("sha_offsets", "sha_hubs", "sha_dists")):
        bad = [i for i, (a, b) in enumerate(zip(got["blocks"], want["blocks"])) if a != b]
        raise AssertionError(f"{what}: labels differ from the oracle's; first differing vertex block {bad[:1]} "
                             f"({len(bad)} blocks of {want.get('block', 1 << 16)} vertices differ)")


def assert_answers_match_digests(ans, want: dict, what: str = ""):
    """uint32 answers hash to the oracle's stored digest; on a mismatch,
    name the first differing chunk of pairs."""
    import hashlib
    ans = np.ascontiguousarray(ans, dtype=np.uint32)
    assert ans.shape[0] == want["count"]
    if hashlib.sha256(ans.tobytes()).hexdigest() != want["sha"]:
        c = want["chunk"]
        bad = [i for i in range(len(want["chunks"]))
               if hashlib.sha256(ans[i * c:(i + 1) * c].tobytes()).hexdigest() != want["chunks"][i]]
        raise AssertionError(f"{what}: answers differ from the oracle's; first differing chunk of {c} pairs: "
                             f"{bad[:1]} ({len(bad)} chunks differ)")
