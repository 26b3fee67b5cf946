"""Autotuners: the many-graph build (one persistent launch) and the query's
label windows.

Tunes, per workload class, the launch parameters that do not change the
labels: the batch size b (which sets the width of the per-batch distance-table
tiles, 64*ceil(b/64) bytes per row, and of the candidate bit-vectors), the
gang scale (how many workgroups each graph gets relative to its share of the
estimated work, i.e. the work per wavefront) and the largest gang.  Every
candidate is timed on the caller's graphs through the C ABI; a candidate
whose exported labels differ in any entry from the first candidate's is
rejected (labels are invariant under all of these, so a difference would be
a bug).  Results are cached in a
JSON file keyed by a coarse signature of the workload.

For queries it tunes the lanes per pair G of an index (the merge reads
windows of 2G entries of one label and 4G of the other): every G is timed on
a sample of the caller's pairs, a G whose answers differ is rejected, and
the best is set on the index and cached per index class (vertex count and
mean label length, bucketed).
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

from . import DEFAULT_BATCH, FLAG_VALIDATE, build_labels_batched

QUERY_LANES = (1, 4, 8, 16, 32, 64)

DEFAULT_CANDIDATES = [
    dict(batch_size=b, gang_scale=s, max_gang=16)
    for b in (256, 512, 1024)
    for s in (200, 400, 800, 1600, 3200)
]


def cache_path() -> str:
    return os.environ.get("PLL_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "pll_mi355x",
                                                         "tune.json"))


def workload_key(graphs) -> str:
    """Coarse class of a list of (row_ptr, col, order) device tensors: graph
    count, mean and largest vertex count and mean degree, each bucketed to a
    power of two."""
    ns = [int(g[2].numel()) for g in graphs]
    nnz = [int(g[1].numel()) for g in graphs]
    def b2(x):
        return int(round(math.log2(max(x, 1))))
    deg = sum(nnz) / max(sum(ns), 1)
    return f"count{b2(len(ns))}_mean{b2(sum(ns) / max(len(ns), 1))}_max{b2(max(ns) if ns else 1)}_deg{b2(deg)}"


def _load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(cache: dict) -> None:
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass


def cached_config(graphs):
    """The tuned launch parameters for this workload class, or None."""
    ent = _load_cache().get(workload_key(graphs))
    return dict(ent["best"]) if ent else None


def _exports(idxs):
    """Every index's exported labels (offsets, hubs, dists), kept on the device."""
    out = []
    for i in idxs:
        ex = i.export()
        out.append((ex.offsets, ex.hubs, ex.dists))
    return out


def _same_labels(a, b) -> bool:
    return len(a) == len(b) and all(torch.equal(x, y) for p, q in zip(a, b) for x, y in zip(p, q))


def tune_batched(graphs, candidates=None, reps: int = 2, flags: int = 0, save: bool = True, verbose: bool = False):
    """Time every candidate on `graphs` (median of `reps` builds after one
    warm-up build) and return {"best": params, "results": [...]}.  The labels
    of every candidate's warm-up build must equal the first candidate's entry
    for entry (they do not depend on any tuned parameter); a candidate that
    changes them raises."""
    candidates = candidates or DEFAULT_CANDIDATES
    results, ref = [], None
    for cand in candidates:
        times = []
        for rep in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            idxs = build_labels_batched(graphs, flags=flags, **cand)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if rep == 0:
                labels = _exports(idxs)
                if ref is None:
                    ref = labels
                elif not _same_labels(labels, ref):
                    for i in idxs:
                        i.free()
                    raise RuntimeError(f"candidate {cand} produced different labels")
                del labels
            for i in idxs:
                i.free()
            if rep > 0:
                times.append(dt)
        times.sort()
        med = times[len(times) // 2]
        results.append(dict(params=cand, seconds=med))
        if verbose:
            print(f"tune {cand}: {med * 1e3:.1f} ms", flush=True)
    best = min(results, key=lambda r: r["seconds"])
    out = {"best": best["params"], "seconds": best["seconds"], "results": results}
    if save:
        cache = _load_cache()
        cache[workload_key(graphs)] = out
        _save_cache(cache)
    return out


def build_tuned(graphs, flags: int = FLAG_VALIDATE, tune_if_missing: bool = False, **kw):
    """build_labels_batched with the cached parameters of this workload class
    (tuning first when asked and nothing is cached)."""
    cfg = cached_config(graphs)
    if cfg is None and tune_if_missing:
        cfg = tune_batched(graphs)["best"]
    if cfg is None:
        cfg = dict(batch_size=DEFAULT_BATCH)
    cfg.update(kw)
    return build_labels_batched(graphs, flags=flags, **cfg)


def index_key(index) -> str:
    """Class of an index for the query tuner: vertex count and mean label
    length (both sides of a directed index), bucketed to powers of two."""
    inf = index.info()
    n = max(inf["n"], 1)
    mean = (inf["in_entries"] + inf["out_entries"]) / (2 * n)
    def b2(x):
        return int(round(math.log2(max(x, 1))))
    return f"query_n{b2(n)}_mean{b2(mean)}_bp{inf['bp_roots']}"


def tune_query(index, u, v, candidates=QUERY_LANES, reps: int = 3, save: bool = True, verbose: bool = False):
    """Time pll_query on the pairs (u, v) (device int32 tensors) for each lanes
    value (median of `reps` after one warm-up), check that every value gives
    the same answers, set the fastest on the index and return
    {"best": lanes, "results": [...]}."""
    out = torch.empty_like(u)
    ref = None
    results = []
    for g in candidates:
        index.set_query_lanes(g)
        times = []
        for rep in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            index.query(u, v, out=out)
            e1.record()
            torch.cuda.synchronize()
            if rep > 0:
                times.append(e0.elapsed_time(e1))
        if ref is None:
            ref = out.clone()
        elif not torch.equal(out, ref):
            raise RuntimeError(f"query lanes {g} gave different answers")
        times.sort()
        results.append(dict(lanes=g, ms=times[len(times) // 2]))
        if verbose:
            print(f"tune query lanes {g}: {results[-1]['ms']:.3f} ms", flush=True)
    best = min(results, key=lambda r: r["ms"])
    index.set_query_lanes(best["lanes"])
    res = {"best": best["lanes"], "results": results}
    if save:
        cache = _load_cache()
        cache[index_key(index)] = res
        _save_cache(cache)
    return res


def apply_cached_query_lanes(index) -> bool:
    """Set the cached best lanes of this index class, if any."""
    ent = _load_cache().get(index_key(index))
    if not ent:
        return False
    index.set_query_lanes(int(ent["best"]))
    return True
