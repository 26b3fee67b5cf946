"""Host-side parts of the autotuner (no GPU): workload keys and the cache."""
import torch

from paper_1906_12018_amd import autotune


def fake(n, nnz):
    return (torch.zeros(n + 1, dtype=torch.int64), torch.zeros(nnz, dtype=torch.int32), torch.zeros(n, dtype=torch.int32))


def test_workload_key_buckets():
    a = autotune.workload_key([fake(1000, 8000), fake(3000, 24000)])
    b = autotune.workload_key([fake(1100, 8800), fake(2900, 23200)])
    c = autotune.workload_key([fake(100000, 800000)])
    assert a == b and a != c


def test_cache_roundtrip(tmp_path, monkeypatch):
    monkeypatch.setenv("PLL_TUNE_CACHE", str(tmp_path / "t.json"))
    gs = [fake(500, 2000)]
    assert autotune.cached_config(gs) is None
    cache = {autotune.workload_key(gs): {"best": {"batch_size": 512, "gang_scale": 100, "max_gang": 8}}}
    autotune._save_cache(cache)
    assert autotune.cached_config(gs) == {"batch_size": 512, "gang_scale": 100, "max_gang": 8}


class _FakeIndex:
    def __init__(self, n, entries, bp=0):
        self._i = {"n": n, "in_entries": entries, "out_entries": entries, "bp_roots": bp}

    def info(self):
        return self._i


def test_index_key_buckets():
    a = autotune.index_key(_FakeIndex(65536, 5_000_000))
    b = autotune.index_key(_FakeIndex(60000, 4_700_000))
    c = autotune.index_key(_FakeIndex(1 << 20, 252_000_000))
    d = autotune.index_key(_FakeIndex(65536, 5_000_000, bp=16))
    assert a == b and a != c and a != d


class _FakeExport:
    def __init__(self, off, hubs, dists):
        self.offsets, self.hubs, self.dists = off, hubs, dists


class _FakeBuilt:
    def __init__(self, ex):
        self._ex = ex

    def export(self):
        return self._ex

    def info(self):
        return {"total_entries": int(self._ex.hubs.numel())}

    def free(self):
        pass


def test_tuner_rejects_same_size_but_different_labels(monkeypatch, tmp_path):
    """A candidate whose labels keep every list length but change one
    distance is rejected; identical labels pass."""
    import pytest
    monkeypatch.setenv("PLL_TUNE_CACHE", str(tmp_path / "t.json"))
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    good = _FakeExport(torch.tensor([0, 2, 3]), torch.tensor([0, 1, 1], dtype=torch.int32),
                       torch.tensor([0, 1, 0], dtype=torch.uint8))
    bad = _FakeExport(good.offsets.clone(), good.hubs.clone(), torch.tensor([0, 2, 0], dtype=torch.uint8))

    def fake_build(graphs, flags=0, batch_size=0, **kw):
        return [_FakeBuilt(bad if batch_size == 999 else good)]

    monkeypatch.setattr(autotune, "build_labels_batched", fake_build)
    gs = [fake(2, 2)]
    ok = autotune.tune_batched(gs, candidates=[dict(batch_size=256), dict(batch_size=512)], reps=1, save=False)
    assert ok["best"] in (dict(batch_size=256), dict(batch_size=512))
    with pytest.raises(RuntimeError, match="different labels"):
        autotune.tune_batched(gs, candidates=[dict(batch_size=256), dict(batch_size=999)], reps=1, save=False)
