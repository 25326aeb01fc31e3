"""Host side of the guide-size autotuner: cache keys, cache file round trip
and the environment override (no GPU needed)."""
import json

from paper_1901_05423_amd import tune


def test_bucket_keys_group_sizes():
    k1 = tune.bucket_key("gfx950", "single", 1 << 24, 1 << 26)
    k2 = tune.bucket_key("gfx950", "single", int(1.1 * (1 << 24)), int(1.1 * (1 << 26)))
    k3 = tune.bucket_key("gfx950", "single", 1 << 20, 1 << 26)
    assert k1 == k2 and k1 != k3
    assert "n2^24" in k1 and "s/n2^2" in k1


def test_cache_round_trip(tmp_path, monkeypatch):
    path = str(tmp_path / "sub" / "tune.json")
    monkeypatch.setenv("RTF_TUNE_CACHE", path)
    assert tune.load_cache() == {}
    tune.store_cache({"a|b": {"ratio": 0.5}})
    assert json.load(open(path)) == {"a|b": {"ratio": 0.5}}
    assert tune.load_cache()["a|b"]["ratio"] == 0.5
    open(path, "w").write("not json")
    assert tune.load_cache() == {}


def test_forced_ratio(monkeypatch):
    monkeypatch.delenv("RTF_CELL_RATIO", raising=False)
    assert tune.forced_ratio() is None
    monkeypatch.setenv("RTF_CELL_RATIO", "0.25")
    assert tune.forced_ratio() == 0.25
    # a forced ratio wins without touching the GPU
    assert tune.best_cell_ratio(None, None) == 0.25
