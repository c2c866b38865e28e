"""Host-side behaviour of the launch-shape autotuner: the cache file round
trip, lookup by problem shape, and the environment the engine reads at
problem creation (restored afterwards).  No GPU."""
import json
import os

from paper_1306_1970_amd import autotune


def test_cache_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("FLR_TUNE_CACHE", str(path))
    monkeypatch.setattr(autotune, "SHIPPED", str(tmp_path / "none.json"))
    assert autotune.load() == {}
    assert autotune.lookup(1000, 10000, 1) is None
    entry = {"target_wg_a": 768, "target_wg_b": 384, "a_us": 8.1, "b_us": 9.2}
    autotune.store(1000, 10000, 1, entry)
    autotune.store(5000, 50000, 2, {"target_wg_a": 1024, "target_wg_b": 512})
    assert autotune.lookup(1000, 10000, 1) == entry
    assert autotune.lookup(5000, 50000, 2)["target_wg_b"] == 512
    assert autotune.lookup(1000, 10000, 2) is None  # dtype is part of the key
    with open(path) as fh:
        assert len(json.load(fh)) == 2


def test_corrupt_cache_is_ignored(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    monkeypatch.setenv("FLR_TUNE_CACHE", str(path))
    monkeypatch.setattr(autotune, "SHIPPED", str(tmp_path / "none.json"))
    assert autotune.load() == {}
    assert autotune.lookup(10, 20, 0) is None


def test_launch_shape_sets_and_restores_environment(monkeypatch):
    monkeypatch.delenv("FLR_TARGET_WG_A", raising=False)
    monkeypatch.setenv("FLR_TARGET_WG_B", "999")
    with autotune.launch_shape(768, 384):
        assert os.environ["FLR_TARGET_WG_A"] == "768"
        assert os.environ["FLR_TARGET_WG_B"] == "384"
    assert "FLR_TARGET_WG_A" not in os.environ
    assert os.environ["FLR_TARGET_WG_B"] == "999"
    with autotune.launch_shape(None, None):  # nothing tuned: the engine's defaults stay
        assert "FLR_TARGET_WG_A" not in os.environ


def test_shipped_cache_entries_are_valid():
    # the repository ships the tuned shapes of the benchmark workloads
    data = autotune.load_shipped()
    assert data, "no shipped tuning entries"
    for key, e in data.items():
        assert key.startswith("gfx950:")
        assert e["target_wg_a"] in autotune.CANDIDATES and e["target_wg_b"] in autotune.CANDIDATES


def test_user_cache_takes_precedence_over_shipped(tmp_path, monkeypatch):
    shipped = tmp_path / "shipped.json"
    shipped.write_text('{"gfx950:n=10:p=20:dtype=0": {"target_wg_a": 256, "target_wg_b": 256}}')
    monkeypatch.setattr(autotune, "SHIPPED", str(shipped))
    monkeypatch.setenv("FLR_TUNE_CACHE", str(tmp_path / "user.json"))
    assert autotune.lookup(10, 20, 0)["target_wg_a"] == 256
    autotune.store(10, 20, 0, {"target_wg_a": 1024, "target_wg_b": 768})
    assert autotune.lookup(10, 20, 0)["target_wg_a"] == 1024
