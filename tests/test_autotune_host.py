"""Host side of the autotuner: the cache of picks and the launch knobs."""
import os

from paper_2012_05348_amd import autotune


def test_cache_round_trip_per_workload(tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    a = {"branching": 8, "treelet_bytes": 8192, "waves_per_cu": 0, "waves_per_group": 2, "ms": 0.5}
    b = {"branching": 4, "treelet_bytes": 2048, "waves_per_cu": 8, "waves_per_group": 1, "ms": 0.7}
    autotune.save("w1", a, p)
    autotune.save("w2", b, p)
    assert autotune.load("w1", p) == a and autotune.load("w2", p) == b
    assert autotune.load("w3", p) is None
    assert autotune.load("w1", str(tmp_path / "missing.json")) is None
    assert autotune.build_kwargs(b) == {"branching": 4, "treelet_bytes": 2048}
    assert autotune.build_kwargs(None) == {"branching": 8, "treelet_bytes": 0}


def test_launch_env_sets_and_restores_the_knobs(monkeypatch):
    monkeypatch.setenv(autotune.WAVES_ENV, "6")
    monkeypatch.delenv(autotune.GROUP_ENV, raising=False)
    with autotune.launch_env({"waves_per_cu": 0, "waves_per_group": 4}):
        assert autotune.WAVES_ENV not in os.environ
        assert os.environ[autotune.GROUP_ENV] == "4"
    assert os.environ[autotune.WAVES_ENV] == "6" and autotune.GROUP_ENV not in os.environ


def test_cache_path_follows_the_environment(monkeypatch, tmp_path):
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "x.json"))
    assert autotune.cache_path() == str(tmp_path / "x.json")
    assert autotune.cache_path("given.json") == "given.json"


def test_launch_env_without_a_pick_changes_nothing(monkeypatch):
    monkeypatch.setenv(autotune.WAVES_ENV, "6")
    with autotune.launch_env(None):
        assert os.environ[autotune.WAVES_ENV] == "6"
    assert os.environ[autotune.WAVES_ENV] == "6"


def test_launch_env_counts_helpers_per_cu(monkeypatch):
    monkeypatch.setattr(autotune, "_cu_count", lambda: 256)
    monkeypatch.setenv(autotune.HELPERS_ENV, "7")
    with autotune.launch_env({"waves_per_group": 1, "helpers_per_cu": 2}):
        assert os.environ[autotune.HELPERS_ENV] == "512"
    assert os.environ[autotune.HELPERS_ENV] == "7"
    with autotune.launch_env({"waves_per_group": 1}):
        assert autotune.HELPERS_ENV not in os.environ
    with autotune.launch_env({"helpers_per_cu": 2, "max_helpers": 32}):
        assert os.environ[autotune.HELPERS_ENV] == "32"
    assert os.environ[autotune.HELPERS_ENV] == "7"
