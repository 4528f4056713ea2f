"""Autotuner schedule cache (host-only logic)."""
from paper_1307_6489_amd import autotune


def test_cache_roundtrip(tmp_path):
    path = str(tmp_path / "sched.json")
    assert autotune.load_cache(path) == {}
    entries = {"gfx950|1855x40x2;1764x25x2;2048x128x2": {"schedule": [4, 4, 0, 16], "ms": 12.7}}
    autotune.save_cache(entries, path)
    assert autotune.load_cache(path) == entries
    entries["other"] = {"schedule": [8, 4, 2, 8], "ms": 14.0}
    autotune.save_cache(entries, path)
    assert autotune.load_cache(path)["other"]["schedule"] == [8, 4, 2, 8]


def test_corrupt_cache_is_ignored(tmp_path):
    path = tmp_path / "bad.json"
    path.write_text("{not json")
    assert autotune.load_cache(str(path)) == {}
