"""The library's schedule tune cache (host-only calls of librta, no GPU)."""
import ctypes

import pytest

import paper_1307_6489_amd as rta

KEY = "gfx950|e0w4|1855x40x2;1764x25x2;2048x128x2"


def test_missing_file_is_untuned(tmp_path):
    assert rta.tune_cache_lookup(str(tmp_path / "none.tsv"), KEY) is None


def test_store_lookup_replace(tmp_path):
    path = str(tmp_path / "sched.tsv")
    rta.tune_cache_store(path, KEY, (4, 4, 0, 16), 12.7)
    s, ms = rta.tune_cache_lookup(path, KEY)
    assert s == (4, 4, 0, 16) and ms == pytest.approx(12.7, rel=1e-6)
    other = "gfx950|e1w4|2048x128x2"
    rta.tune_cache_store(path, other, (8, 4, 2, 8), 14.0)
    rta.tune_cache_store(path, KEY, (8, 8, 0, 8), 11.5)
    assert rta.tune_cache_lookup(path, KEY)[0] == (8, 8, 0, 8)
    assert rta.tune_cache_lookup(path, other)[0] == (8, 4, 2, 8)
    assert rta.tune_cache_lookup(path, "gfx950|e0w4|2048x128x2") is None
    body = open(path).read().splitlines()
    entries = [l for l in body if not l.startswith("#")]
    assert len(entries) == 2 and sum(l.startswith(KEY + "\t") for l in entries) == 1


def test_corrupt_and_foreign_lines_are_ignored(tmp_path):
    path = tmp_path / "bad.tsv"
    path.write_text("{not a cache\n%s\t8 4\t1.0\n%s\t8 4 0 8\t2.0 trailing\n\n# comment\n" % (KEY, KEY))
    assert rta.tune_cache_lookup(str(path), KEY) is None
    # a store keeps only parseable entries and adds its own
    rta.tune_cache_store(str(path), KEY, (2, 4, 1, 8), 3.0)
    assert rta.tune_cache_lookup(str(path), KEY)[0] == (2, 4, 1, 8)
    assert "{not a cache" not in path.read_text()


def test_schedule_not_compiled_is_untuned(tmp_path):
    path = tmp_path / "old.tsv"
    path.write_text("%s\t3 4 0 8\t1.0\n" % KEY)  # 3 pixels per lane is not a compiled schedule
    assert rta.tune_cache_lookup(str(path), KEY) is None
    with pytest.raises(rta.RTAError) as e:
        rta.tune_cache_store(str(path), KEY, (3, 4, 0, 8), 1.0)
    assert e.value.status == 5


def test_bad_keys_and_paths_are_rejected(tmp_path):
    path = str(tmp_path / "k.tsv")
    for key in ("a\tb", "a\nb", ""):
        with pytest.raises(rta.RTAError) as e:
            rta.tune_cache_store(path, key, (8, 4, 0, 8), 1.0)
        assert e.value.status == 1
    with pytest.raises(rta.RTAError) as e:
        rta.tune_cache_store(str(tmp_path / "no_such_dir" / "k.tsv"), KEY, (8, 4, 0, 8), 1.0)
    assert e.value.status == 1


def test_status_string():
    assert rta.lib().rta_status_str(rta.RTA_E_UNTUNED).decode() == "no tuned schedule"
    assert ctypes.sizeof(rta.PipelineParams) == 40
