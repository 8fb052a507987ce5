"""The autotuner's JSON cache, on the CPU: keys separate what should be tuned
apart, entries survive a round trip through the file and merge, and a file
of another format or a damaged one reads as empty."""
import json
import os

from paper_1902_08083_amd import trevr as T

INFO = {"n": 1 << 21, "m": 778791, "n_boxes": 1, "max_depth": 29, "prec": 0}


def _key(**kw):
    info = dict(INFO)
    info.update({k: v for k, v in kw.items() if k in info})
    return T.tune_key(info, kw.get("theta", 0.75), kw.get("tau_ref", 0.1), kw.get("sinks"),
                      kw.get("dev", "gfx950"), kw.get("lib", "abc"))


def test_keys_separate_shapes_parameters_devices_and_builds():
    base = _key()
    assert base == _key()
    others = [_key(n=1 << 20), _key(m=5), _key(n_boxes=64), _key(max_depth=30), _key(prec=1),
              _key(theta=0.5), _key(tau_ref=0.2), _key(sinks=4096), _key(dev="other"),
              _key(lib="abd")]
    assert len({base, *others}) == len(others) + 1


def test_round_trip_and_merge(tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    assert T.tune_cache_load(p) == {}
    a = {"launch": [4, 4, 64], "ms": 193.6, "table": [[193.6, [4, 4, 64]], [210.0, [3, 4, 64]]]}
    b = {"launch": [2, 4, 128], "ms": 30.5, "table": [[30.5, [2, 4, 128]]]}
    T.tune_cache_store(p, "ka", a)
    T.tune_cache_store(p, "kb", b)
    got = T.tune_cache_load(p)
    assert got == {"ka": a, "kb": b}
    assert os.listdir(os.path.dirname(p)) == ["tune.json"]  # no temporary file left
    T.tune_cache_store(p, "ka", b)  # a later tuning of the same key replaces it
    assert T.tune_cache_load(p)["ka"] == b


def test_other_format_or_damaged_file_reads_empty(tmp_path):
    p = tmp_path / "tune.json"
    p.write_text(json.dumps({"format": -1, "entries": {"k": {"launch": [1, 1, 64]}}}))
    assert T.tune_cache_load(str(p)) == {}
    p.write_text("{not json")
    assert T.tune_cache_load(str(p)) == {}
    T.tune_cache_store(str(p), "k", {"launch": [1, 1, 64], "ms": 1.0, "table": []})
    assert T.tune_cache_load(str(p)) == {"k": {"launch": [1, 1, 64], "ms": 1.0, "table": []}}


def test_cache_path_follows_the_environment(monkeypatch, tmp_path):
    monkeypatch.setenv("TREVR_TUNE_CACHE", str(tmp_path / "x.json"))
    assert T.tune_cache_path() == str(tmp_path / "x.json")
    monkeypatch.delenv("TREVR_TUNE_CACHE")
    assert T.tune_cache_path().endswith(os.path.join(".cache", "trevr", "autotune.json"))
