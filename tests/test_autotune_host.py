"""Host checks of the launch-parameter autotuner (paper_2109_13993_amd/autotune.py):
the bucket keys, the descent's 1% rule, the cache round trip, and the shipped
MI355X table.  No GPU: the device key is patched in."""
import json
import os

import pytest

from paper_2109_13993_amd import autotune as at


@pytest.fixture
def fake_device(monkeypatch):
    monkeypatch.setattr(at, "_device_key", "gfx950|256 CUs")
    monkeypatch.setattr(at, "_tables", None)
    monkeypatch.setattr(at, "CACHE", "/nonexistent/tune.json")   # the shipped table only
    yield
    at._tables = None


def test_buckets_round_up_to_powers_of_two():
    assert at.bucket("single", "mixed", 500, 20000) == "single/mixed/p512/n32768"
    assert at.bucket("single", "fp32_storage", 1000, 50000) == "single/fp32_storage/p1024/n65536"
    assert at.bucket("batch", "mixed", 100, 5000) == "batch/mixed/p128/n8192"
    assert at.bucket("single", "fp64", 512, 1024) == "single/fp64/p512/n1024"   # exact powers stay
    assert at.bucket("single", "fp64", 1, 1) == "single/fp64/p2/n2"


def test_descent_moves_only_for_a_one_percent_gain():
    times = {(1, 0): 100.0, (2, 0): 99.5, (3, 0): 97.0, (3, 10): 96.5, (3, 20): 95.0}
    seen = []

    def timer(params):
        seen.append((params["a"], params["b"]))
        return times[(params["a"], params["b"])]

    best, t = at._descend({"a": [1, 2, 3], "b": [10, 20]}, {"a": 1, "b": 0}, timer, lambda *x: None)
    # a=2 is 0.5% faster (kept out), a=3 3% faster (taken); then b=10 is 0.5%
    # faster than that (kept out) and b=20 2% faster (taken)
    assert best == {"a": 3, "b": 20} and t == 95.0
    assert seen == [(1, 0), (2, 0), (3, 0), (3, 10), (3, 20)]


def test_store_and_lookup_round_trip(tmp_path, fake_device):
    path = str(tmp_path / "tune.json")
    at.store("single", "mixed", 300, 7000, {"chunk_samples": 2048, "first_band_blocks": 2, "band_target": 1e8},
             0.05, path)
    table = json.load(open(path))
    entry = table["gfx950|256 CUs"]["single/mixed/p512/n8192"]
    assert entry["params"]["first_band_blocks"] == 2 and entry["seconds"] == 0.05
    assert not [f for f in os.listdir(str(tmp_path)) if ".tmp" in f]   # written by rename
    # a cache entry is found before the shipped table's
    at.CACHE = path
    at._tables = None
    assert at.lookup("single", "mixed", 400, 5000) == entry["params"]


def test_shipped_table_is_well_formed(fake_device):
    table = json.load(open(at.SHIPPED))
    assert list(table) == ["gfx950|256 CUs"]
    entries = table["gfx950|256 CUs"]
    kinds = {b.split("/")[0] for b in entries}
    assert kinds == {"single", "batch"}
    for b, e in entries.items():
        kind, precision, p, n = b.split("/")
        assert precision in ("fp64", "mixed", "fp32_storage")
        q = e["params"]
        # the chunk is fixed: another length would round the sums differently
        assert q["chunk_samples"] == at.CHUNK_SAMPLES, b
        assert q["first_band_blocks"] in at.SINGLE_SPACE["first_band_blocks"], b
        assert q["band_target"] in at.SINGLE_SPACE["band_target"], b
        if kind == "batch":
            assert q["batch_queue"] in (0, 1) and q["graph"] in (0, 1), b
        assert e["seconds"] > 0
    # the shipped entries are found through the bucket of a workload's shape
    assert at.lookup("single", "mixed", 500, 20000) == entries["single/mixed/p512/n32768"]["params"]
    assert at.lookup("single", "fp64", 100, 10000) == entries["single/fp64/p128/n16384"]["params"]
    assert at.lookup("single", "mixed", 3000, 20000) is None


def test_unknown_device_finds_nothing(monkeypatch):
    monkeypatch.setattr(at, "_device_key", "gfx942|304 CUs")
    monkeypatch.setattr(at, "_tables", None)
    monkeypatch.setattr(at, "CACHE", "/nonexistent/tune.json")
    assert at.lookup("single", "mixed", 500, 20000) is None
    at._tables = None
