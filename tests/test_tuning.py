"""The autotuner's JSON cache (host logic, no GPU)."""
import json
import os

import numpy as np

from paper_2409_10743_amd.tuning import TuneCache, batched_key, plain_key, size_class


def test_size_class_rounds_log2():
    assert [size_class(n) for n in (0, 1, 2, 3, 5, 6, 1000, 1 << 24)] == [0, 0, 1, 2, 2, 3, 10, 24]


def test_plain_key_separates_what_changes_the_work():
    k = plain_key("MI355X", 40000, 0.01, 4, "fdbscan")
    assert k == plain_key("MI355X", 41000, np.float32(0.01), 4, "fdbscan")  # same class, same f32
    for other in (plain_key("MI300X", 40000, 0.01, 4, "fdbscan"),
                  plain_key("MI355X", 90000, 0.01, 4, "fdbscan"),
                  plain_key("MI355X", 40000, 0.011, 4, "fdbscan"),
                  plain_key("MI355X", 40000, 0.01, 5, "fdbscan"),
                  plain_key("MI355X", 40000, 0.01, 4, "densebox")):
        assert other != k


def test_batched_key_uses_exact_per_set_parameters():
    off = np.array([0, 10, 30, 60])
    e = np.full(3, 0.05, np.float32)
    m = np.full(3, 5, np.int32)
    k = batched_key("MI355X", off, e, m)
    assert k == batched_key("MI355X", off, e.astype(np.float64), m.astype(np.int64))
    e2 = e.copy()
    e2[1] = np.nextafter(e2[1], np.float32(1))
    assert batched_key("MI355X", off, e2, m) != k
    m2 = m.copy()
    m2[2] = 6
    assert batched_key("MI355X", off, e, m2) != k
    assert batched_key("MI355X", np.array([0, 10, 30]), e[:2], m[:2]) != k


def test_cache_round_trip_and_atomic_file(tmp_path):
    path = tmp_path / "tune.json"
    c = TuneCache(path)
    assert c.get("a") is None and len(c) == 0
    c.put("a", {"block_size": 128, "sort_tile": 0, "ms": 1.5})
    c.put("b", {"block_size": 256, "sort_tile": 2048, "ms": 2.5})
    assert TuneCache(str(path)).get("a") == {"block_size": 128, "sort_tile": 0, "ms": 1.5}
    assert len(c) == 2
    assert json.loads(path.read_text())["b"]["sort_tile"] == 2048
    # no temporary files left beside it
    assert sorted(os.listdir(tmp_path)) == ["tune.json"]
    # a later put replaces the entry
    c.put("a", {"block_size": 64})
    assert c.get("a") == {"block_size": 64}


def test_unreadable_cache_counts_as_empty(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{ not json")
    c = TuneCache(path)
    assert c.get("a") is None
    c.put("a", {"x": 1})
    assert c.get("a") == {"x": 1}
    path.write_text("[1, 2]")  # valid JSON, not an object
    assert c.get("a") is None and len(c) == 0
