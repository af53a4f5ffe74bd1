"""CPU tests of the autotuner's search and cache (no device: the timing
function is replaced by a synthetic cost)."""
import json

from paper_2204_00602_amd import autotune


def test_coordinate_descent_finds_the_separable_minimum():
    space = {"a": [1, 2, 3, 4], "b": [8, 16, 32], "c": [0, 1]}
    best_point = {"a": 3, "b": 16, "c": 1}
    calls = []

    def measure(opts):
        calls.append(dict(opts))
        return sum((opts[k] - best_point[k]) ** 2 for k in opts)

    best, ms, trials = autotune.coordinate_descent(measure, space, {"a": 1, "b": 8, "c": 0}, passes=3)
    assert best == best_point and ms == 0
    # every distinct setting is measured once
    assert trials == len({json.dumps(c, sort_keys=True) for c in calls}) == len(calls)


def test_coordinate_descent_skips_rejected_settings():
    space = {"a": [1, 2, 3]}

    def measure(opts):
        return None if opts["a"] == 3 else 10.0 - opts["a"]

    best, ms, _ = autotune.coordinate_descent(measure, space, {"a": 1})
    assert best == {"a": 2} and ms == 8.0


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    autotune._store(path, "k1", {"options": {"leaf_max": 4096}, "ms": 1.0})
    autotune._store(path, "k2", {"options": {"leaf_max": 8192}, "ms": 2.0})
    data = autotune._load(path)
    assert data["k1"]["options"] == {"leaf_max": 4096} and data["k2"]["ms"] == 2.0
    assert autotune._load(str(tmp_path / "missing.json")) == {}
