"""Host logic of the launch-shape autotuner: the search and the cache."""
import os

from paper_1602_02306_amd import autotune


def test_coordinate_search_finds_separable_minimum():
    # cost separable in the parameters: coordinate descent reaches the optimum
    cost = {"a": {1: 5.0, 2: 1.0, 3: 3.0}, "b": {"x": 2.0, "y": 0.5}}
    calls = []

    def run(cfg):
        calls.append(dict(cfg))
        return 10.0 + cost["a"][cfg["a"]] + cost["b"][cfg["b"]]

    best, ms, trials = autotune.coordinate_search(run, {"a": [1, 2, 3], "b": ["x", "y"]},
                                                  {"a": 1, "b": "x"})
    assert best == {"a": 2, "b": "y"}
    assert ms == 11.5
    assert len(trials) == len(calls) == 1 + 2 + 1


def test_coordinate_search_ignores_small_gains():
    best, ms, _ = autotune.coordinate_search(lambda c: 100.0 - c["a"] * 0.5, {"a": [0, 1, 2]},
                                             {"a": 0})
    assert best == {"a": 0}   # 1% faster is within the 2% noise margin


def test_cache_roundtrip(tmp_path):
    path = os.path.join(tmp_path, "sub", "tune.json")
    assert autotune.load_cache(path) == {}
    autotune.save_cache({"k1": {"tile": "2x4"}}, path)
    assert autotune.load_cache(path) == {"k1": {"tile": "2x4"}}
    open(path, "w").write("not json")
    assert autotune.load_cache(path) == {}


def test_size_class_buckets():
    a = autotune.size_class(5_965_950, 64, 256, 25, "f64", "cheb")
    b = autotune.size_class(6_100_000, 64, 256, 25, "f64", "cheb")
    c = autotune.size_class(5_965_950, 64, 256, 25, "f32", "cheb")
    assert a == b and a != c
