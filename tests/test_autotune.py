"""Host logic of the spreading-tile autotuner (CPU): size classes, the JSON
cache, and the choice of the fastest shape, with a stand-in plan object."""
import json

from paper_2604_07170_amd import autotune


class FakePlan:
    SPREAD_TILES = {1: (8, 8), 2: (16, 8), 3: (16, 16), 4: (32, 16), 5: (32, 32)}

    def __init__(self, times, M=100000, band=1024):
        self.times, self.selected, self.timed = times, None, []
        self._info = {"band": band, "M": M, "precision": 1, "nufft_w": 8}

    def info(self):
        return dict(self._info)

    def time_spread(self, code, reps):
        self.timed.append(code)
        self.selected = code
        return self.times[code]

    def set_spread_tile(self, code):
        self.selected = code


def test_size_class_buckets_density_and_band():
    a = autotune.size_class({"band": 1000, "M": 100000, "precision": 1, "nufft_w": 8})
    b = autotune.size_class({"band": 1024, "M": 100000, "precision": 1, "nufft_w": 8})
    c = autotune.size_class({"band": 1024, "M": 400000, "precision": 1, "nufft_w": 8})
    d = autotune.size_class({"band": 1024, "M": 100000, "precision": 0, "nufft_w": 12})
    assert a == b                     # same band class (rounded to 256)
    assert c != b and d != b          # 4x density, other precision / width


def test_tuner_picks_fastest_and_caches(tmp_path):
    path = str(tmp_path / "tiles.json")
    p = FakePlan({1: 3.0, 2: 2.0, 3: 1.5, 4: 0.9, 5: 1.1})
    r = autotune.tune_spread(p, cache=path)
    assert r["code"] == 4 and p.selected == 4 and sorted(p.timed) == [1, 2, 3, 4, 5]
    data = json.load(open(path))
    assert data[r["class"]]["code"] == 4
    q = FakePlan({1: 0.1, 2: 2.0, 3: 1.5, 4: 0.9, 5: 1.1})
    r2 = autotune.tune_spread(q, cache=path)       # cache hit: no timing, cached choice
    assert r2["ms"] is None and q.timed == [] and q.selected == 4
    r3 = autotune.tune_spread(q, cache=path, retune=True)
    assert r3["code"] == 1 and json.load(open(path))[r3["class"]]["code"] == 1


def test_corrupt_cache_is_ignored(tmp_path):
    path = tmp_path / "tiles.json"
    path.write_text("{not json")
    p = FakePlan({1: 3.0, 2: 2.0, 3: 0.5, 4: 0.9, 5: 1.1})
    assert autotune.tune_spread(p, cache=str(path))["code"] == 3
