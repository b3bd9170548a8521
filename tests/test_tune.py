"""The autotuner's selection and cache logic with a fake clock (no GPU): the
batch is a stand-in that records geometries, the timer returns a cost that
depends on the geometry in force."""
import json

import pytest

from paper_2201_13020_amd import szx, tune

DEV = "gfx950|cu256"


class FakeBatch:
    def __init__(self):
        self.geom = {}
        self.runs = 0
        self.log = []

    def run(self, stream=None):
        self.runs += 1

    def set_geometry(self, encode_wgs, dtype=None):
        self.geom[dtype] = encode_wgs
        self.log.append((dtype, encode_wgs))


def fake_timer(batch, cost):
    """timer(fn, reps): the cost of the geometry in force, fn run reps times."""
    calls = []

    def timer(fn, reps):
        for _ in range(reps):
            fn()
        dtype = batch.log[-1][0]
        calls.append((dtype, batch.geom[dtype]))
        return cost(dtype, batch.geom[dtype])
    return timer, calls


@pytest.fixture
def cache(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("SZX_TUNE_CACHE", str(path))
    table = []
    monkeypatch.setattr(szx, "set_geometry", lambda dt, cls, wgs: table.append((dt, cls, wgs)))
    return path, table


def test_selects_the_fastest_candidate_per_dtype(cache):
    path, table = cache
    b = FakeBatch()
    # float32: fastest at 3 per CU; float64: fastest at 12 per CU
    best = {"float32": 3 * 256, "float64": 12 * 256}
    timer, calls = fake_timer(b, lambda dt, w: 1.0 + abs(w - best[dt]) / 1000.0)
    nbytes = {"float32": 3 << 30, "float64": 5 << 20}
    res = tune.tune_batch(b, nbytes, block=128, reps=3, timer=timer, device=DEV)
    for dt in ("float32", "float64"):
        wgs, ms, times = res[dt]
        assert wgs == best[dt] and ms == pytest.approx(1.0)
        assert sorted(times) == [m * 256 for m in tune.MULTIPLIERS]
        assert b.geom[dt] == best[dt]  # the batch keeps the best
    # every candidate of both types timed once, reps runs each, plus one warm run
    assert len(calls) == 2 * len(tune.MULTIPLIERS)
    assert b.runs == 1 + 3 * len(calls)
    # the library table and the cache hold the size class of each type's bytes
    cls = {dt: szx.size_class(v) for dt, v in nbytes.items()}
    assert cls["float32"] != cls["float64"]
    assert sorted(table) == sorted((dt, cls[dt], best[dt]) for dt in best)
    entries = json.loads(path.read_text())
    assert set(entries) == {f"{DEV}|b128|{dt}|c{cls[dt]}" for dt in best}
    for dt in best:
        e = entries[f"{DEV}|b128|{dt}|c{cls[dt]}"]
        assert e["encode_wgs"] == best[dt] and e["bytes"] == nbytes[dt]


def test_ties_keep_the_smaller_geometry_and_absent_types_are_skipped(cache):
    path, table = cache
    b = FakeBatch()
    timer, calls = fake_timer(b, lambda dt, w: 2.0 if w < 4 * 256 else 1.0)
    res = tune.tune_batch(b, {"float32": 1 << 20, "float64": 0}, reps=1, timer=timer, device=DEV)
    assert set(res) == {"float32"}
    assert res["float32"][0] == 4 * 256  # first of the equal fastest
    assert all(dt == "float32" for dt, _ in calls) and "float64" not in b.geom


def test_store_false_leaves_the_cache_alone(cache):
    path, table = cache
    b = FakeBatch()
    timer, _ = fake_timer(b, lambda dt, w: float(w))
    tune.tune_batch(b, {"float64": 1 << 24}, reps=1, timer=timer, device=DEV, store=False)
    assert not path.exists()
    assert table == [("float64", szx.size_class(1 << 24), 256)]


def test_cache_merges_runs_and_apply_selects_device_and_block(cache):
    path, table = cache
    b = FakeBatch()
    t1, _ = fake_timer(b, lambda dt, w: abs(w - 2048))
    tune.tune_batch(b, {"float32": 1 << 30}, block=128, reps=1, timer=t1, device=DEV)
    t2, _ = fake_timer(b, lambda dt, w: abs(w - 512))
    tune.tune_batch(b, {"float32": 1 << 30}, block=16, reps=1, timer=t2, device=DEV)
    t3, _ = fake_timer(b, lambda dt, w: abs(w - 64 * 6))
    tune.tune_batch(b, {"float64": 1 << 30}, block=128, reps=1, timer=t3, device="gfx942|cu64")
    entries = json.loads(path.read_text())
    assert len(entries) == 3
    c = szx.size_class(1 << 30)
    table.clear()
    assert tune.apply_cache(DEV, block=128) == 1 and table == [("float32", c, 2048)]
    table.clear()
    assert tune.apply_cache(DEV, block=16) == 1 and table == [("float32", c, 512)]
    table.clear()
    assert tune.apply_cache(DEV, block=64) == 0 and table == []
    assert tune.apply_cache("gfx942|cu64", block=128) == 1 and table == [("float64", c, 384)]


def test_apply_cache_tolerates_missing_and_foreign_files(cache):
    path, table = cache
    assert tune.apply_cache(DEV) == 0
    path.write_text("not json")
    assert tune.apply_cache(DEV) == 0
    path.write_text(json.dumps({"odd-key": {"encode_wgs": 1}, f"{DEV}|b128|float32|c2": {"encode_wgs": 999}}))
    assert tune.apply_cache(DEV) == 1 and table == [("float32", 2, 999)]
