"""Autotuner table logic (CPU): nearest-class fill, the library's tuning
table through the C ABI, recorded leaf sizes, and the committed table's
consistency with its own measurements."""
import os

import pytest

import paper_1610_05141_amd as dcs
from paper_1610_05141_amd import autotune

SYNTH = {
    "geometry": [
        {"variant": 0, "log2_n": 10, "cut_bias": 1, "leaf_wgs_per_cu": 2},
        {"variant": 0, "log2_n": 20, "cut_bias": -1, "leaf_wgs_per_cu": 3},
        {"variant": 1, "log2_n": 16, "cut_bias": 2, "leaf_wgs_per_cu": 1},
    ],
    "leaf_size": [
        {"log2_n": 10, "dense": False, "n0": 1024},
        {"log2_n": 20, "dense": False, "n0": 4096},
        {"log2_n": 14, "dense": True, "n0": 2048},
    ],
}


def test_geometry_rows_nearest_class():
    rows = {(v, c): (cb, w) for v, c, cb, w in autotune.geometry_rows(SYNTH)}
    assert len(rows) == 2 * autotune.N_CLASSES
    assert rows[(0, 0)] == (1, 2) and rows[(0, 15)] == (1, 2)   # 15 is nearer 10 (tie -> first)
    assert rows[(0, 16)] == (-1, 3) and rows[(0, 63)] == (-1, 3)
    assert all(rows[(1, c)] == (2, 1) for c in range(autotune.N_CLASSES))


def test_apply_table_calls_library():
    calls = []

    class FakeLib:
        def dcs_tune_set(self, *a):
            calls.append(a)
            return 0

    assert autotune.apply_table(FakeLib(), SYNTH)
    assert len(calls) == 2 * autotune.N_CLASSES
    assert (0, 25, -1, 3) in calls and (1, 3, 2, 1) in calls
    assert not autotune.apply_table(FakeLib(), {})


def test_n0_for_recorded_classes():
    assert autotune.n0_for(1500, 10**9, SYNTH) == 1024          # class 10, sparse
    assert autotune.n0_for(1 << 20, 1 << 40, SYNTH) == 4096     # class 20, sparse
    assert autotune.n0_for(1 << 14, 1 << 15, SYNTH) == 2048     # dense
    assert autotune.n0_for(1 << 22, 1 << 23, SYNTH) == 2048     # nearest dense class
    assert autotune.n0_for(100, 1000, {}) == autotune.DEFAULT_N0


def test_library_tuning_table_roundtrip():
    if not os.path.exists(dcs.LIB_PATH):
        pytest.skip("library not built")
    dcs.lib()
    saved = [(v, c, *dcs.tune_get(v, c)) for v in (0, 1) for c in range(autotune.N_CLASSES)]
    try:
        dcs.tune_set(0, 30, -2, 1)
        dcs.tune_set(1, 0, 16, 64)
        assert dcs.tune_get(0, 30) == (-2, 1)
        assert dcs.tune_get(1, 0) == (16, 64)
        for bad in [(2, 0, 0, 0), (0, 64, 0, 0), (0, 1, 17, 0), (0, 1, -17, 0), (0, 1, 0, 65)]:
            with pytest.raises(dcs.DcsError):
                dcs.tune_set(*bad)
        dcs.tune_reset()
        assert all(dcs.tune_get(v, c) == (0, 0) for v in (0, 1) for c in (0, 17, 63))
    finally:
        for v, c, cb, w in saved:
            dcs.tune_set(v, c, cb, w)


def test_committed_table_is_consistent():
    t = autotune.load_table()
    if t is None:
        pytest.skip("no tuning table committed")
    for e in t["geometry"]:
        assert e["variant"] in (0, 1) and 0 <= e["log2_n"] < autotune.N_CLASSES
        assert e["cut_bias"] in autotune.CUT_BIASES and e["leaf_wgs_per_cu"] in autotune.LEAF_WGS
        best = min(e["ms"], key=e["ms"].get)
        assert best == f"{e['cut_bias']},{e['leaf_wgs_per_cu']}"
        assert e["best_ms"] <= e["default_ms"]
    for e in t["leaf_size"]:
        assert e["n0"] in autotune.N0_CHOICES
        assert min(e["ms"], key=e["ms"].get) == str(e["n0"])
