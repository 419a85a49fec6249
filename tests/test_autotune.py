"""Autotuner host logic: search, result-invariance guard, cache keys and the
JSON cache round trip (a simulated runner stands in for the GPU)."""
import json

import pytest

from paper_2604_01397_amd import autotune as at


def test_key_and_size_class():
    assert at.size_class(1) == 0 and at.size_class(2) == 1 and at.size_class(3) == 1
    assert at.size_class(512 ** 3) == 27
    assert at.make_key("gfx950:sramecc+:xnack-", 3, "f32", 512 ** 3) == "gfx950|3d|f32|2^27"
    assert at.field_ndim((512, 512, 512)) == 3
    assert at.field_ndim((1, 300, 400)) == 2
    assert at.field_ndim((1, 1, 70)) == 1 and at.field_ndim((70,)) == 1


def test_search_space_per_dimensionality():
    s3, s2, s1 = at.search_space(3), at.search_space(2), at.search_space(1)
    assert len({c.tile for c in s3}) == len(at.BOXES_3D)
    assert all(c.tile % 100 == 1 for c in s2)  # planes: one z row per box
    assert {c.tile for c in s1} == {101}
    assert len(at.search_space(3, quick=True)) < len(s3)
    assert len(set(s3)) == len(s3)


def test_search_picks_fastest_and_guards_results():
    cands = at.search_space(3, quick=True)
    cost = {c: 10.0 + i for i, c in enumerate(cands)}
    fast = cands[len(cands) // 2]
    cost[fast] = 1.0
    best, table = at.search(lambda c: (cost[c], "same"), cands, repeats=2)
    assert best == fast and len(table) == len(cands)
    with pytest.raises(at.TuneError):
        at.search(lambda c: (1.0, "bad" if c == fast else "same"), cands)
    with pytest.raises(at.TuneError):
        at.search(lambda c: (1.0, "x"), [])


def test_repeats_take_the_minimum():
    c = at.Candidate(408, -1, 1, 0)
    times = iter([5.0, 3.0, 4.0])
    best, table = at.search(lambda _: (next(times), 0), [c], repeats=3)
    assert table == [(c, 3.0)]


def test_cache_round_trip(tmp_path, monkeypatch):
    p = str(tmp_path / "sub" / "tune.json")
    assert at.load_cache(p) == {}
    key = at.make_key("gfx950", 3, "f32", 1 << 21)
    at.save_cache({key: {"tile": 804, "grid": -1, "frontier": 1, "poll": 0, "ms": 1.5}}, p)
    assert json.load(open(p))[key]["tile"] == 804
    assert at.options_for("gfx950:sramecc+", 3, "f32", (1 << 21) + 5, p) == {
        "tile": 804, "grid": -1, "frontier": 1, "poll": 0}
    assert at.options_for("gfx950", 3, "f32", 1 << 23, p) is None  # other size class
    assert at.options_for("gfx942", 3, "f32", 1 << 21, p) is None  # other architecture
    monkeypatch.setenv("EXACTZ_AUTOTUNE_CACHE", p)
    assert at.cache_path() == p
    open(p, "w").write("{not json")
    assert at.load_cache(p) == {}


def test_batch_key_and_signature():
    sig = at.batch_signature([((64, 64, 64), "f32"), ((1, 300, 400), "f64"), ((70,), "f32")])
    assert sig == ((1, 2, 3), ("f32", "f64"), 64 ** 3 + 300 * 400 + 70)
    key = at.make_batch_key("gfx950:sramecc+:xnack-", *sig)
    assert key == "gfx950|batch|1d+2d+3d|f32+f64|2^18"
    # a batch key never collides with a single-field key
    assert key != at.make_key("gfx950", 3, "f32", 64 ** 3)


def test_coordinate_search_descends_axis_by_axis():
    axes = {"btile3": [0, 804, 404], "bgrid_box": [0, 1024], "bitem": [0, 4, 64]}
    # separable cost with its minimum at (404, 1024, 4)
    cost_axis = {"btile3": {0: 3.0, 804: 2.0, 404: 1.0}, "bgrid_box": {0: 2.0, 1024: 1.0},
                 "bitem": {0: 3.0, 4: 1.0, 64: 2.0}}
    calls = []

    def run(c):
        calls.append(c)
        return sum(cost_axis[k][getattr(c, k)] for k in axes), "same"

    best, table = at.coordinate_search(run, axes, at.BATCH_DEFAULT)
    assert (best.btile3, best.bgrid_box, best.bitem) == (404, 1024, 4)
    assert best.btile2 == 0 and best.bgrid_apply == 0  # untouched axes keep the default
    # every distinct candidate is timed once: 1 + 2 + 1 + 2 new ones
    assert len(table) == len(set(calls)) == 6
    with pytest.raises(at.TuneError):
        at.coordinate_search(lambda c: (1.0, "bad" if c.bitem == 64 else "same"), axes,
                             at.BATCH_DEFAULT)


def test_shipped_table_and_cache_precedence(tmp_path, monkeypatch):
    key = at.make_batch_key("gfx950", (3,), ("f32",), 1 << 24)
    shipped = tmp_path / "tuned"
    shipped.mkdir()
    (shipped / "gfx950.json").write_text(json.dumps({key: {"btile3": 804, "btile2": 0,
                                                           "bgrid_box": 2048, "bgrid_apply": 0,
                                                           "bitem": 4, "ms": 1.0}}))
    monkeypatch.setattr(at, "SHIPPED", str(shipped))
    cache = str(tmp_path / "user.json")
    assert at.batch_options_for(key, cache)["btile3"] == 804  # from the shipped table
    at.save_cache({key: {"btile3": 404, "btile2": 801, "bgrid_box": 0, "bgrid_apply": 0,
                         "bitem": 0}}, cache)
    assert at.batch_options_for(key, cache)["btile3"] == 404  # the user's cache wins
    assert at.batch_options_for(key.replace("gfx950", "gfx942"), cache) is None


def test_shipped_table_keys_are_well_formed():
    """Every entry of the committed tables parses and names only compiled
    boxes and options the library accepts."""
    import glob
    import os
    files = glob.glob(os.path.join(at.SHIPPED, "*.json"))
    for path in files:
        table = json.load(open(path))
        arch = os.path.basename(path)[:-5]
        for key, e in table.items():
            parts = key.split("|")
            assert parts[0] == arch
            if parts[1] in ("batch", "serving"):
                assert set(at.BATCH_KEYS) <= set(e)
                assert e["btile3"] in at.BATCH_AXES["btile3"]
                assert e["btile2"] in at.BATCH_AXES["btile2"]
            else:
                assert {"tile", "grid", "frontier", "poll"} <= set(e)
            assert e["ms"] <= (e.get("default_ms") or e["ms"]) + 1e-9
