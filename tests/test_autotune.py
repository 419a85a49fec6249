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
