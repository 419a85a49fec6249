"""Pins of the CPU oracle against things other than itself.

* the mesh and the link structure against the simplicial complex of the
  Kuhn triangulation, rebuilt independently by the checker;
* critical types / steepest neighbours against brute-force link analysis;
* the band bounds against exact rational arithmetic;
* worked examples constructed from the paper's narrated figures;
* on random tiny fields: the corrected field must have the same critical
  points, extremum graph, join/split/contour trees as f (union-find sweeps),
  stay in the error band, only decrease, respect the vulnerability-graph
  iteration bound (Sec. 4.4) and never edit outside the reduced graph.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import checker as ck

SHAPES = [(9,), (12,), (5, 4), (6, 5), (4, 4, 3), (3, 3, 3), (5, 3, 2)]


def _rand_case(rng, shape, dtype, kind):
    n = int(np.prod(shape))
    if kind == "plateau":
        f = rng.integers(0, 7, size=n).astype(dtype)
        xi = 2.0
        g = f + rng.integers(-8, 9, size=n).astype(dtype) / dtype(4.0)
    else:
        f = rng.standard_normal(n).astype(dtype)
        xi = float(dtype(0.3))
        g = np.clip(f + rng.uniform(-xi, xi, n).astype(dtype), f - dtype(0), f + dtype(0))
        g = (f.astype(np.float64) + rng.uniform(-0.29, 0.29, n)).astype(dtype)
    f = f.reshape(tuple(reversed(shape)))
    g = g.reshape(f.shape).astype(dtype)
    return f, g, xi


# ----------------------------------------------------------------------------
# mesh, links, types


@pytest.mark.parametrize("shape", [(6,), (5, 4), (4, 3, 3)])
def test_neighbours_match_kuhn_complex(shape):
    cx = ck.Complex(list(shape))
    offs = oracle.offsets(len(shape))
    for i in range(cx.n):
        x, y, z = cx.coords(i)
        mine = set()
        for dx, dy, dz in offs:
            X, Y, Z = x + dx, y + dy, z + dz
            if 0 <= X < cx.dims[0] and 0 <= Y < cx.dims[1] and 0 <= Z < cx.dims[2]:
                mine.add(X + cx.dims[0] * (Y + cx.dims[1] * Z))
        assert mine == cx.nbrs[i]


def test_interior_link_shapes():
    # 3D Freudenthal: the link of an interior vertex is a triangulated sphere
    # with 14 vertices, 36 edges and 24 triangles (chi = 2); 2D: a 6-cycle.
    cx = ck.Complex([3, 3, 3])
    c = 13
    counts = {k: sum(1 for t in cx.link[c] if len(t) == k) for k in (1, 2, 3)}
    assert counts == {1: 14, 2: 36, 3: 24}
    assert counts[1] - counts[2] + counts[3] == 2
    cx2 = ck.Complex([3, 3])
    counts2 = {k: sum(1 for t in cx2.link[4] if len(t) == k) for k in (1, 2)}
    assert counts2 == {1: 6, 2: 6}
    assert len(oracle.offsets(3)) == 14 and len(oracle.offsets(2)) == 6


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("shape", SHAPES)
def test_topology_matches_bruteforce(shape, seed):
    rng = np.random.default_rng(seed)
    for dtype in (np.float32, np.float64):
        h = rng.integers(0, 4, size=int(np.prod(shape))).astype(dtype)
        h = h.reshape(tuple(reversed(shape)))
        mine = oracle.topology(h)
        cx = ck.Complex(list(shape))
        ref = ck.classify(cx, h.ravel())
        for v in range(cx.n):
            assert mine["type"][v] == ref[v]["type"], v
            assert mine["asc"][v] == ref[v]["asc"]
            assert mine["desc"][v] == ref[v]["desc"]
            if ref[v]["lower"] and ref[v]["upper"]:
                assert mine["lc"][v] == ref[v]["lc"]
                assert mine["uc"][v] == ref[v]["uc"]


@pytest.mark.parametrize("shape", SHAPES)
def test_euler_sum_is_one(shape):
    # sum_v (1 - chi(lower link of v)) = chi(ball) = 1; pins the checker's
    # complex and lower links.
    rng = np.random.default_rng(7)
    cx = ck.Complex(list(shape))
    for _ in range(3):
        h = rng.integers(0, 3, size=cx.n).astype(np.float64)
        assert ck.euler_sum(cx, h) == 1


def test_critical_order_is_sos_sorted():
    rng = np.random.default_rng(3)
    h = rng.integers(0, 3, size=(4, 4, 4)).astype(np.float32)
    order = oracle.critical_order(h)
    ty = oracle.topology(h)["type"]
    assert set(order.tolist()) == set(np.nonzero(ty != oracle.TYPE_REGULAR)[0].tolist())
    flat = h.ravel()
    assert sorted(order.tolist(), key=lambda i: (flat[i], i)) == order.tolist()


# ----------------------------------------------------------------------------
# bounds


def _exact_bounds(fv, xiT, dtype):
    t_lo = Fraction(float(fv)) - Fraction(float(xiT))
    t_hi = Fraction(float(fv)) + Fraction(float(xiT))
    lo = dtype(float(t_lo))
    while Fraction(float(lo)) < t_lo:
        lo = np.nextafter(lo, dtype(np.inf))
    while Fraction(float(np.nextafter(lo, dtype(-np.inf)))) >= t_lo:
        lo = np.nextafter(lo, dtype(-np.inf))
    hi = dtype(float(t_hi))
    while Fraction(float(hi)) > t_hi:
        hi = np.nextafter(hi, dtype(-np.inf))
    while Fraction(float(np.nextafter(hi, dtype(np.inf)))) <= t_hi:
        hi = np.nextafter(hi, dtype(np.inf))
    return lo, hi


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_bounds_exact(dtype):
    rng = np.random.default_rng(11)
    tiny = np.finfo(dtype).tiny
    vals = np.concatenate([
        rng.standard_normal(300) * 10.0 ** rng.integers(-6, 6, 300),
        [0.0, -0.0, tiny, -tiny, tiny / 8, 1e-8, 5e-9, 1.0, -1.0, 2.0, 0.5,
         np.finfo(dtype).max / 2],
    ]).astype(dtype)
    for xi in (1e-3, 0.3, 1.0, 1.0 / 3.0, 1e-30):
        L, U, xiT, delta = oracle.bounds(vals, xi, n_steps=5)
        # xi_T = largest dtype value <= xi
        assert Fraction(xiT) <= Fraction(xi)
        assert Fraction(float(np.nextafter(dtype(xiT), dtype(np.inf)))) > Fraction(xi)
        # Delta = xi_T / 5 rounded to nearest
        q = Fraction(xiT) / 5
        d = dtype(delta)
        for nb in (np.nextafter(d, dtype(np.inf)), np.nextafter(d, dtype(-np.inf))):
            assert abs(Fraction(float(d)) - q) <= abs(Fraction(float(nb)) - q)
        for k in range(vals.size):
            lo, hi = _exact_bounds(vals[k], xiT, dtype)
            assert L[k] == lo, (vals[k], xi)
            assert U[k] == hi, (vals[k], xi)


# ----------------------------------------------------------------------------
# worked examples


GOLDEN_RUNS = ["cascade_1d.txt", "edit_minimum_1d.txt", "floor_collapse_1d.txt",
               "original_mode_join_c2_2d.txt", "original_mode_split_c2_2d.txt",
               "original_mode_join_glink_2d.txt", "original_mode_split_tie_2d.txt"]


@pytest.mark.parametrize("name", GOLDEN_RUNS)
def test_golden_examples(golden, name):
    gd = golden(name)
    dt = np.dtype(gd["dtype"][0]).type
    shape = tuple(reversed([int(v) for v in gd["dims"]]))
    mode = {"reformulated": oracle.REFORMULATED,
            "original": oracle.ORIGINAL}[gd.get("mode", ["reformulated"])[0]]
    f = np.array([float(v) for v in gd["f"]], dt).reshape(shape)
    g = np.array([float(v) for v in gd["g_hat"]], dt).reshape(shape)
    xi = float(gd["xi"][0])
    N = int(gd["n_steps"][0])
    g_out, cnt, st, _ = oracle.correct(f, g, xi, n_steps=N, mode=mode)
    assert g_out.ravel().tolist() == [dt(float(v)) for v in gd["g_out"]]
    assert cnt.ravel().tolist() == [int(v) for v in gd["cnt"]]
    assert st["iterations"] == int(gd["iterations"][0])
    assert st["status"] == int(gd.get("status", ["0"])[0])
    assert st["residual_violations"] == int(gd.get("residual", ["0"])[0])
    if "lossless" in gd:
        assert st["lossless_vertices"] == int(gd["lossless"][0])
    # per-iteration target sets (every iteration the fixture lists)
    listed = [k for k in gd if k.startswith("targets_")]
    assert all(int(k.split("_")[1]) <= st["iterations"] for k in listed)
    cur = g.copy()
    for it in range(1, st["iterations"] + 1):
        key = "targets_%d" % it
        tg = np.nonzero(oracle.targets(f, cur, mode).ravel())[0].tolist()
        if key in gd:
            assert tg == [int(v) for v in gd[key]], it
        cur, _, _, _ = oracle.correct(f, g, xi, n_steps=N, mode=mode, max_iters=it)
    assert not oracle.targets(f, g_out, mode).any() or st["status"] == oracle.STUCK


# ----------------------------------------------------------------------------
# random tiny fields: certificates


def _check_certificates(f, g, xi, g_out, cnt, st, N, mode):
    shape = list(reversed(f.shape))
    cx = ck.Complex(shape)
    L, U, xiT, _ = oracle.bounds(f.ravel(), xi, N)
    fo, go, gh = f.ravel(), g_out.ravel(), g.ravel()
    # band and monotone
    assert np.all(go >= L) and np.all(go <= U)
    assert np.all(go <= gh)
    assert np.all(cnt <= N + 1)
    assert np.all((go != gh) <= (cnt.ravel() > 0))
    # counters
    c = cnt.ravel()
    assert st["edited_vertices"] == int((c > 0).sum())
    assert st["lossless_vertices"] == int((c > N).sum())
    assert st["edit_ops"] == int(c.sum())
    assert st["floor_vertices"] == int(((go == L) & (c > 0)).sum())
    tg = oracle.targets(f, g_out, mode)
    if st["status"] == oracle.STUCK:
        assert tg.sum() == st["residual_violations"] > 0
        return False
    assert st["status"] == oracle.OK
    assert not tg.any()
    # topology identity.  Both modes keep the critical points and the
    # extremum graph; only the reformulated constraints (total order of all
    # critical points) also pin the merge-tree pairing, see
    # test_original_mode_can_change_a_split_pair.
    a = ck.topology_signature(cx, fo)
    b = ck.topology_signature(cx, go)
    keys = list(a) if mode == oracle.REFORMULATED else ["critical", "eg"]
    for key in keys:
        assert a[key] == b[key], key
    if mode == oracle.ORIGINAL:
        # C2: the saddles of f keep their order; C3: every saddle of f pairs
        # with the same extremum as in f (the checker's own links and paths)
        assert ck.saddle_sequence(cx, fo, go) == ck.saddle_sequence(cx, fo, fo)
        assert ck.event_selections(cx, fo, go) == ck.event_selections(cx, fo, fo)
    # iteration bound and edit locality (reformulated mode pairs)
    if mode == oracle.REFORMULATED:
        vg = ck.vulnerability(cx, fo, gh, xiT)
        assert st["iterations"] <= (N + 1) * vg["D_max"]
        edited = set(np.nonzero(c)[0].tolist())
        assert edited <= vg["GR_vertices"]
    return True


# 1D fields have no saddles, so the original event constraints (C2, C3) say
# nothing there: the original mode is certified on 2D and 3D shapes only.
@pytest.mark.parametrize("shape,mode", [(s, m) for m in (oracle.REFORMULATED, oracle.ORIGINAL)
                                        for s in SHAPES
                                        if not (m == oracle.ORIGINAL and len(s) == 1)])
def test_random_tiny_certificates(shape, mode):
    rng = np.random.default_rng(hash((shape, mode)) % 2 ** 32)
    converged = 0
    for trial in range(8):
        dtype = np.float32 if trial % 2 == 0 else np.float64
        kind = "plateau" if trial % 4 < 2 else "real"
        f, g, xi = _rand_case(rng, shape, dtype, kind)
        N = 5 if trial % 3 else 2
        g_out, cnt, st, _ = oracle.correct(f, g, xi, n_steps=N, mode=mode)
        converged += _check_certificates(f, g, xi, g_out, cnt, st, N, mode)
        # visiting vertices in another order changes nothing (Jacobi rounds)
        g2, c2, st2, _ = oracle.correct(f, g, xi, n_steps=N, mode=mode, shuffle_seed=99 + trial)
        assert np.array_equal(g2.view(np.uint8), g_out.view(np.uint8))
        assert np.array_equal(c2, cnt) and st2 == st
    assert converged >= 6


def test_original_mode_can_change_a_split_pair(golden):
    gd = golden("original_mode_split_pair_2d.txt")
    f = np.array([float(v) for v in gd["f"]], np.float64).reshape(4, 5)
    g = np.array([float(v) for v in gd["g_hat"]], np.float64).reshape(4, 5)
    xi, N = float(gd["xi"][0]), int(gd["n_steps"][0])
    cx = ck.Complex([5, 4])
    ref = ck.topology_signature(cx, f.ravel())
    g1, _, st1, _ = oracle.correct(f, g, xi, n_steps=N, mode=oracle.ORIGINAL)
    assert st1["status"] == oracle.OK and not oracle.targets(f, g1, oracle.ORIGINAL).any()
    s1 = ck.topology_signature(cx, g1.ravel())
    assert s1["critical"] == ref["critical"] and s1["eg"] == ref["eg"]
    assert s1["split_pairs"] != ref["split_pairs"]
    g0, _, st0, _ = oracle.correct(f, g, xi, n_steps=N, mode=oracle.REFORMULATED)
    assert st0["status"] == oracle.OK
    assert ck.topology_signature(cx, g0.ravel()) == ref


def test_no_error_no_edit():
    rng = np.random.default_rng(5)
    f = rng.standard_normal((6, 7, 5)).astype(np.float32)
    g_out, cnt, st, _ = oracle.correct(f, f.copy(), 0.1)
    assert st["iterations"] == 0 and st["status"] == oracle.OK
    assert np.array_equal(g_out, f) and not cnt.any()


def test_uniform_shift_keeps_order():
    # g_hat = f - c with dyadic values keeps every comparison: no edit.
    rng = np.random.default_rng(6)
    f = rng.integers(0, 64, size=(5, 6, 7)).astype(np.float32) / 4
    g_out, cnt, st, _ = oracle.correct(f, f - np.float32(0.5), 0.5)
    assert st["iterations"] == 0 and not cnt.any()


@pytest.mark.parametrize("mode", [oracle.REFORMULATED, oracle.ORIGINAL])
def test_resume_is_identical(mode):
    rng = np.random.default_rng(8)
    f, g, xi = _rand_case(rng, (6, 5, 4), np.float32, "plateau")
    g_full, c_full, st_full, _ = oracle.correct(f, g, xi, mode=mode)
    assert st_full["iterations"] >= 3
    k = st_full["iterations"] // 2
    g_half, c_half, st_half, _ = oracle.correct(f, g, xi, mode=mode, max_iters=k)
    assert st_half["status"] == oracle.MAX_ITERS and st_half["iterations"] == k
    g_res, c_res, st_res, _ = oracle.correct(f, g_half, xi, mode=mode, cnt=c_half)
    assert np.array_equal(g_res, g_full) and np.array_equal(c_res, c_full)
    assert st_half["iterations"] + st_res["iterations"] == st_full["iterations"]
    assert st_half["edit_ops"] + st_res["edit_ops"] == st_full["edit_ops"]


def test_validation_errors():
    f = np.zeros(8, np.float32)
    g = f.copy()
    assert oracle.correct(f, g, 0.0)[2]["status"] == oracle.E_INVALID
    assert oracle.correct(f, g, float("nan"))[2]["status"] == oracle.E_INVALID
    assert oracle.correct(f, g, 0.1, n_steps=0)[2]["status"] == oracle.E_INVALID
    bad = g.copy()
    bad[3] = np.nan
    assert oracle.correct(f, bad, 0.1)[2]["status"] == oracle.E_NONFINITE
    out = g.copy()
    out[2] = np.float32(0.25)
    assert oracle.correct(f, out, 0.125)[2]["status"] == oracle.E_BOUND
    # exactly on the band edge is fine
    edge = g.copy()
    edge[2] = np.float32(0.125)
    assert oracle.correct(f, edge, 0.125)[2]["status"] == oracle.OK


def test_trace_counts():
    rng = np.random.default_rng(9)
    f, g, xi = _rand_case(rng, (6, 6), np.float64, "plateau")
    g_out, cnt, st, tr = oracle.correct(f, g, xi, trace_cap=100)
    assert tr.shape[0] == st["iterations"]
    assert int(tr[:, 1].sum()) == st["edit_ops"]
    assert np.all(tr[:, 1] <= tr[:, 0])
