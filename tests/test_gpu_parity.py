"""GPU parity: the HIP library against the CPU oracle, element by element.

Integer outputs (edit counts, iteration counts, statuses, target sets) and
the corrected values themselves must be bit-identical: the method is a
discrete ordering problem with exact IEEE arithmetic on both sides, so the
tolerance is zero.
"""
import numpy as np
import pytest

import oracle
from paper_2604_01397_amd import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_01397_amd import exactz
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = exactz.Context(0)
    yield c
    c.close()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint32 if a.dtype == np.float32 else np.uint64)


def _compare(ctx, f, g, xi, label, n_steps=5, max_iters=0, cnt=None):
    print("case:", label, f.shape, f.dtype, "xi=%r" % xi, "N=%d" % n_steps,
          "max_iters=%d" % max_iters, flush=True)
    fo, go = _dev(f), _dev(g)
    c_in = _dev(cnt) if cnt is not None else None
    g_out, c_out, res = ctx.correct(fo, go, xi, n_steps=n_steps, max_iters=max_iters,
                                    cnt=c_in, resume=cnt is not None)
    torch.cuda.synchronize()
    ro, rc, st, _ = oracle.correct(f, g, xi, n_steps=n_steps, max_iters=max_iters, cnt=cnt)
    assert res["status"] == st["status"], (res, st)
    assert np.array_equal(_bits(g_out.cpu().numpy()), _bits(ro)), label
    assert np.array_equal(c_out.cpu().numpy(), rc), label
    for k in ("iterations", "edited_vertices", "edit_ops", "lossless_vertices",
              "floor_vertices", "residual_violations", "num_critical"):
        assert res[k] == st[k], (k, res[k], st[k])
    return res, st


def _rand_case(rng, shape, dtype, kind):
    n = int(np.prod(shape))
    if kind == "plateau":
        f = rng.integers(0, 7, size=n).astype(dtype)
        xi = 2.0
        g = f + rng.integers(-8, 9, size=n).astype(dtype) / dtype(4.0)
    else:
        f = rng.standard_normal(n).astype(dtype)
        xi = float(dtype(0.3))
        g = (f.astype(np.float64) + rng.uniform(-0.29, 0.29, n)).astype(dtype)
    shp = tuple(reversed(shape))
    return f.reshape(shp), g.reshape(shp).astype(dtype), xi


def test_bounds_match_oracle(ctx):
    rng = np.random.default_rng(1)
    for dtype in (np.float32, np.float64):
        tiny = np.finfo(dtype).tiny
        vals = np.concatenate([
            rng.standard_normal(4000) * 10.0 ** rng.integers(-8, 8, 4000),
            [0.0, -0.0, tiny, -tiny, tiny / 8, -tiny / 8, 1e-8, 5e-9, 1.0, -1.0,
             np.finfo(dtype).max / 2, -np.finfo(dtype).max, np.finfo(dtype).max],
        ]).astype(dtype)
        for xi in (1e-3, 0.3, 1.0, 1.0 / 3.0, 1e-30, 1e30):
            print("bounds", dtype.__name__, xi, flush=True)
            L, U = ctx.debug_bounds(_dev(vals), xi)
            Lr, Ur, _, _ = oracle.bounds(vals, xi)
            assert np.array_equal(_bits(L.cpu().numpy()), _bits(Lr))
            # the upper bound can differ only in the sign of a zero
            assert np.array_equal(U.cpu().numpy(), Ur)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape", [(1,), (2,), (9,), (130,), (5, 4), (67, 3), (3, 70),
                                   (4, 4, 3), (3, 3, 3), (65, 3, 2), (2, 9, 17), (1, 1, 5)])
def test_tiny_fields_bit_exact(ctx, shape, dtype):
    rng = np.random.default_rng(abs(hash((shape, dtype.__name__))) % 2 ** 32)
    for trial in range(6):
        f, g, xi = _rand_case(rng, shape, dtype, "plateau" if trial % 2 == 0 else "real")
        _compare(ctx, f, g, xi, "tiny %s trial %d" % (shape, trial), n_steps=5 if trial % 3 else 2)


def test_worked_examples(ctx, golden):
    for name in ("cascade_1d.txt", "edit_minimum_1d.txt", "floor_collapse_1d.txt"):
        gd = golden(name)
        dt = np.dtype(gd["dtype"][0]).type
        f = np.array([float(v) for v in gd["f"]], dt)
        g = np.array([float(v) for v in gd["g_hat"]], dt)
        res, _ = _compare(ctx, f, g, float(gd["xi"][0]), name, n_steps=int(gd["n_steps"][0]))
        assert res["iterations"] == int(gd["iterations"][0])


def test_gauss2d_256_bit_exact(ctx):
    c = synth.config0()
    res, st = _compare(ctx, c.f, c.g_hat, c.xi, c.name)
    assert res["iterations"] > 5


@pytest.mark.parametrize("k", [1, 2, 3, 7])
def test_per_iteration_states(ctx, k):
    c = synth.config0()
    res, _ = _compare(ctx, c.f, c.g_hat, c.xi, c.name, max_iters=k)
    assert res["status"] == 2 and res["iterations"] == k


def test_iteration0_target_set(ctx):
    for c in (synth.config0(), synth.case_grf3d(40, seed=9, rel=1e-3)):
        print("targets:", c.name, flush=True)
        mark, count = ctx.debug_targets(_dev(c.f), _dev(c.g_hat), c.xi)
        ref = oracle.targets(c.f, c.g_hat)
        assert count == int(ref.sum())
        assert np.array_equal(mark.cpu().numpy(), ref)


def test_resume_matches(ctx):
    c = synth.case_gauss2d(80, seed=4, rel=1e-3)
    f, g = _dev(c.f), _dev(c.g_hat)
    full, cfull, rfull = ctx.correct(f, g, c.xi)
    half, chalf, rhalf = ctx.correct(f, g, c.xi, max_iters=3)
    rest, crest, rrest = ctx.correct(f, half.clone(), c.xi, cnt=chalf.clone(), resume=True)
    torch.cuda.synchronize()
    assert rhalf["status"] == 2
    assert torch.equal(rest, full) and torch.equal(crest, cfull)
    assert rhalf["iterations"] + rrest["iterations"] == rfull["iterations"]


def test_in_place(ctx):
    c = synth.case_gauss2d(70, seed=5, rel=1e-3)
    f, g = _dev(c.f), _dev(c.g_hat)
    ref, cref, _ = ctx.correct(f, g, c.xi)
    g2 = g.clone()
    out, cout, _ = ctx.correct(f, g2, c.xi, g_out=g2)
    torch.cuda.synchronize()
    assert out.data_ptr() == g2.data_ptr()
    assert torch.equal(out, ref) and torch.equal(cout, cref)


def test_error_statuses(ctx):
    from paper_2604_01397_amd import exactz
    f = np.zeros((8, 9), np.float32)
    g = f.copy()
    g[3, 3] = np.nan
    _, _, r = ctx.correct(_dev(f), _dev(g), 0.1, raise_on_error=False)
    assert r["status"] == exactz.E_NONFINITE
    g = f.copy()
    g[2, 5] = np.float32(0.25)
    _, _, r = ctx.correct(_dev(f), _dev(g), 0.125, raise_on_error=False)
    assert r["status"] == exactz.E_BOUND
    g[2, 5] = np.float32(0.125)
    _, _, r = ctx.correct(_dev(f), _dev(g), 0.125, raise_on_error=False)
    assert r["status"] == exactz.OK
    _, _, r = ctx.correct(_dev(f), _dev(f), -1.0, raise_on_error=False)
    assert r["status"] == exactz.E_INVALID
    with pytest.raises(exactz.ExactzError):
        ctx.correct(_dev(f), _dev(f), 0.1, n_steps=0)


BOX_SHAPES = [(1, 1), (2, 2), (4, 1), (4, 2), (4, 4), (8, 1), (8, 2), (4, 8), (16, 1), (16, 2)]


@pytest.mark.parametrize("tile_y,tile_z", BOX_SHAPES)
def test_tile_shape_invariance(ctx, tile_y, tile_z):
    c = synth.case_grf3d((37, 45, 70), seed=6, rel=1e-3)
    f, g = _dev(c.f), _dev(c.g_hat)
    ref, cref, rref = ctx.correct(f, g, c.xi)
    ctx.set_option("tile", tile_y * 100 + tile_z)
    try:
        out, cout, r = ctx.correct(f, g, c.xi)
    finally:
        ctx.set_option("tile", 0)
    torch.cuda.synchronize()
    assert torch.equal(out, ref) and torch.equal(cout, cref)
    assert r["iterations"] == rref["iterations"]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_one_group_per_box_large_grid(ctx, dtype):
    """One work-group per box on a field of 2^26 vertices (box 64 x 8 x 4:
    32768 work-groups, whose grid strides over the critical-point ranks
    pass 2^32 within 64 steps) gives the persistent grid's result, through
    the dense and the frontier passes."""
    c = synth.case_grf3d((512, 512, 256), seed=41, slope=-11.0 / 3.0, rel=1e-4, dtype=dtype,
                         quantizer="lorenzo")
    print("case: 512x512x256", np.dtype(dtype).name, "box 8x4, grid 0 vs persistent", flush=True)
    f, g = _dev(c.f), _dev(c.g_hat)
    ref, cref, rref = ctx.correct(f, g, c.xi)
    ctx.set_option("tile", 804)
    ctx.set_option("grid", 0)
    try:
        out, cout, r = ctx.correct(f, g, c.xi)
    finally:
        ctx.set_option("tile", 0)
        ctx.set_option("grid", -1)
    torch.cuda.synchronize()
    assert r["iterations"] == rref["iterations"] and r["iterations"] > 5, (r, rref)
    assert torch.equal(out, ref) and torch.equal(cout, cref)


@pytest.mark.parametrize("poll", [1, 3, 64])
def test_poll_interval_invariance(ctx, poll):
    c = synth.case_gauss2d(100, seed=7, rel=1e-3)
    f, g = _dev(c.f), _dev(c.g_hat)
    ref, cref, rref = ctx.correct(f, g, c.xi)
    ctx.set_option("poll", poll)
    try:
        out, cout, r = ctx.correct(f, g, c.xi)
    finally:
        ctx.set_option("poll", 0)
    torch.cuda.synchronize()
    assert torch.equal(out, ref) and torch.equal(cout, cref) and r == {**r, **{k: rref[k] for k in ("iterations", "edit_ops")}}


def test_grf128_bit_exact(ctx):
    c = synth.config1()
    res, st = _compare(ctx, c.f, c.g_hat, c.xi, c.name)
    print("128^3:", res, flush=True)


def test_unsupported_tile_rejected(ctx):
    from paper_2604_01397_amd import exactz
    with pytest.raises(exactz.ExactzError):
        ctx.set_option("tile", 305)


def test_float64_grf_bit_exact(ctx):
    c = synth.case_grf3d(36, seed=12, rel=1e-4, dtype=np.float64, quantizer="lorenzo")
    _compare(ctx, c.f, c.g_hat, c.xi, c.name)


def test_float64_grf128_bit_exact(ctx):
    """float64 volume at 128^3 (the 8-byte path over the persistent box walk,
    several boxes per work-group, frontier passes)."""
    c = synth.case_grf3d(128, seed=13, slope=-11.0 / 3.0, rel=1e-4, dtype=np.float64,
                         quantizer="lorenzo")
    res, _ = _compare(ctx, c.f, c.g_hat, c.xi, c.name)
    print("128^3 f64:", res, flush=True)


@pytest.mark.parametrize("n_steps", [1, 3, 10, 14])
def test_n_steps_bit_exact(ctx, n_steps):
    """Step counts across the range the boundary accepts (Sec. 3.3: Delta =
    xi_T / N, the (N+1)-th edit lossless)."""
    c = synth.case_grf3d(40, seed=31, slope=-11.0 / 3.0, rel=1e-3, quantizer="lorenzo")
    _compare(ctx, c.f, c.g_hat, c.xi, c.name, n_steps=n_steps)
    d = synth.case_gauss2d(128, seed=32, rel=1e-3)
    _compare(ctx, d.f, d.g_hat, d.xi, d.name, n_steps=n_steps)


def _ramp_cascade(shape, rows):
    """A slow ramp f = -0.2 x - 0.01 y - 0.001 z and g_hat = f except that, in
    the given (y, z) rows, vertex x = 1 is put just below vertex x = 2.  Each
    iteration then moves one vertex of such a row down by Delta = 0.25, which
    puts it below its successor (the cascading effect, Sec. 4.4): about nx
    iterations while the rest of the field stays settled."""
    nx = shape[0]
    ny = shape[1] if len(shape) > 1 else 1
    nz = shape[2] if len(shape) > 2 else 1
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    f = (-0.2 * x - 0.01 * y - 0.001 * z).astype(np.float32)
    g = f.copy()
    for (yy, zz) in rows:
        g[zz, yy, 1] = f[zz, yy, 2] - np.float32(0.05)
    shp = tuple(reversed(shape))
    return f.reshape(shp), g.reshape(shp)


@pytest.mark.parametrize("shape,rows", [((300,), [(0, 0)]),
                                        ((320, 40, 12), [(0, 0), (1, 0), (17, 5), (39, 11)])])
def test_long_cascade_bit_exact(ctx, shape, rows):
    """About 300 iterations, so the per-pass mark tags run through their
    whole cycle (the pass that wipes the marks included), with most boxes
    and chunks idle in every frontier pass."""
    f, g = _ramp_cascade(shape, rows)
    res, _ = _compare(ctx, f, g, 1.25, "ramp cascade", n_steps=5)
    assert res["iterations"] > 254, res


# ----------------------------------------------------------------------------
# original event constraints (integral paths by pointer jumping) and the
# extremum-graph certificate


def _compare_mode(ctx, f, g, xi, label, mode, n_steps=5, max_iters=0):
    print("case:", label, f.shape, f.dtype, "mode=%d" % mode, flush=True)
    g_out, c_out, res = ctx.correct(_dev(f), _dev(g), xi, n_steps=n_steps, mode=mode,
                                    max_iters=max_iters)
    torch.cuda.synchronize()
    ro, rc, st, _ = oracle.correct(f, g, xi, n_steps=n_steps, mode=mode, max_iters=max_iters)
    assert res["status"] == st["status"], (res, st)
    assert np.array_equal(_bits(g_out.cpu().numpy()), _bits(ro)), label
    assert np.array_equal(c_out.cpu().numpy(), rc), label
    for k in ("iterations", "edited_vertices", "edit_ops", "lossless_vertices",
              "floor_vertices", "residual_violations", "num_critical"):
        assert res[k] == st[k], (k, res[k], st[k])
    return res


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("shape", [(9,), (5, 4), (67, 3), (4, 4, 3), (65, 3, 2), (2, 9, 17)])
def test_original_mode_tiny_bit_exact(ctx, shape, dtype):
    rng = np.random.default_rng(abs(hash((shape, dtype.__name__, "orig"))) % 2 ** 32)
    for trial in range(6):
        f, g, xi = _rand_case(rng, shape, dtype, "plateau" if trial % 2 == 0 else "real")
        _compare_mode(ctx, f, g, xi, "orig %s trial %d" % (shape, trial), 1,
                      n_steps=5 if trial % 3 else 2)


def test_original_mode_fields(ctx):
    for c in (synth.config0(), synth.case_grf3d(40, seed=13, rel=1e-3),
              synth.case_grf3d(24, seed=14, rel=1e-2, dtype=np.float64)):
        res = _compare_mode(ctx, c.f, c.g_hat, c.xi, c.name, 1)
        assert res["iterations"] > 0
    c = synth.config0()
    for k in (1, 4):
        _compare_mode(ctx, c.f, c.g_hat, c.xi, c.name, 1, max_iters=k)


def test_original_mode_split_pair_case(ctx, golden):
    gd = golden("original_mode_split_pair_2d.txt")
    f = np.array([float(v) for v in gd["f"]], np.float64).reshape(4, 5)
    g = np.array([float(v) for v in gd["g_hat"]], np.float64).reshape(4, 5)
    _compare_mode(ctx, f, g, float(gd["xi"][0]), "split-pair", 1, n_steps=int(gd["n_steps"][0]))


@pytest.mark.parametrize("name", ["original_mode_join_c2_2d.txt", "original_mode_split_c2_2d.txt",
                                  "original_mode_join_glink_2d.txt",
                                  "original_mode_split_tie_2d.txt"])
def test_original_mode_worked_examples(ctx, golden, name):
    """The hand-built original-mode fixtures (C2 and both sides of C3 named
    in the first iteration) against the fixture's own values and the oracle."""
    gd = golden(name)
    shape = tuple(reversed([int(v) for v in gd["dims"]]))
    f = np.array([float(v) for v in gd["f"]], np.float64).reshape(shape)
    g = np.array([float(v) for v in gd["g_hat"]], np.float64).reshape(shape)
    res = _compare_mode(ctx, f, g, float(gd["xi"][0]), name, 1, n_steps=int(gd["n_steps"][0]))
    assert res["iterations"] == int(gd["iterations"][0])
    g_out, c_out, _ = ctx.correct(_dev(f), _dev(g), float(gd["xi"][0]), mode=1,
                                  n_steps=int(gd["n_steps"][0]))
    torch.cuda.synchronize()
    assert g_out.cpu().numpy().ravel().tolist() == [float(v) for v in gd["g_out"]]
    assert c_out.cpu().numpy().ravel().tolist() == [int(v) for v in gd["cnt"]]


def test_certificate(ctx):
    from paper_2604_01397_amd import exactz
    c = synth.case_grf3d(48, seed=15, rel=1e-3)
    f, g = _dev(c.f), _dev(c.g_hat)
    for mode in (exactz.REFORMULATED, exactz.ORIGINAL):
        _, _, r = ctx.correct(f, g, c.xi, mode=mode, certify=True)
        assert r["status"] in (exactz.OK, exactz.W_STUCK)
        if r["status"] == exactz.OK:
            assert r["certified"] == 1
    # one iteration is not enough here: the certificate must see the damage
    _, _, r = ctx.correct(f, g, c.xi, max_iters=1, certify=True)
    assert r["status"] == exactz.W_MAX_ITERS and r["certified"] == 0
    # without certify the field is left untested
    _, _, r = ctx.correct(f, g, c.xi)
    assert r["certified"] == -1


def _terminus(info, v, key):
    while info[v][key] != v:
        v = info[v][key]
    return v


def _certificate_by_checker(cx, f, h):
    """What the device certificate decides, from the brute-force link analysis
    of oracle/checker.py: every vertex keeps its critical type (minimum,
    maximum, saddle, regular) and the ends of its steepest-descent and
    steepest-ascent paths."""
    from oracle import checker
    fi, gi = checker.classify(cx, f), checker.classify(cx, h)
    for v in range(cx.n):
        if fi[v]["type"] != gi[v]["type"]:
            return 0
        for key in ("desc", "asc"):
            if _terminus(fi, v, key) != _terminus(gi, v, key):
                return 0
    return 1


@pytest.mark.parametrize("shape,seed", [((23, 19), 51), ((7, 8, 9), 52), ((6, 5, 11), 53)])
def test_certificate_matches_checker(ctx, shape, seed):
    """The device certificate against the checker on the same g', after one,
    two, three passes and at the fixpoint, in both event modes; where it
    certifies, the extremum graphs (Sec. 4.1) are equal."""
    from oracle import checker
    from paper_2604_01397_amd import exactz
    rng = np.random.default_rng(seed)
    f, g, xi = _rand_case(rng, shape, np.float32, "normal")
    cx = checker.Complex(list(shape))
    seen = set()
    for mode in (exactz.REFORMULATED, exactz.ORIGINAL):
        for max_iters in (1, 2, 3, 0):
            print("case: certificate", shape, "mode", mode, "max_iters", max_iters, flush=True)
            g_out, _, r = ctx.correct(_dev(f), _dev(g), xi, mode=mode, max_iters=max_iters,
                                      certify=True)
            torch.cuda.synchronize()
            h = g_out.cpu().numpy()
            want = _certificate_by_checker(cx, f, h)
            assert r["certified"] == want, (mode, max_iters, r)
            if want:
                assert checker.extremum_graph(cx, f) == checker.extremum_graph(cx, h)
            seen.add(want)
    assert seen == {0, 1}, "the cases should exercise both outcomes"


# ----------------------------------------------------------------------------
# frontier check passes: after the first pass only boxes whose cells changed
# are re-checked; the outcome must not move by a bit


FRONTIER_CASES = [
    ("gauss2d-150", lambda: synth.case_gauss2d(150, seed=21, rel=1e-3)),
    ("grf3d-48-lorenzo", lambda: synth.case_grf3d(48, seed=22, rel=1e-4, quantizer="lorenzo")),
    ("grf3d-(70,33,21)-f64", lambda: synth.case_grf3d((21, 33, 70), seed=23, rel=1e-3,
                                                       dtype=np.float64)),
]


@pytest.mark.parametrize("name,make", FRONTIER_CASES, ids=[c[0] for c in FRONTIER_CASES])
def test_frontier_matches_dense_and_oracle(name, make):
    from paper_2604_01397_amd import exactz
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = make()
    # dense: every pass checks every box; front: the default frontier passes
    dense = exactz.Context(0, profile=1, frontier=0)
    front = exactz.Context(0, profile=1, frontier=1)
    try:
        f, g = _dev(c.f), _dev(c.g_hat)
        print("case:", name, "dense", flush=True)
        gd, cd, rd = dense.correct(f, g, c.xi)
        print("case:", name, "frontier", flush=True)
        gf, cf, rf = front.correct(f, g, c.xi)
        torch.cuda.synchronize()
        assert torch.equal(gd, gf) and torch.equal(cd, cf)
        for k in ("status", "iterations", "edited_vertices", "edit_ops", "lossless_vertices",
                  "floor_vertices", "residual_violations", "num_critical"):
            assert rd[k] == rf[k], (k, rd[k], rf[k])
        n = c.f.size
        passes = rd["iterations"] + (rd["status"] != exactz.W_MAX_ITERS)
        assert rd["check_vertices"] == passes * n
        print("checked vertices: dense %d frontier %d" % (
            rd["check_vertices"], rf["check_vertices"]), flush=True)
        ro, rc, st, _ = oracle.correct(c.f, c.g_hat, c.xi)
        assert rf["status"] == st["status"] and rf["residual_violations"] == st["residual_violations"]
        assert np.array_equal(_bits(gf.cpu().numpy()), _bits(ro))
        assert np.array_equal(cf.cpu().numpy(), rc)
    finally:
        dense.close()
        front.close()


def test_frontier_checks_fewer_vertices():
    """On a field large enough for boxes to go quiet, frontier passes check
    fewer vertices than dense ones (same results)."""
    from paper_2604_01397_amd import exactz
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = synth.config1()
    f, g = _dev(c.f), _dev(c.g_hat)
    out = {}
    for fr in (0, 1):
        cx = exactz.Context(0, profile=1, frontier=fr)
        try:
            out[fr] = cx.correct(f, g, c.xi)
        finally:
            cx.close()
    torch.cuda.synchronize()
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    r0, r1 = out[0][2], out[1][2]
    print("checked vertices: dense %d frontier %d, iterations %d" % (
        r0["check_vertices"], r1["check_vertices"], r0["iterations"]), flush=True)
    assert r1["check_vertices"] < r0["check_vertices"]


@pytest.mark.parametrize("tile", [101, 202, 801, 1602])
def test_frontier_box_shapes(ctx, tile):
    c = synth.case_grf3d((33, 19, 130), seed=24, rel=1e-3)
    f, g = _dev(c.f), _dev(c.g_hat)
    ctx.set_option("frontier", 0)
    try:
        ref, cref, rref = ctx.correct(f, g, c.xi)
    finally:
        ctx.set_option("frontier", 1)
    ctx.set_option("tile", tile)
    try:
        out, cout, r = ctx.correct(f, g, c.xi)
    finally:
        ctx.set_option("tile", 0)
    torch.cuda.synchronize()
    assert torch.equal(out, ref) and torch.equal(cout, cref)
    assert (r["iterations"], r["status"], r["residual_violations"]) == (
        rref["iterations"], rref["status"], rref["residual_violations"])


def test_unaligned_buffers_match(ctx):
    """Buffers that are not 16-byte aligned take the apply's scalar loads;
    the result must not change."""
    for dtype in (np.float32, np.float64):
        c = synth.case_grf3d((23, 30, 41), seed=41, rel=1e-3, dtype=dtype)
        f, g = _dev(c.f), _dev(c.g_hat)
        ref, cref, rref = ctx.correct(f, g, c.xi)
        n = c.f.size
        fb = torch.empty(n + 1, dtype=f.dtype, device="cuda")
        gb = torch.empty(n + 1, dtype=f.dtype, device="cuda")
        ob = torch.empty(n + 1, dtype=f.dtype, device="cuda")
        cb = torch.zeros(n + 1, dtype=torch.uint8, device="cuda")
        fu, gu = fb[1:].view(f.shape), gb[1:].view(f.shape)
        ou, cu = ob[1:].view(f.shape), cb[1:].view(f.shape)
        fu.copy_(f)
        gu.copy_(g)
        assert fu.data_ptr() % 16 != 0
        out, cout, r = ctx.correct(fu, gu, c.xi, g_out=ou, cnt=cu)
        torch.cuda.synchronize()
        assert torch.equal(out, ref) and torch.equal(cout, cref)
        assert r["iterations"] == rref["iterations"] and r["status"] == rref["status"]


# ----------------------------------------------------------------------------
# frontier passes (boxes flagged by the last apply, including the box of the
# previous critical point of every moved vertex) against dense passes, for
# every box shape and for runs cut short by the iteration cap


@pytest.mark.parametrize("tile", [0, 202, 404, 408, 804, 1602, 101, 401])
def test_frontier_matches_dense_per_box(ctx, tile):
    cases = [synth.case_grf3d((29, 35, 70), seed=61, rel=1e-3),
             synth.case_grf3d(40, seed=62, rel=1e-4, quantizer="lorenzo"),
             synth.case_gauss2d(140, seed=63, rel=1e-3, dtype=np.float64)]
    ctx.set_option("tile", tile)
    try:
        for c in cases:
            f, g = _dev(c.f), _dev(c.g_hat)
            print("case:", c.name, "tile", tile, flush=True)
            ctx.set_option("frontier", 0)
            ref, cref, rref = ctx.correct(f, g, c.xi)
            ctx.set_option("frontier", 1)
            out, cout, r = ctx.correct(f, g, c.xi)
            torch.cuda.synchronize()
            assert torch.equal(out, ref) and torch.equal(cout, cref), c.name
            for k in ("status", "iterations", "edited_vertices", "edit_ops", "lossless_vertices",
                      "floor_vertices", "residual_violations"):
                assert r[k] == rref[k], (c.name, k, r[k], rref[k])
            for mi in (1, 2, 5):
                o1, c1, r1 = ctx.correct(f, g, c.xi, max_iters=mi)
                ctx.set_option("frontier", 0)
                o0, c0, r0 = ctx.correct(f, g, c.xi, max_iters=mi)
                ctx.set_option("frontier", 1)
                torch.cuda.synchronize()
                assert torch.equal(o1, o0) and torch.equal(c1, c0), (c.name, mi)
                assert (r1["status"], r1["iterations"]) == (r0["status"], r0["iterations"])
    finally:
        ctx.set_option("tile", 0)
        ctx.set_option("frontier", 1)
