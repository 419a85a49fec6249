"""Batched correction: every field's result in a batch equals its plain
result bit for bit (and the CPU oracle's for the small fields)."""
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


def _mixed_cases():
    cases = [
        synth.case_gauss2d(96, seed=21, rel=1e-3),
        synth.case_gauss2d(150, seed=22, rel=1e-2, dtype=np.float64, ny=77),
        synth.case_grf3d(32, seed=23, rel=1e-3),
        synth.case_grf3d((20, 33, 41), seed=24, rel=1e-4, dtype=np.float64),
        synth.case_grf3d(28, seed=25, rel=1e-2, quantizer="lorenzo"),
        synth.case_gauss2d(64, seed=26, rel=1e-4),
    ]
    rng = np.random.default_rng(27)
    f = rng.integers(0, 7, size=(6, 5, 4)).astype(np.float32)
    g = f + rng.integers(-8, 9, size=f.shape).astype(np.float32) / np.float32(4)
    cases.append(synth.Case("plateau3d", f, g, 2.0))
    f1 = rng.standard_normal(257).astype(np.float32)
    g1 = (f1.astype(np.float64) + rng.uniform(-0.29, 0.29, f1.size)).astype(np.float32)
    cases.append(synth.Case("line1d", f1, g1, float(np.float32(0.3))))
    return cases


def test_batch_equals_plain_and_oracle(ctx):
    cases = _mixed_cases()
    items = [{"f": _dev(c.f), "g_hat": _dev(c.g_hat), "xi": c.xi} for c in cases]
    print("batch of", len(items), flush=True)
    out = ctx.correct_batch(items)
    torch.cuda.synchronize()
    for c, it, (g_out, cnt, r) in zip(cases, items, out):
        print("field", c.name, r["iterations"], r["status"], flush=True)
        g1, c1, r1 = ctx.correct(it["f"], it["g_hat"], c.xi)
        torch.cuda.synchronize()
        assert torch.equal(g_out, g1) and torch.equal(cnt, c1), c.name
        for k in ("iterations", "edited_vertices", "edit_ops", "lossless_vertices",
                  "floor_vertices", "residual_violations", "num_critical", "status"):
            assert r[k] == r1[k], (c.name, k)
        go, co, st, _ = oracle.correct(c.f, c.g_hat, c.xi)
        assert np.array_equal(_bits(g_out.cpu().numpy()), _bits(go)), c.name
        assert np.array_equal(cnt.cpu().numpy(), co)
        assert r["iterations"] == st["iterations"] and r["status"] == st["status"]


def test_batch_composition_invariance(ctx):
    cases = _mixed_cases()
    items = [{"f": _dev(c.f), "g_hat": _dev(c.g_hat), "xi": c.xi} for c in cases]
    a = ctx.correct_batch(items)
    b = ctx.correct_batch(list(reversed(items)))[::-1]
    c = ctx.correct_batch(items[::2])
    torch.cuda.synchronize()
    for k in range(len(items)):
        assert torch.equal(a[k][0], b[k][0]) and torch.equal(a[k][1], b[k][1])
    for k in range(0, len(items), 2):
        assert torch.equal(a[k][0], c[k // 2][0])


def test_batch_errors_and_modes(ctx):
    from paper_2604_01397_amd import exactz
    good = synth.case_gauss2d(48, seed=28, rel=1e-3)
    bad = np.zeros((8, 9), np.float32)
    badg = bad.copy()
    badg[1, 1] = np.nan
    items = [
        {"f": _dev(good.f), "g_hat": _dev(good.g_hat), "xi": good.xi},
        {"f": _dev(bad), "g_hat": _dev(badg), "xi": 0.1},
        {"f": _dev(good.f), "g_hat": _dev(good.g_hat), "xi": good.xi, "mode": exactz.ORIGINAL},
        {"f": _dev(good.f), "g_hat": _dev(good.g_hat), "xi": good.xi, "max_iters": 2},
        {"f": _dev(good.f), "g_hat": _dev(good.g_hat), "xi": good.xi, "certify": True},
    ]
    out = ctx.correct_batch(items)
    torch.cuda.synchronize()
    assert out[1][2]["status"] == exactz.E_NONFINITE
    ref, cref, rref = ctx.correct(items[0]["f"], items[0]["g_hat"], good.xi)
    orig, corig, rorig = ctx.correct(items[0]["f"], items[0]["g_hat"], good.xi, mode=exactz.ORIGINAL)
    two, ctwo, rtwo = ctx.correct(items[0]["f"], items[0]["g_hat"], good.xi, max_iters=2)
    torch.cuda.synchronize()
    assert torch.equal(out[0][0], ref)
    assert torch.equal(out[2][0], orig) and out[2][2]["iterations"] == rorig["iterations"]
    assert torch.equal(out[3][0], two) and out[3][2]["status"] == exactz.W_MAX_ITERS
    assert torch.equal(out[4][0], ref)
    if out[4][2]["status"] == exactz.OK:
        assert out[4][2]["certified"] == 1


def test_batch_graph_and_poll_invariance(ctx):
    cases = _mixed_cases()[:4]
    items = [{"f": _dev(c.f), "g_hat": _dev(c.g_hat), "xi": c.xi} for c in cases]
    ref = ctx.correct_batch(items)
    for graph, poll in ((0, 0), (1, 1), (1, 5), (0, 3)):
        ctx.set_option("graph", graph)
        ctx.set_option("poll", poll)
        try:
            out = ctx.correct_batch(items)
        finally:
            ctx.set_option("graph", 1)
            ctx.set_option("poll", 0)
        torch.cuda.synchronize()
        for a, b in zip(ref, out):
            assert torch.equal(a[0], b[0]) and a[2]["iterations"] == b[2]["iterations"]


def test_batch_apply_blocks_cross_fields(ctx):
    """With a tiny apply grid and one quad per thread per item, every apply
    work-group walks items of several fields and flushes its edit counts
    once per field: counters and results must still equal the plain runs
    and the oracle."""
    cases = _mixed_cases()
    items = [{"f": _dev(c.f), "g_hat": _dev(c.g_hat), "xi": c.xi} for c in cases]
    ref = ctx.correct_batch(items)
    for grid, item in ((2, 1), (3, 2), (1, 1)):
        ctx.set_option("bgrid_apply", grid)
        ctx.set_option("bitem", item)
        ctx.set_option("bgrid_box", 5)
        try:
            out = ctx.correct_batch(items)
        finally:
            ctx.set_option("bgrid_apply", 0)
            ctx.set_option("bitem", 0)
            ctx.set_option("bgrid_box", 0)
        torch.cuda.synchronize()
        print("apply grid", grid, "item", item, flush=True)
        for c, a, b in zip(cases, ref, out):
            assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), c.name
            for k in ("iterations", "edited_vertices", "edit_ops", "lossless_vertices",
                      "floor_vertices", "residual_violations", "status"):
                assert a[2][k] == b[2][k], (c.name, k)
    for c, (g_out, cnt, r) in zip(cases, ref):
        go, co, st, _ = oracle.correct(c.f, c.g_hat, c.xi)
        assert np.array_equal(_bits(g_out.cpu().numpy()), _bits(go)), c.name
        assert r["edit_ops"] == st["edit_ops"] and r["lossless_vertices"] == st["lossless_vertices"]


def test_batch_box_shapes_invariance(ctx):
    """Batched box shapes and grids chosen by the autotuner never change a
    result."""
    cases = _mixed_cases()
    items = [{"f": _dev(c.f), "g_hat": _dev(c.g_hat), "xi": c.xi} for c in cases]
    ref = ctx.correct_batch(items)
    for b3, b2 in ((202, 401), (804, 801), (404, 101), (1602, 1601)):
        ctx.set_option("btile3", b3)
        ctx.set_option("btile2", b2)
        try:
            out = ctx.correct_batch(items)
        finally:
            ctx.set_option("btile3", 0)
            ctx.set_option("btile2", 0)
        torch.cuda.synchronize()
        for c, a, b in zip(cases, ref, out):
            assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), (c.name, b3, b2)


def test_batch_original_members_in_the_batched_loop(ctx):
    """Original-mode members (Sec. 4.2) run in the batched launches with the
    reformulated ones (their event kernel over per-field items, their path
    workspace set up in the batch): each equals its plain original-mode
    correction and the oracle's, certificates included, and the reformulated
    members are unchanged."""
    from paper_2604_01397_amd import exactz
    cases = _mixed_cases()
    items = []
    for k, c in enumerate(cases):
        mode = exactz.ORIGINAL if k % 2 == 0 else exactz.REFORMULATED
        items.append({"f": _dev(c.f), "g_hat": _dev(c.g_hat), "xi": c.xi, "mode": mode,
                      "certify": k % 3 == 0})
    print("batch of", len(items), "with original-mode members", flush=True)
    out = ctx.correct_batch(items)
    torch.cuda.synchronize()
    for c, it, (g_out, cnt, r) in zip(cases, items, out):
        print("field", c.name, "mode", it["mode"], r["iterations"], r["status"], flush=True)
        g1, c1, r1 = ctx.correct(it["f"], it["g_hat"], c.xi, mode=it["mode"],
                                 certify=it["certify"])
        torch.cuda.synchronize()
        assert torch.equal(g_out, g1) and torch.equal(cnt, c1), c.name
        for k in ("iterations", "edited_vertices", "edit_ops", "num_critical", "status",
                  "certified"):
            assert r[k] == r1[k], (c.name, k, r[k], r1[k])
        go, co, st, _ = oracle.correct(c.f, c.g_hat, c.xi, mode=it["mode"])
        assert np.array_equal(_bits(g_out.cpu().numpy()), _bits(go)), c.name
        assert np.array_equal(cnt.cpu().numpy(), co), c.name
