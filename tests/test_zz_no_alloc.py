"""exz_correct_noalloc (the entry point that allocates nothing) against
exz_correct, through the C ABI: two calls in a row, the second on a smaller
field, must each equal the allocating entry point bit for bit."""
import numpy as np
import pytest

from paper_2604_01397_amd import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

KEYS = ("iterations", "edited_vertices", "edit_ops", "lossless_vertices", "floor_vertices",
        "residual_violations", "num_critical", "status", "certified")


def _same(a, b, label):
    ga, ca, ra = a
    gb, cb, rb = b
    torch.cuda.synchronize()
    assert torch.equal(ga, gb) and torch.equal(ca, cb), label
    for k in KEYS:
        assert ra[k] == rb[k], (label, k, ra[k], rb[k])


def test_noalloc_matches_correct_twice_then_smaller():
    from paper_2604_01397_amd import exactz
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = exactz.Context(0)
    try:
        big = synth.case_grf3d(96, seed=71, rel=1e-3)
        small = synth.case_gauss2d(90, seed=72, rel=1e-3, dtype=np.float64, ny=57)
        runs = [(big, {}), (small, {}), (big, {"mode": exactz.ORIGINAL}),
                (synth.case_grf3d(40, seed=73, rel=1e-3), {"certify": True}),
                (small, {"max_iters": 3})]
        for c, kw in runs:
            print("case:", c.name, kw, flush=True)
            f = torch.from_numpy(np.ascontiguousarray(c.f)).cuda()
            g = torch.from_numpy(np.ascontiguousarray(c.g_hat)).cuda()
            ref = ctx.correct(f, g, c.xi, **kw)
            got = ctx.correct_noalloc(f, g, c.xi, **kw)
            _same(ref, got, c.name)
        # in place, from the state of an earlier call (resume)
        c = small
        f = torch.from_numpy(np.ascontiguousarray(c.f)).cuda()
        g = torch.from_numpy(np.ascontiguousarray(c.g_hat)).cuda()
        half, ch, _ = ctx.correct_noalloc(f, g, c.xi, max_iters=2)
        g2 = half.clone()
        rest = ctx.correct_noalloc(f, g2, c.xi, g_out=g2, cnt=ch.clone(), resume=True)
        full = ctx.correct(f, g, c.xi)
        torch.cuda.synchronize()
        assert torch.equal(rest[0], full[0]) and torch.equal(rest[1], full[1])
    finally:
        ctx.close()


def test_noalloc_rejects_fields_beyond_its_buffer():
    from paper_2604_01397_amd import exactz
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = exactz.Context(0)
    try:
        # 512 x 512 x 128 needs about 7 bytes per vertex of per-vertex
        # workspace (235 MB): refused before any work is issued
        f = torch.zeros((128, 512, 512), dtype=torch.float32, device="cuda")
        with pytest.raises(exactz.ExactzError) as e:
            ctx.correct_noalloc(f, f.clone(), 0.1)
        assert e.value.status == exactz.E_NOMEM
        assert "static buffer" in ctx.last_error()
        # white noise: many critical points; either their workspace does not
        # fit (refused once K is known) or the result equals exz_correct
        rng = np.random.default_rng(74)
        fn = rng.standard_normal((192, 192, 192)).astype(np.float32)
        gn = (fn.astype(np.float64) + rng.uniform(-0.09, 0.09, fn.shape)).astype(np.float32)
        fd, gd = torch.from_numpy(fn).cuda(), torch.from_numpy(gn).cuda()
        _, _, r = ctx.correct_noalloc(fd, gd, 0.1, raise_on_error=False)
        print("white noise 192^3:", r["status"], ctx.last_error(), flush=True)
        if r["status"] == exactz.E_NOMEM:
            assert "critical-point workspace" in ctx.last_error()
        else:
            ref = ctx.correct(fd, gd, 0.1)
            got = ctx.correct_noalloc(fd, gd, 0.1)
            _same(ref, got, "white noise")
        # and the entry point still works afterwards
        c = synth.case_gauss2d(64, seed=75, rel=1e-3)
        f = torch.from_numpy(c.f).cuda()
        g = torch.from_numpy(c.g_hat).cuda()
        _same(ctx.correct(f, g, c.xi), ctx.correct_noalloc(f, g, c.xi), c.name)
    finally:
        ctx.close()
