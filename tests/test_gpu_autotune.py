"""Autotuner on the GPU: a quick tuning run stores an entry, every candidate
reproduced the same result (the tuner checks it), and a tuned context
corrects a field of that class exactly as the default one does."""
import numpy as np
import pytest

from paper_2604_01397_amd import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def test_tune_then_correct(tmp_path):
    from paper_2604_01397_amd import autotune, exactz
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cache = str(tmp_path / "tune.json")
    c = synth.case_grf3d(40, seed=51, rel=1e-3)
    f = torch.from_numpy(c.f).cuda()
    g = torch.from_numpy(c.g_hat).cuda()
    ctx = exactz.Context(0)
    try:
        print("tuning", c.name, flush=True)
        entry = autotune.tune(ctx, f, g, c.xi, quick=True, cache=cache, log=print)
        assert entry["candidates"] == len(autotune.search_space(3, quick=True))
        assert autotune.options_for(autotune.device_arch(0), 3, "f32", f.numel(), cache)
        ref, cref, rref = ctx.correct(f, g, c.xi)
    finally:
        ctx.close()
    tc = autotune.TunedContext(0, cache=cache)
    try:
        # a different field of the same class
        c2 = synth.case_grf3d(41, seed=52, rel=1e-3)
        f2, g2 = torch.from_numpy(c2.f).cuda(), torch.from_numpy(c2.g_hat).cuda()
        out, cout, r = tc.correct(f2, g2, c2.xi)
        plain = exactz.Context(0)
        try:
            o2, co2, r2 = plain.correct(f2, g2, c2.xi)
        finally:
            plain.close()
        torch.cuda.synchronize()
        assert torch.equal(out, o2) and torch.equal(cout, co2)
        assert r["iterations"] == r2["iterations"]
    finally:
        tc.close()


def test_tune_batch_then_correct_batch_matches_oracle(tmp_path):
    """A batched tuning run (reduced axes) stores an entry; the tuned batch
    corrects a mix of 1-D, 2-D and 3-D float32 / float64 fields exactly as
    the oracle does."""
    import oracle
    from paper_2604_01397_amd import autotune, exactz
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cache = str(tmp_path / "tune.json")
    cases = [synth.case_grf3d(24, seed=61, rel=1e-3),
             synth.case_grf3d((9, 17, 40), seed=62, rel=1e-3, dtype=np.float64),
             synth.case_gauss2d(70, seed=63, rel=1e-3),
             synth.case_gauss2d(33, seed=64, rel=1e-3, ny=1)]
    items = [{"f": torch.from_numpy(c.f).cuda(), "g_hat": torch.from_numpy(c.g_hat).cuda(),
              "xi": c.xi} for c in cases]
    axes = {"btile3": [0, 804], "btile2": [0, 401], "bgrid_box": [0, 64], "bgrid_apply": [0, 64],
            "bitem": [0, 1]}
    ctx = exactz.Context(0)
    try:
        print("tuning a 4-field batch", flush=True)
        entry = autotune.tune_batch(ctx, items, cache=cache, axes=axes, log=print)
        assert entry["key"] == autotune.batch_key_of(items)
        assert autotune.batch_options_for(entry["key"], cache) is not None
    finally:
        ctx.close()
    tc = autotune.TunedContext(0, cache=cache)
    try:
        out = tc.correct_batch(items)
        torch.cuda.synchronize()
    finally:
        tc.close()
    for c, (g_out, cnt, res) in zip(cases, out):
        ro, rc, st, _ = oracle.correct(c.f, c.g_hat, c.xi)
        assert np.array_equal(g_out.cpu().numpy().view(np.uint8), ro.view(np.uint8)), c.name
        assert np.array_equal(cnt.cpu().numpy(), rc), c.name
        assert res["iterations"] == st["iterations"] and res["status"] == st["status"], c.name
