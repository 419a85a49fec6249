"""The rest of the C boundary on the GPU: the host-pointer entry point and
the context's HBM budget (admission by footprint)."""
import numpy as np
import pytest

import oracle
from paper_2604_01397_amd import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint32 if a.dtype == np.float32 else np.uint64)


def test_correct_host_matches_device_and_oracle():
    from paper_2604_01397_amd import exactz
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = exactz.Context(0)
    try:
        for c in (synth.case_gauss2d(120, seed=51, rel=1e-3),
                  synth.case_grf3d((30, 41, 66), seed=52, rel=1e-3, dtype=np.float64)):
            print("case:", c.name, flush=True)
            g_h, c_h, r_h = ctx.correct_host(c.f, c.g_hat, c.xi)
            f = torch.from_numpy(np.ascontiguousarray(c.f)).cuda()
            g = torch.from_numpy(np.ascontiguousarray(c.g_hat)).cuda()
            g_d, c_d, r_d = ctx.correct(f, g, c.xi)
            torch.cuda.synchronize()
            assert np.array_equal(_bits(g_h), _bits(g_d.cpu().numpy()))
            assert np.array_equal(c_h, c_d.cpu().numpy())
            go, co, st, _ = oracle.correct(c.f, c.g_hat, c.xi)
            assert np.array_equal(_bits(g_h), _bits(go)) and np.array_equal(c_h, co)
            assert r_h["iterations"] == st["iterations"] and r_h["status"] == st["status"]
        # resume from host counts
        c = synth.case_gauss2d(80, seed=53, rel=1e-3)
        half, ch, rh = ctx.correct_host(c.f, c.g_hat, c.xi, max_iters=2)
        rest, cr, rr = ctx.correct_host(c.f, half, c.xi, cnt=ch, resume=True)
        full, cf, rf = ctx.correct_host(c.f, c.g_hat, c.xi)
        assert rh["status"] == exactz.W_MAX_ITERS
        assert np.array_equal(rest, full) and np.array_equal(cr, cf)
        # errors come back as statuses, the output untouched
        bad = c.g_hat.copy()
        bad[3, 3] = np.nan
        _, _, r = ctx.correct_host(c.f, bad, c.xi, raise_on_error=False)
        assert r["status"] == exactz.E_NONFINITE
    finally:
        ctx.close()


def test_context_budget():
    from paper_2604_01397_amd import exactz
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    small = synth.case_gauss2d(64, seed=54, rel=1e-3)
    big = synth.case_grf3d(96, seed=55, rel=1e-3)
    need_big = exactz.workspace_bytes(tuple(reversed(big.f.shape)))
    budget = 8 << 20
    assert need_big > budget  # the big field cannot fit, the small one can
    ctx = exactz.Context(0, budget=budget)
    free = exactz.Context(0)
    try:
        fs = torch.from_numpy(small.f).cuda()
        gs = torch.from_numpy(small.g_hat).cuda()
        ref, cref, _ = free.correct(fs, gs, small.xi)
        out, cout, _ = ctx.correct(fs, gs, small.xi)
        torch.cuda.synchronize()
        assert torch.equal(out, ref) and torch.equal(cout, cref)
        used = ctx.bytes_in_use()
        print("in use after the small field:", used, flush=True)
        assert 0 < used <= budget
        fb = torch.from_numpy(big.f).cuda()
        gb = torch.from_numpy(big.g_hat).cuda()
        with pytest.raises(exactz.ExactzError) as e:
            ctx.correct(fb, gb, big.xi)
        assert e.value.status == exactz.E_NOMEM
        assert ctx.bytes_in_use() <= budget
        # the context still works, and jobs are admitted by the same budget
        out2, _, _ = ctx.correct(fs, gs, small.xi)
        torch.cuda.synchronize()
        assert torch.equal(out2, ref)
        with pytest.raises(exactz.ExactzError) as e:
            ctx.job_create(fb, gb, big.xi)
        assert e.value.status == exactz.E_NOMEM
        before = ctx.bytes_in_use()
        job = ctx.job_create(fs, gs.clone(), small.xi)
        assert ctx.bytes_in_use() > before
        for _ in range(100):
            ctx.step([job], 4)
            if job.poll()[0]:
                break
        assert torch.equal(job.g_out, ref)
        job.release()
        # the released workspace is pooled for later jobs (still counted),
        # and trimming the pool gives it back
        assert ctx.bytes_in_use() <= budget
        ctx.set_option("trim", 1)
        assert ctx.bytes_in_use() == before
    finally:
        ctx.close()
        free.close()


def test_workspace_bytes_k_prices_a_job():
    """exz_workspace_bytes_k with a job's real number of critical points is
    what the job's set-up reserves: a job's two reservations are exact, and
    the counts live in the caller's buffer here (the binding always passes
    one), so the job holds the priced bytes less those n."""
    from paper_2604_01397_amd import exactz
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = exactz.Context(0)
    try:
        c = synth.case_grf3d(48, seed=71, rel=1e-3)
        f = torch.from_numpy(c.f).cuda()
        g = torch.from_numpy(c.g_hat).cuda()
        before = ctx.bytes_in_use()
        job = ctx.job_create(f, g.clone(), c.xi)
        delta = ctx.bytes_in_use() - before
        _, r = job.poll()
        k = r["num_critical"]
        print("job reserved", delta, "bytes, K =", k, flush=True)
        want = exactz.workspace_bytes((48, 48, 48), num_critical=k)
        assert 0 < k < 48 ** 3
        n = 48 ** 3
        assert want - n - 2 * 256 <= delta <= want - n + 2 * 256, (want, delta)
        assert want < exactz.workspace_bytes((48, 48, 48))  # the worst case (K = n)
        job.release()
    finally:
        ctx.close()
