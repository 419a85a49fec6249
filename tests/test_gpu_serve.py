"""Serving on the GPU: every job's corrected field, edit counts and counters
are the same when it runs alone and when it runs in the mix of a
continuous-batching server (bit for bit)."""
import numpy as np
import pytest

import oracle
from paper_2604_01397_amd import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _cases():
    return [
        synth.case_grf3d(34, seed=31, rel=1e-3),
        synth.case_grf3d((18, 40, 66), seed=32, rel=1e-3),
        synth.case_gauss2d(130, seed=33, rel=1e-3),
        synth.case_grf3d(26, seed=34, rel=1e-2, quantizer="lorenzo"),
        synth.case_grf3d(50, seed=35, rel=1e-3),
        synth.case_gauss2d(64, seed=36, rel=1e-4, dtype=np.float64),
        synth.case_grf3d(20, seed=37, rel=1e-3),
        synth.case_grf3d(42, seed=38, rel=1e-4),
    ]


@pytest.mark.parametrize("tuned,blocking", [(False, False), (True, False), (False, True)])
def test_served_jobs_equal_alone_runs(tuned, blocking, monkeypatch):
    """With tuned=True the executor sets the batched launch options of the
    autotune table's serving entry (here a table that answers every key with
    non-default boxes, grid caps and item size); with blocking=False (the
    default) jobs are submitted and polled without waiting (exz_job_submit,
    exz_job_query), with blocking=True created and polled with waits."""
    from paper_2604_01397_amd import autotune, exactz
    from paper_2604_01397_amd.serve import DeviceExecutor, JobSpec, Server
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if tuned:
        monkeypatch.setattr(autotune, "batch_options_for", lambda key, cache=None: {
            "btile3": 804, "btile2": 401, "bgrid_box": 64, "bgrid_apply": 64, "bitem": 1})
    cases = _cases()
    ctx = exactz.Context(0)
    try:
        specs = []
        for j, c in enumerate(cases):
            def make(stream, c=c):
                f = torch.from_numpy(np.ascontiguousarray(c.f)).cuda()
                g = torch.from_numpy(np.ascontiguousarray(c.g_hat)).cuda()
                return f, g, c.xi
            # all arrive at once, so that the budget (not the timing) decides how
            # many run together
            specs.append(JobSpec(j, 0.0, c.f.shape, c.f.nbytes, make))
        ex = DeviceExecutor(ctx, keep_outputs=True, tuned=tuned, blocking=blocking)
        # a budget of about three jobs: later arrivals wait for memory
        budget = 3 * max(ex.footprint(s) for s in specs)
        print("serving", len(specs), "jobs, budget", budget, flush=True)
        rep = Server(ex, budget, max_active=4, iters_per_step=3, keep_outputs=True).run(specs)
        torch.cuda.synchronize()
        s = rep.summary()
        print(s, flush=True)
        assert s["completed"] == len(cases) and rep.max_active >= 2
        for r, c in zip(rep.records, cases):
            print("job", r.spec.job_id, c.name, r.result["iterations"], flush=True)
            g_srv, c_srv = r.outputs
            f = torch.from_numpy(np.ascontiguousarray(c.f)).cuda()
            g = torch.from_numpy(np.ascontiguousarray(c.g_hat)).cuda()
            g1, c1, r1 = ctx.correct(f, g, c.xi)
            torch.cuda.synchronize()
            assert torch.equal(g_srv, g1) and torch.equal(c_srv, c1), c.name
            for k in ("iterations", "edited_vertices", "edit_ops", "lossless_vertices",
                      "floor_vertices", "residual_violations", "status"):
                assert r.result[k] == r1[k], (c.name, k, r.result[k], r1[k])
        # and one of them against the CPU oracle
        c = cases[3]
        go, co, st, _ = oracle.correct(c.f, c.g_hat, c.xi)
        g_srv, c_srv = rep.records[3].outputs
        assert np.array_equal(g_srv.cpu().numpy().view(np.uint32), go.view(np.uint32))
        assert np.array_equal(c_srv.cpu().numpy(), co)
    finally:
        ctx.close()


def test_job_api_rejects_bad_requests():
    from paper_2604_01397_amd import exactz
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = exactz.Context(0)
    try:
        f = torch.zeros((8, 9), dtype=torch.float32, device="cuda")
        g = f.clone()
        g[2, 3] = 0.5
        with pytest.raises(exactz.ExactzError) as e:
            ctx.job_create(f, g, 0.125)
        assert e.value.status == exactz.E_BOUND
        g[2, 3] = float("nan")
        with pytest.raises(exactz.ExactzError) as e:
            ctx.job_create(f, g, 0.125)
        assert e.value.status == exactz.E_NONFINITE
        job = ctx.job_create(f, f.clone(), 0.125)
        ctx.step([job], 2)
        done, r = job.poll()
        assert done and r["status"] == exactz.OK and r["iterations"] == 0
        job.release()
    finally:
        ctx.close()


def test_job_stepped_at_once_on_another_stream():
    """A job created on one stream and stepped at once on another (no poll in
    between) must wait for its own set-up: the result equals exz_correct."""
    from paper_2604_01397_amd import exactz
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = exactz.Context(0)
    try:
        cases = [synth.case_grf3d(48, seed=41, rel=1e-3), synth.case_grf3d(36, seed=42, rel=1e-3),
                 synth.case_gauss2d(200, seed=43, rel=1e-3)]
        s_create, s_step = torch.cuda.Stream(), torch.cuda.Stream()
        jobs, ins = [], []
        for c in cases:
            with torch.cuda.stream(s_create):
                f = torch.from_numpy(np.ascontiguousarray(c.f)).cuda()
                g = torch.from_numpy(np.ascontiguousarray(c.g_hat)).cuda()
                cnt = torch.zeros(f.shape, dtype=torch.uint8, device="cuda")
                g_out = torch.empty_like(f)
            s_create.synchronize()  # inputs ready; the job set-up itself stays queued
            print("job", c.name, flush=True)
            jobs.append(ctx.job_create(f, g, c.xi, g_out=g_out, cnt=cnt, stream=s_create))
            ins.append((f, g))
        # step all of them on another stream right away, with the 3D jobs
        # in one step and the plane in its own
        for _ in range(200):
            ctx.step(jobs[:2], 2, stream=s_step)
            ctx.step(jobs[2:], 2, stream=s_step)
            if all(j.poll()[0] for j in jobs):
                break
        for c, j, (f, g) in zip(cases, jobs, ins):
            done, r = j.poll()
            assert done
            g1, c1, r1 = ctx.correct(f, g, c.xi)
            torch.cuda.synchronize()
            assert torch.equal(j.g_out, g1) and torch.equal(j.cnt, c1), c.name
            assert r["iterations"] == r1["iterations"] and r["status"] == r1["status"]
            j.release()
    finally:
        ctx.close()


def test_submitted_jobs_and_bad_input_reported_later():
    """exz_job_submit returns before the set-up has run: jobs stepped at once
    on another stream and followed with exz_job_query (which never waits)
    end equal to exz_correct; a field outside the band is reported by the
    query (done, EXZ_E_BOUND) and a step skips it."""
    from paper_2604_01397_amd import exactz
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = exactz.Context(0)
    try:
        cases = [synth.case_grf3d(40, seed=44, rel=1e-3), synth.case_grf3d(30, seed=45, rel=1e-3)]
        s_create, s_step = torch.cuda.Stream(), torch.cuda.Stream()
        jobs, ins = [], []
        for c in cases:
            with torch.cuda.stream(s_create):
                f = torch.from_numpy(np.ascontiguousarray(c.f)).cuda()
                g = torch.from_numpy(np.ascontiguousarray(c.g_hat)).cuda()
            print("submit", c.name, flush=True)
            jobs.append(ctx.job_submit(f, g.clone(), c.xi, stream=s_create))
            ins.append((f, g))
        fb = torch.zeros((8, 9), dtype=torch.float32, device="cuda")
        gb = fb.clone()
        gb[2, 3] = 0.5  # outside [f - xi, f + xi]
        bad = ctx.job_submit(fb, gb, 0.125, stream=s_create)
        done = [False] * len(jobs)
        results = [None] * len(jobs)
        for _ in range(400):
            ctx.step(jobs + [bad], 2, stream=s_step)
            for k, j in enumerate(jobs):
                if not done[k]:
                    done[k], results[k] = j.query()
            if all(done):
                break
        assert all(done)
        with pytest.raises(exactz.ExactzError) as e:
            bad.query()
        assert e.value.status == exactz.E_BOUND
        bad.release()
        s_step.synchronize()
        for c, j, r, (f, g) in zip(cases, jobs, results, ins):
            g1, c1, r1 = ctx.correct(f, g, c.xi)
            torch.cuda.synchronize()
            assert torch.equal(j.g_out, g1) and torch.equal(j.cnt, c1), c.name
            for k in ("iterations", "edited_vertices", "edit_ops", "status"):
                assert r[k] == r1[k], (c.name, k)
            j.release()
    finally:
        ctx.close()


def test_query_sees_completion_while_steps_queue_up():
    """The host runs one step ahead of the device: with the device slowed
    down before every step, the latest two steps are still in flight at each
    query, and exz_job_query must still report the job done (it reads the
    latest step whose work has ended)."""
    from paper_2604_01397_amd import exactz
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = exactz.Context(0)
    try:
        c = synth.case_grf3d(24, seed=46, rel=1e-3)
        f = torch.from_numpy(np.ascontiguousarray(c.f)).cuda()
        g = torch.from_numpy(np.ascontiguousarray(c.g_hat)).cuda()
        s = torch.cuda.Stream()
        job = ctx.job_create(f, g.clone(), c.xi, stream=s)
        done, r, n = False, None, 0
        for n in range(300):
            with torch.cuda.stream(s):
                torch.cuda._sleep(2_000_000)  # a bounded spin: the device falls behind
            ctx.step([job], 1, stream=s)
            done, r = job.query()
            if done:
                break
        print("reported done after", n + 1, "steps", flush=True)
        assert done
        s.synchronize()
        g1, c1, r1 = ctx.correct(f, g, c.xi)
        torch.cuda.synchronize()
        assert torch.equal(job.g_out, g1) and r["iterations"] == r1["iterations"]
        job.release()
    finally:
        ctx.close()


def test_released_job_workspace_is_reused():
    """A released job's workspace goes to the context's pool; the next job
    of the same shape takes it (no new device memory) and its result equals
    exz_correct; "trim" gives the pooled memory back."""
    from paper_2604_01397_amd import exactz
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx, ref = exactz.Context(0), exactz.Context(0)  # jobs; the plain corrections
    try:
        base = ctx.bytes_in_use()
        cases = [synth.case_grf3d(48, seed=51, rel=1e-3), synth.case_grf3d(48, seed=52, rel=1e-3)]
        held = []
        for i, c in enumerate(cases):
            print("job", i, c.name, flush=True)
            f = torch.from_numpy(np.ascontiguousarray(c.f)).cuda()
            g = torch.from_numpy(np.ascontiguousarray(c.g_hat)).cuda()
            job = ctx.job_create(f, g.clone(), c.xi)
            for _ in range(200):
                ctx.step([job], 2)
                if job.poll()[0]:
                    break
            done, r = job.poll()
            assert done
            g1, c1, r1 = ref.correct(f, g, c.xi)
            torch.cuda.synchronize()
            assert torch.equal(job.g_out, g1) and torch.equal(job.cnt, c1)
            assert r["iterations"] == r1["iterations"]
            job.release()
            torch.cuda.synchronize()
            held.append(ctx.bytes_in_use())
            want = exactz.workspace_bytes((48, 48, 48), num_critical=r["num_critical"]) - 48 ** 3
        # the second job took at least the first one's per-vertex block (same
        # size) from the pool, so it allocated less than its whole workspace
        assert held[1] - held[0] < want, (held, want)
        ctx.set_option("trim", 1)
        assert ctx.bytes_in_use() < held[1]
        ctx.set_option("job_pool", 0)  # no pool: a released job frees at once
        assert ctx.bytes_in_use() == base
    finally:
        ctx.close()
        ref.close()
