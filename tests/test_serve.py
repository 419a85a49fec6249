"""Serving loop (host logic) on a simulated executor and a virtual clock:
admission by footprint, first-come-first-served order, continuous batching,
rejection of oversized or failing jobs, latency and throughput bookkeeping."""
import numpy as np
import pytest

from paper_2604_01397_amd.serve import JobSpec, Server


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class SimExecutor:
    """Each job needs `need` iterations; a step costs `per_step` seconds plus
    `per_item` per active job; start costs `setup` seconds."""

    def __init__(self, clock, per_step=1e-3, per_item=1e-4, setup=2e-3, fail_ids=()):
        self.clock = clock
        self.per_step, self.per_item, self.setup = per_step, per_item, setup
        self.fail_ids = set(fail_ids)
        self.used = 0
        self.peak = 0
        self.live = {}
        self.log = []  # (event, job_id, time)

    def footprint(self, spec):
        return spec.meta["bytes"]

    def start(self, spec):
        if spec.job_id in self.fail_ids:
            raise ValueError("bad input")
        self.clock.t += self.setup
        h = {"id": spec.job_id, "need": spec.meta["need"], "done": 0, "bytes": spec.meta["bytes"]}
        self.used += h["bytes"]
        self.peak = max(self.peak, self.used)
        self.live[spec.job_id] = h
        self.log.append(("start", spec.job_id, self.clock.t))
        return h

    def step(self, handles, iters):
        assert handles
        self.clock.t += self.per_step + self.per_item * len(handles)
        for h in handles:
            h["done"] = min(h["need"], h["done"] + iters)

    def poll(self, h):
        done = h["done"] >= h["need"]
        return done, {"iterations": h["done"], "job": h["id"]}

    def finish(self, h):
        self.used -= h["bytes"]
        del self.live[h["id"]]
        self.log.append(("finish", h["id"], self.clock.t))
        return ("out", h["id"])


def _trace(n, rate, seed, big=None):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    specs = []
    for j in range(n):
        b = int(rng.integers(1, 8)) * 100
        if big is not None and j in big:
            b = big[j]
        specs.append(JobSpec(j, float(t[j]), (4, 4, 4), 256,
                             meta={"bytes": b, "need": int(rng.integers(1, 12))}))
    return specs


def test_all_jobs_complete_within_budget():
    clk = VirtualClock()
    ex = SimExecutor(clk)
    srv = Server(ex, budget_bytes=1500, max_active=8, iters_per_step=2, clock=clk, sleep=clk.sleep,
                 keep_outputs=True)
    rep = srv.run(_trace(60, rate=400.0, seed=1))
    s = rep.summary()
    assert s["completed"] == 60 and s["rejected"] == 0
    assert ex.peak <= 1500 and rep.max_bytes <= 1500
    assert rep.max_active <= 8
    assert not ex.live
    for r in rep.records:
        assert r.latency > 0 and r.admitted >= r.spec.arrival - 1e-12
        assert r.completed >= r.admitted
        assert r.outputs == ("out", r.spec.job_id)
        # a job needs ceil(need / 2) steps of 2 iterations
        assert r.result["iterations"] == r.spec.meta["need"]
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0
    assert s["throughput_GBps"] > 0


def test_first_come_first_served_admission():
    clk = VirtualClock()
    ex = SimExecutor(clk)
    srv = Server(ex, budget_bytes=900, max_active=4, clock=clk, sleep=clk.sleep)
    rep = srv.run(_trace(40, rate=1000.0, seed=2))
    starts = [j for ev, j, _ in ex.log if ev == "start"]
    assert starts == sorted(starts)  # arrivals are in id order
    adm = [r.admitted for r in rep.records]
    assert adm == sorted(adm)


def test_continuous_batching_admits_while_others_run():
    clk = VirtualClock()
    ex = SimExecutor(clk)
    srv = Server(ex, budget_bytes=10_000, max_active=16, clock=clk, sleep=clk.sleep)
    specs = _trace(30, rate=2000.0, seed=3)
    rep = srv.run(specs)
    # some job started while an earlier one was still active
    live, overlap = set(), False
    for ev, j, _ in ex.log:
        if ev == "start":
            overlap |= bool(live)
            live.add(j)
        else:
            live.discard(j)
    assert overlap
    # and a late job finished before an early long one
    fin = [j for ev, j, _ in ex.log if ev == "finish"]
    assert fin != sorted(fin)
    assert rep.summary()["completed"] == 30


def test_oversized_and_failing_jobs_are_reported_not_fatal():
    clk = VirtualClock()
    ex = SimExecutor(clk, fail_ids={5})
    srv = Server(ex, budget_bytes=1000, max_active=4, clock=clk, sleep=clk.sleep)
    rep = srv.run(_trace(12, rate=100.0, seed=4, big={3: 5000}))
    errs = {r.spec.job_id: r.error for r in rep.records if r.error}
    assert set(errs) == {3, 5}
    assert "budget" in errs[3] and "bad input" in errs[5]
    s = rep.summary()
    assert s["completed"] == 10 and s["rejected"] == 2
    assert not ex.live


def test_idle_server_waits_for_arrivals():
    clk = VirtualClock()
    ex = SimExecutor(clk)
    specs = [JobSpec(0, 5.0, (2, 2), 16, meta={"bytes": 10, "need": 1}),
             JobSpec(1, 9.0, (2, 2), 16, meta={"bytes": 10, "need": 3})]
    rep = Server(ex, 100, clock=clk, sleep=clk.sleep).run(specs)
    a, b = rep.records
    assert a.admitted >= 5.0 and b.admitted >= 9.0
    assert a.latency < 1.0 and b.latency < 1.0


def test_bad_configuration_rejected():
    clk = VirtualClock()
    with pytest.raises(ValueError):
        Server(SimExecutor(clk), budget_bytes=0)
    with pytest.raises(ValueError):
        Server(SimExecutor(clk), budget_bytes=10, iters_per_step=0)


def test_admission_estimate_gives_way_to_the_real_footprint():
    """An executor that reports a job's real footprint after its set-up:
    the server's accounting follows it (here the real one is half the
    estimate, so a third job fits once the first two have reported)."""
    from paper_2604_01397_amd.serve import JobSpec, Server

    class Ex:
        def __init__(self):
            self.polls = {}
            self.started = []

        def footprint(self, spec):
            return 100

        def footprint_of(self, spec, res):
            return 50 if res.get("num_critical") else None

        def start(self, spec):
            self.started.append(spec.job_id)
            self.polls[spec.job_id] = 0
            return spec.job_id

        def step(self, handles, iters):
            pass

        def poll(self, h):
            self.polls[h] += 1
            return self.polls[h] > 3, {"num_critical": 7}

        def finish(self, h):
            return None

    ex = Ex()
    specs = [JobSpec(j, 0.0, (4, 4, 4), 256) for j in range(3)]
    rep = Server(ex, 200, max_active=8, iters_per_step=1, sleep=lambda t: None).run(specs)
    s = rep.summary()
    assert s["completed"] == 3
    # two admitted at 100 each; after their first poll they count 50 each,
    # so the third is admitted before either finishes
    assert rep.max_active == 3


class TightExecutor(SimExecutor):
    """Memory the budget does not see: allocations fail (transiently) while
    more than `room` bytes are live, until `reclaim` is called once."""

    def __init__(self, clock, room, **kw):
        super().__init__(clock, **kw)
        self.room = room
        self.reclaims = 0

    def transient(self, e):
        return isinstance(e, MemoryError)

    def reclaim(self):
        self.reclaims += 1

    def start(self, spec):
        if self.used + spec.meta["bytes"] > self.room:
            raise MemoryError("device allocation failed")
        return super().start(spec)


def test_transient_allocation_failures_requeue_jobs():
    """Jobs whose allocation fails while others run go back to the head of
    the queue and finish later, in arrival order; none is rejected."""
    clk = VirtualClock()
    ex = TightExecutor(clk, room=1200)
    specs = _trace(60, rate=2000.0, seed=5)
    rep = Server(ex, budget_bytes=5000, max_active=16, clock=clk, sleep=clk.sleep).run(specs)
    s = rep.summary()
    assert s["completed"] == 60 and s["rejected"] == 0, s
    assert s["requeued"] > 0 and ex.reclaims > 0
    starts = [j for ev, j, _ in ex.log if ev == "start"]
    assert starts == sorted(starts)  # first come, first served despite the retries
    assert ex.peak <= 1200


def test_transient_failure_with_nothing_running_is_rejected():
    """A job that cannot be allocated even alone, after a reclaim, is
    rejected instead of being retried for ever."""
    clk = VirtualClock()
    ex = TightExecutor(clk, room=250)
    specs = [JobSpec(0, 0.0, (4, 4, 4), 256, meta={"bytes": 400, "need": 3}),
             JobSpec(1, 0.01, (4, 4, 4), 256, meta={"bytes": 200, "need": 3})]
    rep = Server(ex, budget_bytes=5000, max_active=4, clock=clk, sleep=clk.sleep).run(specs)
    s = rep.summary()
    assert s["completed"] == 1 and s["rejected"] == 1, s
    assert rep.records[0].error is not None and "MemoryError" in rep.records[0].error


class LateFailExecutor(SimExecutor):
    """The set-up of some jobs fails on the device (transiently) the first
    time; the failure shows at the job's first poll."""

    def __init__(self, clock, late_ids, **kw):
        super().__init__(clock, **kw)
        self.late = set(late_ids)
        self.reclaims = 0

    def transient(self, e):
        return isinstance(e, MemoryError)

    def reclaim(self):
        self.reclaims += 1

    def poll(self, h):
        if h["id"] in self.late:
            self.late.discard(h["id"])
            raise MemoryError("critical-point workspace did not fit")
        return super().poll(h)


def test_transient_setup_failure_at_poll_restarts_the_job():
    clk = VirtualClock()
    ex = LateFailExecutor(clk, late_ids=(3, 4, 9))
    specs = _trace(20, rate=500.0, seed=8)
    rep = Server(ex, budget_bytes=4000, max_active=8, clock=clk, sleep=clk.sleep).run(specs)
    s = rep.summary()
    assert s["completed"] == 20 and s["rejected"] == 0 and s["requeued"] == 3, s
    assert [j for ev, j, _ in ex.log if ev == "start"].count(3) == 2
    assert not ex.live  # every started job was finished (released)
