"""Continuous-batching correction server on one GPU.

Jobs arrive over time.  The server admits a job once its device footprint
(the job workspace plus its field, output and count buffers) fits the HBM
budget, materialises its inputs and builds its reference topology on a
side stream while the admitted jobs keep iterating, advances every active
job together with one batched step per tick (``exz_step``: shared launches,
per-job state, per-job convergence), retires finished jobs, frees their
memory and admits the next ones.  Admission is first come, first served;
a job larger than the whole budget is rejected.  Memory the budget does not
see (a caching allocator's free blocks, say) can still make a job's
allocation fail: the executor calls such an error transient, and the job
goes back to the head of the queue, the executor gives back what it can
(``reclaim``), and nothing is admitted until a running job has finished; a
job is rejected for it only when nothing else runs and a retry after
reclaiming fails too.

Latency of a job = its completion (result polled, corrected field on the
device) minus its arrival; aggregate throughput = field bytes of all
completed jobs over the time from the first arrival to the last
completion.

The scheduling loop is plain host logic over an executor interface
(``footprint / start / step / poll / finish``), so it is tested on the CPU
with a simulated executor; ``DeviceExecutor`` drives the library.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Optional

import numpy as np


@dataclass
class JobSpec:
    """One request: when it arrives and how to materialise its inputs."""
    job_id: int
    arrival: float                 # seconds after the start of the trace
    shape: tuple                   # C-order shape of the field
    field_bytes: int               # n * bytes per value
    make: Optional[Callable[[Any], tuple]] = None  # stream -> (f, g_hat, xi) on the device
    meta: dict = field(default_factory=dict)


@dataclass
class JobRecord:
    spec: JobSpec
    admitted: float = float("nan")
    completed: float = float("nan")
    result: Optional[dict] = None
    outputs: Optional[tuple] = None
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.completed - self.spec.arrival


@dataclass
class Report:
    records: list
    wall: float
    max_active: int
    max_bytes: int
    steps: int
    requeued: int = 0   # admissions retried after a transient failure

    def completed(self):
        return [r for r in self.records if r.error is None and not np.isnan(r.completed)]

    def summary(self) -> dict:
        done = self.completed()
        lat = np.array([r.latency for r in done]) if done else np.zeros(0)
        first = min((r.spec.arrival for r in self.records), default=0.0)
        last = max((r.completed for r in done), default=first)
        span = max(last - first, 1e-12)
        nbytes = sum(r.spec.field_bytes for r in done)
        return {
            "jobs": len(self.records),
            "completed": len(done),
            "rejected": sum(r.error is not None for r in self.records),
            "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_latency_s": float(lat.mean()) if lat.size else None,
            "throughput_GBps": nbytes / span / 1e9,
            "field_GB": nbytes / 1e9,
            "span_s": span,
            "max_active": self.max_active,
            "max_resident_GB": self.max_bytes / 1e9,
            "steps": self.steps,
            "requeued": self.requeued,
        }


class Server:
    """The scheduling loop (see the module docstring).

    ``executor`` provides ``footprint(spec) -> bytes``, ``start(spec) ->
    handle``, ``step(handles, iters)``, ``poll(handle) -> (done, result)`` and
    ``finish(handle) -> outputs``.

    ``max_active`` caps the jobs that advance together.  More active jobs
    are not faster: on one MI355X the 1000-job overload trace of (L+2)^3
    float32 blocks was served at 7.9, 8.1, 8.0 and 6.8 GB/s with caps of 8,
    16, 32 and 64, so 16 is the default.
    """

    def __init__(self, executor, budget_bytes: int, max_active: int = 16,
                 iters_per_step: int = 2, clock=time.perf_counter, sleep=time.sleep,
                 keep_outputs: bool = False, progress: Optional[Callable[[dict], None]] = None,
                 progress_every: float = 10.0):
        if budget_bytes <= 0 or max_active < 1 or iters_per_step < 1:
            raise ValueError("budget, max_active and iters_per_step must be positive")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.iters = int(iters_per_step)
        self.clock = clock
        self.sleep = sleep
        self.keep_outputs = keep_outputs
        self.progress = progress
        self.progress_every = progress_every

    def _transient(self, e) -> bool:
        return bool(getattr(self.ex, "transient", lambda _e: False)(e))

    def _reclaim(self):
        getattr(self.ex, "reclaim", lambda: None)()

    def run(self, specs) -> Report:
        pending = collections.deque(sorted(specs, key=lambda s: (s.arrival, s.job_id)))
        queue = collections.deque()
        active = []          # (record, handle, footprint)
        records = {s.job_id: JobRecord(s) for s in pending}
        used = 0
        max_active = max_bytes = steps = 0
        finished = 0
        hold = False         # a transient failure: admit nothing until a job finishes
        retried = set()      # jobs already retried with nothing else running
        self.requeued = 0
        t0 = self.clock()
        last_report = 0.0
        while pending or queue or active:
            now = self.clock() - t0
            if self.progress and now - last_report >= self.progress_every:
                last_report = now
                self.progress({"t": round(now, 1), "finished": finished, "active": len(active),
                               "queued": len(queue), "pending": len(pending), "steps": steps})
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            # the batched step of the active jobs goes out first, so the
            # set-up of newly admitted jobs overlaps it on the device
            if active:
                self.ex.step([h for _, h, _ in active], self.iters)
                steps += 1
            while queue and len(active) < self.max_active and not hold:
                spec = queue[0]
                need = int(self.ex.footprint(spec))
                if need > self.budget:
                    queue.popleft()
                    records[spec.job_id].error = "footprint %d B exceeds the budget" % need
                    continue
                if used + need > self.budget:
                    break
                queue.popleft()
                rec = records[spec.job_id]
                rec.admitted = self.clock() - t0
                try:
                    h = self.ex.start(spec)
                except Exception as e:  # a bad request must not stop the server
                    if self._transient(e) and (active or spec.job_id not in retried):
                        # memory the budget does not see: retry this job later
                        if not active:
                            retried.add(spec.job_id)
                        queue.appendleft(spec)
                        rec.admitted = float("nan")
                        self.requeued += 1
                        self._reclaim()
                        hold = bool(active)
                        break
                    rec.error = "%s: %s" % (type(e).__name__, e)
                    continue
                used += need
                active.append((rec, h, need))
            max_active = max(max_active, len(active))
            max_bytes = max(max_bytes, used)
            if not active:
                if pending and not queue:
                    self.sleep(max(0.0, min(pending[0].arrival - (self.clock() - t0), 0.05)))
                continue
            still = []
            back = []
            for rec, h, need in active:
                try:
                    done, res = self.ex.poll(h)
                except Exception as e:  # a job whose set-up failed (bad input)
                    self.ex.finish(h)
                    used -= need
                    if self._transient(e) and (len(active) > 1 or rec.spec.job_id not in retried):
                        if len(active) == 1:
                            retried.add(rec.spec.job_id)
                        back.append(rec.spec)
                        rec.admitted = float("nan")
                        self.requeued += 1
                        continue
                    rec.error = "%s: %s" % (type(e).__name__, e)
                    finished += 1
                    hold = False
                    continue
                if done:
                    rec.completed = self.clock() - t0
                    rec.result = res
                    out = self.ex.finish(h)
                    if self.keep_outputs:
                        rec.outputs = out
                    used -= need
                    finished += 1
                    hold = False
                else:
                    # the admission estimate gives way to the real footprint
                    # once the job's set-up has counted its critical points
                    real = getattr(self.ex, "footprint_of", lambda *_: None)(rec.spec, res)
                    if real is not None and real != need:
                        used += real - need
                        need = real
                    still.append((rec, h, need))
            active = still
            if back:  # requeued in arrival order, ahead of the waiting jobs
                queue.extendleft(reversed(back))
                self._reclaim()
                hold = bool(active)
        wall = self.clock() - t0
        return Report([records[k] for k in sorted(records)], wall, max_active, max_bytes, steps,
                      self.requeued)


class DeviceExecutor:
    """Runs jobs through the library's job API on one device.

    Inputs are materialised by ``spec.make(stream)`` on a side stream, then
    the job is submitted there (exz_job_submit: its set-up overlaps the
    batched steps issued on the main stream, and nothing waits for it); the
    corrected field is written in place over the job's copy of g_hat.
    ``poll`` never waits (exz_job_query), so the host keeps the main stream
    fed; exz_step itself lets the host run at most about one step ahead.
    With ``blocking=True`` the executor uses exz_job_create / exz_job_poll
    instead (the host waits for each set-up and each step).
    """

    def __init__(self, ctx, n_steps: int = 5, keep_outputs: bool = False, tuned: bool = False,
                 tune_cache: Optional[str] = None, blocking: bool = False):
        import torch

        from . import exactz
        self.torch = torch
        self.exactz = exactz
        self.ctx = ctx
        self.n_steps = n_steps
        self.keep = keep_outputs
        self.main = torch.cuda.Stream()
        self.side = torch.cuda.Stream()
        self.blocking = blocking
        # batched launch options from the autotune table's serving entry, set
        # once before the first job (a job keeps the box shape it was created
        # with, and the jobs of one step must share it)
        self.tuned_options = None
        if tuned:
            from . import autotune
            key = autotune.make_serving_key(autotune.device_arch(ctx.device))
            self.tuned_options = autotune.apply_batch_options(ctx, key, tune_cache)

    # critical points per vertex assumed at admission; the real count, known
    # once a job's set-up has run, replaces the estimate (footprint_of)
    CP_FRACTION = 0.25

    def footprint(self, spec, num_critical=None) -> int:
        shape_xyz = tuple(reversed(spec.shape))
        n = int(np.prod(spec.shape))
        b = spec.field_bytes // max(n, 1)
        k = int(self.CP_FRACTION * n) if num_critical is None else int(num_critical)
        work = self.exactz.workspace_bytes(shape_xyz, self.exactz.F32 if b == 4 else self.exactz.F64,
                                           n_steps=self.n_steps, num_critical=min(k, n))
        return work + 2 * spec.field_bytes + n  # f, g (in place), counts

    def transient(self, e) -> bool:
        """An allocation failure: the library's out-of-memory status, or the
        caching allocator's while the job's inputs are made."""
        if isinstance(e, self.exactz.ExactzError):
            return e.status == self.exactz.E_NOMEM
        return isinstance(e, self.torch.cuda.OutOfMemoryError)

    def reclaim(self):
        """Returns the caching allocator's free blocks, and the library's
        pooled job arenas, to the device."""
        self.torch.cuda.empty_cache()
        self.ctx.set_option("trim", 1)

    def footprint_of(self, spec, result) -> Optional[int]:
        """The job's real footprint once its set-up has run, else None."""
        k = (result or {}).get("num_critical", 0)
        return self.footprint(spec, k) if k else None

    def start(self, spec):
        with self.torch.cuda.stream(self.side):
            f, g, xi = spec.make(self.side)
            cnt = self.torch.zeros(f.shape, dtype=self.torch.uint8, device=f.device)
        # the steps on the main stream use these buffers too: the caching
        # allocator must not hand them out again before that work has ended
        for t in (f, g, cnt):
            t.record_stream(self.main)
        create = self.ctx.job_create if self.blocking else self.ctx.job_submit
        return create(f, g, xi, n_steps=self.n_steps, g_out=g, cnt=cnt, stream=self.side)

    def step(self, handles, iters):
        self.ctx.step(handles, iters, stream=self.main)

    def poll(self, job):
        return job.poll() if self.blocking else job.query()

    def finish(self, job):
        out = (job.g_out, job.cnt) if self.keep else None
        job.release()
        return out
