"""Benchmark: GB/s of field corrected on one MI355X.

Default workload: the plain correction of a 512^3 float32 turbulence-like
field (Gaussian random field with P(k) ~ k^-11/3, seed 2) quantised by a
Lorenzo predictor + bin-2*eps residual quantiser, eps = 1e-4 of the value
range, 14-neighbour Freudenthal mesh, N = 5, reformulated event constraints.
One step = one full exz_correct call (validation, reference topology, sorted
critical points, loop to the fixpoint) from g_hat into a separate output,
with f and g_hat already resident in HBM.

Prints one JSON line.  ``roofline`` is for the dominant kernel (the check
pass): algorithmic bytes over the check launches' device time, measured with
HIP events on the library's stream during the timed steps.  The algorithmic
bytes of a checked vertex are those the method must move: its value (b), a
one-byte reference code of f, one mark bit, and at a critical point the
value of its successor in f's order (b per critical point, K of n):
(b + 1) + 1/8 + b K / n.  A frontier pass checks only the boxes the last
apply touched.  ``correction_frac`` prices the whole correction the same
way: set-up (3b + 1) n, every iteration a dense pass ((b + 1) n + n/8 + b K),
the edits (3b + 2) per target, and the sort of the critical points
(2 (b + 4) K per 8-bit pass, b passes), over 8 TB/s and the wall time.
``cpu_baseline`` is the CPU oracle, one thread pinned to one core, on a
bounded sample of the same input (a 128^3 sub-block of the field, corrected
to convergence).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STATUS_TEXT = {0: "converged", 1: "stuck (float floor collapse, residual violations)",
               2: "max_iters"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_check_512cube_f32_traffic.txt")


def measured_traffic(edge):
    """HBM bytes per k_check launch from the committed counter runs
    (rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by a copy kernel), or None if
    the workload differs or the check kernel's sources changed since."""
    import hashlib
    if edge != 512 or not os.path.exists(TRAFFIC_RECORD):
        return None
    with open(TRAFFIC_RECORD) as fh:
        rec = json.load(fh)
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"]


def host_cpu():
    """(logical CPUs this process may use, CPU model name)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return len(os.sched_getaffinity(0)), os.cpu_count(), model


def pinned_call(fn):
    """Run fn() with the calling thread pinned to one core (the first one this
    process may use), then restore the affinity.  Returns (result, core)."""
    allowed = os.sched_getaffinity(0)
    core = min(allowed)
    os.sched_setaffinity(0, {core})
    try:
        return fn(), core
    finally:
        os.sched_setaffinity(0, allowed)


def cpu_baseline(case, edge=128):
    """Time the CPU oracle on an edge^3 sub-block of the workload."""
    import numpy as np
    import oracle

    f = np.ascontiguousarray(case.f[:edge, :edge, :edge])
    g = np.ascontiguousarray(case.g_hat[:edge, :edge, :edge])
    oracle.lib()

    def run():
        t0 = time.perf_counter()
        _, _, st, _ = oracle.correct(f, g, case.xi)
        return st, time.perf_counter() - t0

    (st, dt), core = pinned_call(run)
    allowed, total, model = host_cpu()
    return {"value": f.size * f.itemsize / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "nproc": allowed, "cpu_count": total, "cpu_model": model, "pinned_core": core,
            "sample": "%d^3 sub-block of the same field (1/%d of it), corrected to convergence "
                      "(%d iterations) in %.1f s, one thread pinned to one core"
                      % (edge, case.f.size // f.size, st["iterations"], dt)}


def algorithmic_bytes(n, b, K, iterations, targets_total):
    """Bytes the method must move for one correction (see the module text)."""
    setup = (3 * b + 1) * n
    per_iter = (b + 1) * n + n / 8 + b * K
    edits = (3 * b + 2) * targets_total
    sort = 2 * (b + 4) * K * b
    return setup + iterations * per_iter + edits + sort


def run_batched(torch, exactz, synth, reps=2):
    """The 96-field batched workload: one exz_correct_batch call vs the same
    fields corrected one by one with exz_correct (same context, same GPU)."""
    import numpy as np
    t0 = time.time()
    cases = [synth.config3_field(s) for s in synth.config3_specs(96)]
    log("batched: generated %d fields in %.1f s" % (len(cases), time.time() - t0))
    dev = torch.device("cuda:0")
    items = [{"f": torch.from_numpy(c.f).to(dev), "g_hat": torch.from_numpy(c.g_hat).to(dev),
              "xi": c.xi} for c in cases]
    for it in items:
        it["g_out"] = torch.empty_like(it["f"])
        it["cnt"] = torch.zeros(it["f"].shape, dtype=torch.uint8, device=dev)
    nbytes = sum(c.f.nbytes for c in cases)
    ctx = exactz.Context(0)
    ctx.correct_batch(items)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out_b = ctx.correct_batch(items)
    torch.cuda.synchronize()
    t_b = (time.perf_counter() - t0) / reps
    plain_out = [(torch.empty_like(it["f"]), torch.zeros_like(it["cnt"])) for it in items]
    for it, (go, co) in zip(items, plain_out):  # warm-up
        ctx.correct(it["f"], it["g_hat"], it["xi"], g_out=go, cnt=co)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res_p = [ctx.correct(it["f"], it["g_hat"], it["xi"], g_out=go, cnt=co)[2]
                 for it, (go, co) in zip(items, plain_out)]
    torch.cuda.synchronize()
    t_p = (time.perf_counter() - t0) / reps
    same = all(torch.equal(b[0], p[0]) and torch.equal(b[1], p[1])
               for b, p in zip(out_b, plain_out))
    # the same batch with the launch options the shipped autotune table holds
    # for its class (the defaults when it has none)
    from paper_2604_01397_amd import autotune
    key = autotune.batch_key_of(items)
    tuned_opts = autotune.apply_batch_options(ctx, key)
    t_t = None
    if tuned_opts:
        out_t = ctx.correct_batch(items)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out_t = ctx.correct_batch(items)
        torch.cuda.synchronize()
        t_t = (time.perf_counter() - t0) / reps
        same = same and all(torch.equal(b[0], t[0]) and torch.equal(b[1], t[1])
                            for b, t in zip(out_b, out_t))
        for k, v in autotune.BATCH_DEFAULT.options().items():  # back to the defaults
            ctx.set_option(k, v)
    ctx.close()
    its = [r["iterations"] for r in res_p]
    return {"workload": "96 fields, 2D 128^2-2048^2 and 3D 32^3-256^3 (log-uniform), 80 % f32, "
                        "eps in {1e-2, 1e-3, 1e-4} range, uniform quantiser (seed 3)",
            "fields": len(cases), "n_total": int(sum(c.f.size for c in cases)),
            "field_bytes": int(nbytes),
            "batched_GBps": round(nbytes / t_b / 1e9, 3), "batched_ms": round(t_b * 1e3, 3),
            "plain_per_field_GBps": round(nbytes / t_p / 1e9, 3),
            "plain_per_field_ms": round(t_p * 1e3, 3),
            "speedup": round(t_p / t_b, 3), "identical": bool(same),
            "tuned_key": key, "tuned_options": tuned_opts,
            "tuned_batched_GBps": round(nbytes / t_t / 1e9, 3) if t_t else None,
            "tuned_batched_ms": round(t_t * 1e3, 3) if t_t else None,
            "iterations_max": int(max(its)), "iterations_mean": round(float(np.mean(its)), 2)}


def run_float64(torch, exactz, synth, edge=512, reps=3):
    """The 512^3 recipe in float64 (8-byte values, the paper's Table 2
    sizes), with the shipped autotune table's options for its class."""
    import numpy as np
    from paper_2604_01397_amd import autotune
    t0 = time.time()
    case = synth.case_grf3d(edge, seed=2, slope=-11.0 / 3.0, rel=1e-4, dtype=np.float64,
                            quantizer="lorenzo")
    log("float64: generated %s in %.1f s" % (case.name, time.time() - t0))
    dev = torch.device("cuda:0")
    f = torch.from_numpy(case.f).to(dev)
    g = torch.from_numpy(case.g_hat).to(dev)
    g_out = torch.empty_like(f)
    cnt = torch.zeros(f.shape, dtype=torch.uint8, device=dev)
    ctx = exactz.Context(0)
    opts = autotune.apply_options(ctx, f)
    ctx.correct(f, g, case.xi, g_out=g_out, cnt=cnt)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, _, res = ctx.correct(f, g, case.xi, g_out=g_out, cnt=cnt)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    ctx.close()
    return {"workload": "%d^3 float64 GRF k^-11/3 (seed 2), Lorenzo quantiser, eps = 1e-4 range, "
                        "N = 5, reformulated" % edge,
            "ms_per_correction": round(ms, 3), "GBps": round(case.f.nbytes / (ms * 1e-3) / 1e9, 3),
            "tuned_options": opts, "iterations": res["iterations"], "status": res["status"],
            "status_text": STATUS_TEXT.get(res["status"], "?"),
            "residual_violations": res["residual_violations"]}


def run_serving(torch, exactz, synth, serve, jobs, rate, plain=True, max_active=16):
    """Continuous-batching server on a Poisson trace of (L+2)^3 float32 blocks,
    then (same jobs, same inputs) plain per-field exz_correct one after the
    other."""
    import numpy as np
    src_edge = 1024
    t0 = time.time()
    src = synth.grf3d_device(src_edge, seed=4, slope=-3.0)
    torch.cuda.synchronize()
    log("serving: %d^3 source volume in %.1f s" % (src_edge, time.time() - t0))
    trace = synth.config4_specs(jobs, rate)

    def crop(e, off):
        # the periodic crop as at most 8 block copies into one new tensor (no
        # temporaries of other sizes to fill the caching allocator)
        f = torch.empty((e, e, e), dtype=src.dtype, device=src.device)

        def runs(o):  # (source start, length, target start) of each piece
            o = int(o) % src_edge
            a = min(e, src_edge - o)
            return [(o, a, 0)] + ([(0, e - a, a)] if e > a else [])

        for (s0, l0, t0) in runs(off[0]):
            for (s1, l1, t1) in runs(off[1]):
                for (s2, l2, t2) in runs(off[2]):
                    f[t0:t0 + l0, t1:t1 + l1, t2:t2 + l2].copy_(
                        src[s0:s0 + l0, s1:s1 + l1, s2:s2 + l2])
        return f

    # each block's eps (1e-3 of its range) before the served window: inside
    # it, a job's input is cut and quantised on the GPU with no host wait
    t0 = time.time()
    offs, eps = {}, {}
    for s in trace:
        offs[s["j"]] = np.random.default_rng(s["seed"]).integers(0, src_edge, 3)
        eps[s["j"]] = synth.eps_for_device(crop(s["edge"], offs[s["j"]]), 1e-3)
    torch.cuda.empty_cache()
    log("serving: eps of %d blocks in %.1f s" % (len(trace), time.time() - t0))

    def inputs(j, e):
        f = crop(e, offs[j])
        return f, synth.quantize_uniform_device(f, eps[j], checked=False), eps[j]

    specs = []
    for s in trace:
        e = s["edge"]
        specs.append(serve.JobSpec(s["j"], s["arrival"], (e, e, e), 4 * e ** 3,
                                   lambda stream, j=s["j"], e=e: inputs(j, e), meta={"edge": e}))
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    ctx = exactz.Context(0)
    ex = serve.DeviceExecutor(ctx, tuned=True)
    rep = serve.Server(ex, budget, max_active=max_active, iters_per_step=4,
                       progress=lambda d: log("serving: %s" % d)).run(specs)
    torch.cuda.synchronize()
    out = rep.summary()
    field_bytes = sum(s.field_bytes for s in specs)
    out.update({"workload": "Poisson arrivals %.0f jobs/s, %d jobs of (L+2)^3 float32, L "
                            "log-uniform in [64, 1024], GRF k^-3 crops of a periodic %d^3 volume "
                            "made on the GPU (each job's input cut and quantised on the GPU inside "
                            "the window, no host waits), eps = 1e-3 range of each block"
                            % (rate, jobs, src_edge),
                "budget_GB": round(budget / 1e9, 1), "offered_GBps": round(
                    field_bytes / max(specs[-1].arrival, 1e-9) / 1e9, 1),
                "tuned_options": ex.tuned_options})
    if plain:
        # the same jobs, each corrected alone by exz_correct (inputs made
        # outside the timed calls)
        t_plain = 0.0
        its = 0
        for k, s in enumerate(trace):
            f, g, xi = inputs(s["j"], s["edge"])
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, _, r = ctx.correct(f, g, xi, g_out=g)
            torch.cuda.synchronize()
            t_plain += time.perf_counter() - t1
            its += r["iterations"]
            del f, g
            if k % 100 == 99:
                log("serving: plain per-field %d / %d jobs, %.1f s" % (k + 1, len(trace), t_plain))
        out.update({"plain_per_field_GBps": round(field_bytes / t_plain / 1e9, 3),
                    "plain_per_field_s": round(t_plain, 3),
                    "served_over_plain": round(out["throughput_GBps"] * t_plain * 1e9 / field_bytes, 3)
                    if out.get("throughput_GBps") else None})
    ctx.close()
    for k in ("p50_latency_s", "p99_latency_s", "mean_latency_s", "throughput_GBps", "span_s",
              "field_GB", "max_resident_GB"):
        if out.get(k) is not None:
            out[k] = round(out[k], 4)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--edge", type=int, default=512, help="field edge (default 512)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--poll", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0,
                    help="box shape tile_y*100+tile_z (0: by dimensionality, 4 x 8 here)")
    ap.add_argument("--sweep", action="store_true", help="time every compiled box shape first")
    ap.add_argument("--grid", type=int, default=-1, help="stencil grid (-1 persistent, 0 per box)")
    ap.add_argument("--frontier", type=int, default=1, help="1: frontier check passes (default)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched and serving measurements")
    ap.add_argument("--serve-jobs", type=int, default=1000, help="jobs in the serving trace")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="mean arrivals per second")
    ap.add_argument("--serve-max-active", type=int, default=16,
                    help="most jobs the server keeps active at once")
    ap.add_argument("--no-serve-plain", action="store_true",
                    help="skip the plain per-field run of the serving jobs")
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the 96-field batched workload (for profiling) and print its "
                         "figures as one JSON line")
    ap.add_argument("--serving-only", action="store_true",
                    help="only run the serving trace (--serve-jobs, --serve-rate, "
                         "--no-serve-plain) and print its figures as one JSON line")
    ap.add_argument("--copy-calibrate", action="store_true",
                    help="only run a plain 1 GiB read + 1 GiB write elementwise kernel 3 times "
                         "(scale for the HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibrate:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "torch.neg over float32", "read_bytes": src.numel() * 4,
                          "write_bytes": dst.numel() * 4, "launches": 3}), flush=True)
        return

    from paper_2604_01397_amd import exactz, synth

    if args.batched_only:
        print(json.dumps({"batched": run_batched(torch, exactz, synth)}), flush=True)
        return
    if args.serving_only:
        from paper_2604_01397_amd import serve
        print(json.dumps({"serving": run_serving(torch, exactz, synth, serve, args.serve_jobs,
                                                 args.serve_rate, plain=not args.no_serve_plain,
                                                 max_active=args.serve_max_active)}),
              flush=True)
        return

    t0 = time.time()
    case = synth.config2(args.edge)
    log("generated %s in %.1f s (xi=%g)" % (case.name, time.time() - t0, case.xi))
    dev = torch.device("cuda:0")
    f = torch.from_numpy(case.f).to(dev)
    g = torch.from_numpy(case.g_hat).to(dev)
    g_out = torch.empty_like(f)
    cnt = torch.zeros(f.shape, dtype=torch.uint8, device=dev)
    ctx = exactz.Context(0, profile=1, poll=args.poll, tile=args.tile, grid=args.grid,
                         frontier=args.frontier)
    if args.sweep:
        for grid in (-1, 0):
            ctx.set_option("grid", grid)
            for shape in (202, 402, 404, 802, 804, 408, 1602):
                ctx.set_option("tile", shape)
                ctx.correct(f, g, case.xi, g_out=g_out, cnt=cnt, max_iters=2)
                _, _, r = ctx.correct(f, g, case.xi, g_out=g_out, cnt=cnt)
                log("grid %2d tile %4d: check %.4f ms/launch (%d launches, "
                    "%.3g vertices), loop %.2f ms, setup %.2f ms" % (
                        grid, shape, r["check_ms"] / max(r["check_launches"], 1),
                        r["check_launches"], r["check_vertices"], r["loop_ms"], r["setup_ms"]))
        ctx.set_option("tile", args.tile)
        ctx.set_option("grid", args.grid)
    stream = torch.cuda.current_stream()
    res = None
    for w in range(args.warmup):
        _, _, res = ctx.correct(f, g, case.xi, g_out=g_out, cnt=cnt)
        log("warmup %d: %s" % (w, res))
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    check_ms, check_n, check_v = 0.0, 0, 0
    results = []
    for k in range(args.steps):
        _, _, res = ctx.correct(f, g, case.xi, g_out=g_out, cnt=cnt, stream=stream)
        check_ms += res["check_ms"]
        check_n += res["check_launches"]
        check_v += res["check_vertices"]
        results.append(res)
        log("step %d: iters=%d edited=%d status=%d setup=%.2f ms loop=%.2f ms" % (
            k, res["iterations"], res["edited_vertices"], res["status"], res["setup_ms"],
            res["loop_ms"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms = elapsed * 1e3 / args.steps
    n = case.f.size
    b = case.f.itemsize
    value = n * b / (ms * 1e-3) / 1e9
    avg_check_ms = check_ms / max(check_n, 1)
    # algorithmic bytes per vertex checked; critical points at their share
    K = res["num_critical"]
    per_vertex = (b + 1) + 1.0 / 8 + b * K / n
    algo_bytes = per_vertex * check_v / max(check_n, 1)  # per launch, on average
    achieved = per_vertex * check_v / (check_ms * 1e-3) / 1e9
    b_alg = algorithmic_bytes(n, b, K, res["iterations"], res["targets_total"])
    traffic = measured_traffic(args.edge)
    line = {
        "metric": "GB/s of field corrected on 1 MI355X (plain vs batched); p50/p99 job latency",
        "value": round(value, 3),
        "unit": "GB/s",
        "value_GiBps": round(n * b / (ms * 1e-3) / 2 ** 30, 3),  # the paper quotes GiB/s
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plain correction, %d^3 float32 GRF k^-11/3 (seed 2), Lorenzo "
                               "quantiser, eps = 1e-4 range, N = 5, reformulated" % args.edge,
                   "n": n, "iterations": res["iterations"], "edited_vertices": res["edited_vertices"],
                   "num_critical": K, "setup_ms": round(res["setup_ms"], 3),
                   "loop_ms": round(res["loop_ms"], 3), "frontier": args.frontier,
                   "status": res["status"], "status_text": STATUS_TEXT.get(res["status"], "?"),
                   "residual_violations": res["residual_violations"],
                   "targets_total": res["targets_total"]},
        "roofline": {"bound": "hbm", "kernel": "k_check (with the order test)", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "traffic_over_algorithmic": (round(traffic / algo_bytes, 3)
                                                  if traffic else None),
                     "avg_launch_ms": round(avg_check_ms, 5),
                     "launches": check_n, "bytes_per_launch": round(algo_bytes),
                     "bytes_per_vertex": round(per_vertex, 4),
                     "vertices_checked_per_step": check_v // args.steps,
                     "correction_bytes": round(b_alg),
                     "correction_roof_ms": round(b_alg / (HBM_PEAK_GBS * 1e9) * 1e3, 3),
                     "correction_frac": round(b_alg / (HBM_PEAK_GBS * 1e9) / (ms * 1e-3), 4)},
    }
    ctx.close()
    del f, g, g_out, cnt
    torch.cuda.empty_cache()
    if not args.no_extras:
        from paper_2604_01397_amd import serve
        line["batched"] = run_batched(torch, exactz, synth)
        log("batched: %s" % line["batched"])
        torch.cuda.empty_cache()
        line["float64"] = run_float64(torch, exactz, synth, args.edge)
        log("float64: %s" % line["float64"])
        torch.cuda.empty_cache()
        line["serving"] = run_serving(torch, exactz, synth, serve, args.serve_jobs, args.serve_rate,
                                      plain=not args.no_serve_plain,
                                      max_active=args.serve_max_active)
        log("serving: %s" % line["serving"])
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sub-block ...")
        line["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
