"""Two studies of the correction on one GPU (Markdown tables on stdout).

--tradeoff   original vs reformulated event constraints (Sec. 4.2 vs 4.3)
             over relative error bounds 1e-6 .. 1e-3: correction time,
             iterations, edited vertices and edit-stream size (the
             reformulation trades extra edits for cheaper iterations,
             Sec. 5.4);
--nsweep     N = 1 .. 10 at one bound: time, iterations, edited vertices,
             lossless edits and edit-stream size (App. C: fewer steps mean
             fewer iterations and more lossless edits);
--table1     the Table 1 analogue (Sec. 4.4): vertices in the weak, strong
             and reduced vulnerability graphs, edited vertices, the
             iteration bound from D_max(G_R) and the actual iterations, for
             the 128^3, 256^3 and 512^3 GRF fields at bound 1e-4.

Input: the 3D float32 GRF k^-11/3 of the 512^3 workload (seed 2, or an
--edge^3 version), Lorenzo quantiser at each bound.  The edit stream is
editcodec's (counts + exact values), raw and after zlib level 1.
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np


STATUS = {0: "converged", 1: "stuck", 2: "max iters"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_one(ctx, exactz, editcodec, torch, f_host, g_host, f, g, xi, mode, n_steps):
    g_out = torch.empty_like(f)
    cnt = torch.zeros(f.shape, dtype=torch.uint8, device=f.device)
    # one untimed call (workspace growth), then the measured one
    ctx.correct(f, g, xi, n_steps=n_steps, mode=mode, g_out=g_out, cnt=cnt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, r = ctx.correct(f, g, xi, n_steps=n_steps, mode=mode, g_out=g_out, cnt=cnt)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    go = g_out.cpu().numpy()
    cn = cnt.cpu().numpy()
    es = editcodec.encode(g_host, go, cn, editcodec.step(xi, f_host.dtype, n_steps), n_steps)
    return {"ms": ms, "iterations": r["iterations"], "edited": r["edited_vertices"],
            "edit_ops": r["edit_ops"], "lossless": int(np.count_nonzero(cn == n_steps + 1)),
            "status": r["status"], "residual": r["residual_violations"],
            "stream": len(es.data), "zlib": es.compressed(1), "exact": es.exact}


def table1(torch, exactz, synth, edges=(128, 256, 512), rel=1e-4, n_steps=5):
    from . import vulnerability
    print("### Vulnerability graphs vs actual iterations, rel. bound %g, N = %d\n" % (rel, n_steps))
    print("| field | \\|G_V\\| % | \\|G_S\\| % | \\|G_R\\| % | edit % | D_max(G_R) | "
          "bound (N+1)·D_max | N·D_max | actual iterations | analysis s |")
    print("|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|")
    fields = [("128^3 GRF k^-3, uniform", 128, -3.0, 1, "uniform"),
              ("256^3 GRF k^-11/3, Lorenzo", 256, -11.0 / 3.0, 2, "lorenzo"),
              ("512^3 GRF k^-11/3, Lorenzo", 512, -11.0 / 3.0, 2, "lorenzo")]
    ctx = exactz.Context(0)
    try:
        for name, edge, slope, seed, q in fields:
            if edge not in edges:
                continue
            fh = synth.grf3d(edge, seed=seed, slope=slope)
            log("%s: generated" % name)
            xi = synth.eps_for(fh, rel)
            gh = synth.quantize_lorenzo(fh, xi) if q == "lorenzo" else synth.quantize_uniform(fh, xi)
            f = torch.from_numpy(fh).cuda()
            g = torch.from_numpy(gh).cuda()
            _, _, r = ctx.correct(f, g, xi, n_steps=n_steps)
            torch.cuda.synchronize()
            log("%s: corrected (%d iterations)" % (name, r["iterations"]))
            t0 = time.perf_counter()
            m = vulnerability.metrics(f.view(-1), g.view(-1), xi, (edge, edge, edge),
                                      log=lambda s, name=name: log("%s: %s" % (name, s)))
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            n = fh.size
            log("%s: %s, result %s" % (name, m, r))
            print("| %s | %.2f | %.2f | %.2f | %.2f | %d | %d | %d | %d | %.1f |" % (
                name, 100.0 * m["V_GV"] / n, 100.0 * m["V_GS"] / n, 100.0 * m["V_GR"] / n,
                100.0 * r["edited_vertices"] / n, m["D_max"], (n_steps + 1) * m["D_max"],
                n_steps * m["D_max"], r["iterations"], dt))
            del f, g
            torch.cuda.empty_cache()
    finally:
        ctx.close()
    print()


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--edge", type=int, default=512)
    ap.add_argument("--tradeoff", action="store_true")
    ap.add_argument("--nsweep", action="store_true")
    ap.add_argument("--rel", type=float, default=1e-4, help="bound of the N sweep")
    ap.add_argument("--table1", action="store_true")
    ap.add_argument("--table1-edges", type=int, nargs="*", default=[128, 256, 512])
    a = ap.parse_args(argv)
    import torch

    from . import editcodec, exactz, synth
    if a.table1:
        table1(torch, exactz, synth, edges=tuple(a.table1_edges))
        if not (a.tradeoff or a.nsweep):
            return 0
    t0 = time.time()
    f_host = synth.grf3d(a.edge, seed=2, slope=-11.0 / 3.0)
    log("field %d^3 in %.1f s" % (a.edge, time.time() - t0))
    f = torch.from_numpy(f_host).cuda()
    n = f_host.size
    gb = f_host.nbytes / 1e9
    ctx = exactz.Context(0)
    try:
        if a.tradeoff:
            print("### Original vs reformulated event constraints, %d^3 float32, N = 5\n" % a.edge)
            print("| rel. bound | mode | time ms | GB/s | iterations | edited % | edit ops | "
                  "status | stream bytes | zlib bytes |")
            print("|---|---|---:|---:|---:|---:|---:|---|---:|---:|")
            for rel in (1e-6, 1e-5, 1e-4, 1e-3):
                xi = synth.eps_for(f_host, rel)
                g_host = synth.quantize_lorenzo(f_host, xi)
                g = torch.from_numpy(g_host).cuda()
                for mode, name in ((exactz.ORIGINAL, "original"), (exactz.REFORMULATED, "reformulated")):
                    r = run_one(ctx, exactz, editcodec, torch, f_host, g_host, f, g, xi, mode, 5)
                    log("rel %g %s: %s" % (rel, name, r))
                    print("| %g | %s | %.1f | %.2f | %d | %.3f | %d | %s | %d | %d |" % (
                        rel, name, r["ms"], gb / (r["ms"] * 1e-3), r["iterations"],
                        100.0 * r["edited"] / n, r["edit_ops"], STATUS.get(r["status"], str(r["status"])),
                        r["stream"], r["zlib"]))
                del g
            print()
        if a.nsweep:
            xi = synth.eps_for(f_host, a.rel)
            g_host = synth.quantize_lorenzo(f_host, xi)
            g = torch.from_numpy(g_host).cuda()
            print("### N sweep, %d^3 float32, rel. bound %g, reformulated\n" % (a.edge, a.rel))
            print("| N | time ms | iterations | edited % | lossless edits | exact values | "
                  "stream bytes | zlib bytes |")
            print("|---:|---:|---:|---:|---:|---:|---:|---:|")
            for n_steps in range(1, 11):
                r = run_one(ctx, exactz, editcodec, torch, f_host, g_host, f, g, xi,
                            exactz.REFORMULATED, n_steps)
                log("N %d: %s" % (n_steps, r))
                print("| %d | %.1f | %d | %.3f | %d | %d | %d | %d |" % (
                    n_steps, r["ms"], r["iterations"], 100.0 * r["edited"] / n, r["lossless"],
                    r["exact"], r["stream"], r["zlib"]))
            print()
    finally:
        ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
