"""Oracle fingerprints of the full-size workloads (test infrastructure).

Runs only the seeded input generators (paper_2604_01397_amd.synth) and the
CPU oracle (oracle/): for every field it records SHA-256 of f and g_hat, of
the oracle's corrected field g' and edit counts, and all of the oracle's
counters.  tests/test_gpu_fingerprints.py rebuilds the same inputs, corrects
them on the GPU and compares.  Nothing here touches a GPU.

    python tests/golden/make_fingerprints.py c2          # 512^3 float32 (minutes)
    python tests/golden/make_fingerprints.py c3 -w 8     # the 96 batched fields
    python tests/golden/make_fingerprints.py c4 -w 8     # serving jobs with L <= 256
    python tests/golden/make_fingerprints.py orig -w 2   # original event constraints, 128^3, 192^3
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2604_01397_amd import synth  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden")
C4_MAX_L = 256
C4_JOBS, C4_RATE = 1000, 200.0


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def fingerprint(case, name=None, mode=0) -> dict:
    t0 = time.perf_counter()
    g, cnt, st, _ = oracle.correct(case.f, case.g_hat, case.xi, mode=mode)
    dt = time.perf_counter() - t0
    return {"name": name or case.name, "shape": list(case.f.shape), "dtype": str(case.f.dtype),
            "xi": case.xi, "f_sha256": sha(case.f), "g_hat_sha256": sha(case.g_hat),
            "g_out_sha256": sha(g), "cnt_sha256": sha(cnt), "oracle_s": round(dt, 2), **st}


ORIG_EDGES = (128, 192)


def _orig_one(edge):
    c = synth.case_grf3d(edge, seed=2, slope=-11.0 / 3.0, rel=1e-4, quantizer="lorenzo")
    out = fingerprint(c, mode=1)
    out["edge"] = edge
    return out


def _c3_one(spec):
    return fingerprint(synth.config3_field(spec))


_SOURCE = None


def _c4_one(spec):
    c = synth.config4_job(_SOURCE, spec)
    out = fingerprint(c)
    out.update({"j": spec["j"], "edge": spec["edge"]})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("config", choices=["c2", "c3", "c4", "orig"])
    ap.add_argument("-w", "--workers", type=int, default=1)
    args = ap.parse_args()
    oracle.build()
    t0 = time.time()
    if args.config == "c2":
        items = [fingerprint(synth.config2(512))]
        meta = {"workload": "512^3 float32 GRF k^-11/3 (seed 2), Lorenzo quantiser, "
                            "eps = 1e-4 range, N = 5, reformulated"}
    elif args.config == "orig":
        with mp.get_context("fork").Pool(args.workers) as pool:
            items = pool.map(_orig_one, ORIG_EDGES, chunksize=1)
        meta = {"workload": "GRF k^-11/3 (seed 2), Lorenzo quantiser, eps = 1e-4 range, N = 5, "
                            "original event constraints (Sec. 4.2), float32, edges %s"
                            % (ORIG_EDGES,)}
    elif args.config == "c3":
        specs = synth.config3_specs(96)
        with mp.get_context("fork").Pool(args.workers) as pool:
            items = pool.map(_c3_one, specs, chunksize=1)
        meta = {"workload": "96 batched fields (seed 3), N = 5, reformulated"}
    else:
        global _SOURCE
        _SOURCE = synth.config4_source()
        print("source volume in %.1f s" % (time.time() - t0), flush=True)
        specs = [s for s in synth.config4_specs(C4_JOBS, C4_RATE) if s["edge"] - 2 <= C4_MAX_L]
        # the largest first, so the pool's tail is short
        specs.sort(key=lambda s: -s["edge"])
        with mp.get_context("fork").Pool(args.workers) as pool:
            items = pool.map(_c4_one, specs, chunksize=1)
        items.sort(key=lambda d: d["j"])
        meta = {"workload": "serving trace (1000 jobs, seed 4): every job with L <= %d, "
                            "(L+2)^3 float32 crops of the 1024^3 GRF k^-3 source (seed 4), "
                            "eps = 1e-3 range of the block, N = 5, reformulated" % C4_MAX_L}
    meta.update({"generator": "tests/golden/make_fingerprints.py %s" % args.config,
                 "oracle_total_s": round(sum(d["oracle_s"] for d in items), 1),
                 "wall_s": round(time.time() - t0, 1), "items": items})
    path = os.path.join(OUT, "fingerprints_%s.json" % args.config)
    with open(path, "w") as fh:
        json.dump(meta, fh, indent=1)
    print("wrote %s (%d fields, %.1f s)" % (path, len(items), time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
