"""Text summaries of rocprofv3 output.

``--stats DIR``   per-kernel dispatch statistics from a
                  ``rocprofv3 --kernel-trace --stats`` run (its
                  ``*_kernel_stats.csv``);
``--pmc DIR ...`` per-kernel averages of every counter of one or more
                  ``rocprofv3 --pmc`` runs (their ``*_counter_collection.csv``);
``--match RE``    keep kernels whose name matches RE.
``--record FILE`` write the HBM traffic record of one kernel (``--kernel RE``)
                  from a FETCH_SIZE run and a WRITE_SIZE run (the two
                  ``--pmc`` directories, in that order), each scaled by what
                  the same counter reads for a calibration kernel
                  (``--cal-kernel RE`` in ``--cal-fetch`` / ``--cal-write``)
                  that reads and writes ``--cal-bytes`` bytes per dispatch.

Counters such as FETCH_SIZE / WRITE_SIZE are reported per dispatch (mean
over the kernel's dispatches, in KiB) and in total.  Prints Markdown.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import os
import re
import sys


def _one(pattern: str) -> str:
    hits = sorted(glob.glob(pattern, recursive=True))
    if not hits:
        raise FileNotFoundError(pattern)
    return hits[0]


def kernel_stats(path: str):
    """Rows of the kernel statistics CSV as dicts (durations in ns)."""
    f = _one(os.path.join(path, "**", "*kernel_stats.csv"))
    out = []
    with open(f, newline="") as fh:
        for r in csv.DictReader(fh):
            out.append({"name": r["Name"], "calls": int(r["Calls"]),
                        "total_ns": float(r["TotalDurationNs"]), "avg_ns": float(r["AverageNs"]),
                        "min_ns": float(r["MinNs"]), "max_ns": float(r["MaxNs"]),
                        "pct": float(r["Percentage"])})
    return out


def counters(path: str):
    """{kernel: {counter: [per-dispatch values]}} from a counter collection CSV."""
    f = _one(os.path.join(path, "**", "*counter_collection.csv"))
    acc = collections.defaultdict(lambda: collections.defaultdict(dict))
    with open(f, newline="") as fh:
        for r in csv.DictReader(fh):
            # several rows of one dispatch and counter (one per hardware
            # instance) are summed
            d = acc[r["Kernel_Name"]][r["Counter_Name"]]
            key = r["Dispatch_Id"]
            d[key] = d.get(key, 0.0) + float(r["Counter_Value"])
    return {k: {c: list(v.values()) for c, v in cs.items()} for k, cs in acc.items()}


def _mean(cs, rx, counter):
    """Mean per dispatch of one counter over the kernels matching rx."""
    vals = []
    for k, c in cs.items():
        if rx.search(k) and counter in c:
            vals += c[counter]
    if not vals:
        raise KeyError("no %s values for kernels matching %r" % (counter, rx.pattern))
    return sum(vals) / len(vals), len(vals)


def write_record(a) -> int:
    """The traffic record: counter means in KiB per dispatch, scaled to bytes
    by the calibration kernel's known traffic."""
    import hashlib
    import json
    if len(a.pmc) != 2 or not (a.kernel and a.cal_kernel and a.cal_fetch and a.cal_write
                               and a.cal_bytes):
        raise SystemExit("--record needs --pmc FETCH_DIR WRITE_DIR, --kernel, --cal-kernel, "
                         "--cal-fetch, --cal-write and --cal-bytes")
    krx, crx = re.compile(a.kernel), re.compile(a.cal_kernel)
    fetch_kib, nd = _mean(counters(a.pmc[0]), krx, "FETCH_SIZE")
    write_kib, _ = _mean(counters(a.pmc[1]), krx, "WRITE_SIZE")
    cal_f, _ = _mean(counters(a.cal_fetch), crx, "FETCH_SIZE")
    cal_w, _ = _mean(counters(a.cal_write), crx, "WRITE_SIZE")
    fs, ws = a.cal_bytes / (cal_f * 1024.0), a.cal_bytes / (cal_w * 1024.0)
    h = hashlib.sha256()
    for src in a.sources:
        with open(src, "rb") as fh:
            h.update(fh.read())
    rec = {"kernel": a.kernel, "workload": a.workload, "dispatches": nd,
           "fetch_bytes_per_launch": round(fetch_kib * 1024.0 * fs),
           "write_bytes_per_launch": round(write_kib * 1024.0 * ws),
           "fetch_scale": fs, "write_scale": ws,
           "algorithmic_bytes_per_launch": a.algo_bytes,
           "sources": a.sources, "source_sha256": h.hexdigest()}
    rec["traffic_bytes_per_launch"] = rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    with open(a.record, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec))
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--stats", help="directory of a --kernel-trace --stats run")
    ap.add_argument("--pmc", nargs="*", default=[], help="directories of --pmc runs")
    ap.add_argument("--match", default=".", help="regex on kernel names")
    ap.add_argument("--top", type=int, default=12)
    ap.add_argument("--record", help="traffic record file to write (JSON)")
    ap.add_argument("--kernel", help="regex of the recorded kernel")
    ap.add_argument("--cal-kernel", help="regex of the calibration kernel")
    ap.add_argument("--cal-fetch", help="FETCH_SIZE run of the calibration kernel")
    ap.add_argument("--cal-write", help="WRITE_SIZE run of the calibration kernel")
    ap.add_argument("--cal-bytes", type=float, help="bytes the calibration kernel reads and writes")
    ap.add_argument("--algo-bytes", type=float, help="algorithmic bytes per launch (recorded)")
    ap.add_argument("--workload", default="", help="workload description (recorded)")
    ap.add_argument("--sources", nargs="*", default=[],
                    help="source files whose SHA-256 the record carries")
    a = ap.parse_args(argv)
    if a.record:
        return write_record(a)
    rx = re.compile(a.match)
    if a.stats:
        rows = [r for r in kernel_stats(a.stats) if rx.search(r["name"])]
        rows.sort(key=lambda r: -r["total_ns"])
        print("| kernel | calls | total ms | avg us | min us | max us | % |")
        print("|---|---:|---:|---:|---:|---:|---:|")
        for r in rows[: a.top]:
            print("| `%s` | %d | %.3f | %.2f | %.2f | %.2f | %.2f |" % (
                r["name"][:90], r["calls"], r["total_ns"] / 1e6, r["avg_ns"] / 1e3,
                r["min_ns"] / 1e3, r["max_ns"] / 1e3, r["pct"]))
        print()
    for d in a.pmc:
        cs = counters(d)
        print("counters from `%s`:" % d)
        print()
        print("| kernel | counter | dispatches | mean per dispatch | total |")
        print("|---|---|---:|---:|---:|")
        for k in sorted(cs):
            if not rx.search(k):
                continue
            for c in sorted(cs[k]):
                v = cs[k][c]
                print("| `%s` | %s | %d | %.6g | %.6g |" % (k[:90], c, len(v), sum(v) / len(v), sum(v)))
        print()
    return 0


if __name__ == "__main__":
    sys.exit(main())
