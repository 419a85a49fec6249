"""Text summaries of rocprofv3 output.

``--stats DIR``   per-kernel dispatch statistics from a
                  ``rocprofv3 --kernel-trace --stats`` run (its
                  ``*_kernel_stats.csv``);
``--pmc DIR ...`` per-kernel averages of every counter of one or more
                  ``rocprofv3 --pmc`` runs (their ``*_counter_collection.csv``);
``--match RE``    keep kernels whose name matches RE.

Counters such as FETCH_SIZE / WRITE_SIZE are reported per dispatch (mean
over the kernel's dispatches) and in total.  Prints Markdown.
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


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--stats", help="directory of a --kernel-trace --stats run")
    ap.add_argument("--pmc", nargs="*", default=[], help="directories of --pmc runs")
    ap.add_argument("--match", default=".", help="regex on kernel names")
    ap.add_argument("--top", type=int, default=12)
    a = ap.parse_args(argv)
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
