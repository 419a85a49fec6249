"""Autotuner for the library's launch options.

The options (check box shape, stencil grid, frontier passes, poll interval)
never change a result; they change only speed.  ``tune`` times every
candidate of a search space on a representative problem, checks that all
of them produce the same corrected field and edit counts (so a broken
configuration can never be selected), and stores the fastest one in a JSON
cache keyed by (GPU architecture, dimensionality, dtype, size class).
``apply_options`` / ``TunedContext`` look the key up for each field and set
the cached options on the context before correcting it.

Size class = floor(log2(number of vertices)), so one tuning run serves
fields within a factor of two of the tuned size.

Batched calls (``exz_correct_batch``) and the job API's steps (``exz_step``)
have launch options of their own: the boxes of their 3D and 1D/2D members,
the work-group caps of the batched check and apply passes and the apply
item size.  ``tune_batch`` searches them by coordinate descent (one axis at
a time from the defaults, keeping the best value of each) on a
representative batch, with the same result-invariance check, under a key
of (architecture, "batch", the members' dimensionalities and dtypes, size
class of the total vertex count).  ``TunedContext.correct_batch`` and
``apply_batch_options`` use it.  The serving executor sets the options of
the table's "serving" entry (tuned on a serving step's active set) once,
before its first job: jobs keep the box shape they were created with.

A table tuned on MI355X ships with the package (``tuned/gfx950.json``); the
per-user cache, when it has an entry for the key, takes precedence.
"""
from __future__ import annotations

import json
import math
import os
import tempfile
import time
from dataclasses import dataclass
from typing import Callable, Iterable, Optional

# Box shapes (tile_y, tile_z) compiled into the library.
BOXES_3D = [(2, 2), (4, 2), (4, 4), (8, 2), (8, 4), (4, 8), (16, 2)]
BOXES_2D = [(1, 1), (4, 1), (8, 1), (16, 1)]
BOXES_1D = [(1, 1)]

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "exactz", "autotune.json")
SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned")


def cache_path(path: Optional[str] = None) -> str:
    return path or os.environ.get("EXACTZ_AUTOTUNE_CACHE") or DEFAULT_CACHE


def size_class(n: int) -> int:
    return int(math.floor(math.log2(max(int(n), 1))))


def make_key(arch: str, ndim: int, dtype: str, n: int) -> str:
    arch = arch.split(":")[0]  # gfx950:sramecc+:xnack- -> gfx950
    return "%s|%dd|%s|2^%d" % (arch, ndim, dtype, size_class(n))


def field_ndim(shape) -> int:
    """Dimensionality as the library sees it (trailing unit axes dropped)."""
    dims = [int(d) for d in reversed(tuple(shape))]  # x fastest
    nd = len(dims)
    while nd > 1 and dims[nd - 1] == 1:
        nd -= 1
    return nd


@dataclass(frozen=True)
class Candidate:
    tile: int       # tile_y * 100 + tile_z
    grid: int       # -1 persistent, 0 one work-group per box
    frontier: int   # 0 / 1
    poll: int       # 0 adaptive, else fixed

    def options(self) -> dict:
        return {"tile": self.tile, "grid": self.grid, "frontier": self.frontier, "poll": self.poll}


def search_space(ndim: int, quick: bool = False) -> list:
    boxes = BOXES_3D if ndim == 3 else BOXES_2D if ndim == 2 else BOXES_1D
    if quick:
        boxes = boxes[-3:] if ndim == 3 else boxes[-2:] if ndim == 2 else boxes
    grids = (-1,) if quick else (-1, 0)
    polls = (0,) if quick else (0, 16)
    out = []
    for ty, tz in boxes:
        for g in grids:
            for fr in (1, 0):
                for p in polls:
                    out.append(Candidate(ty * 100 + tz, g, fr, p))
    return out


class TuneError(RuntimeError):
    pass


def _read_json(p: str) -> dict:
    if not os.path.exists(p):
        return {}
    with open(p) as fh:
        try:
            data = json.load(fh)
        except json.JSONDecodeError:
            return {}
    return data if isinstance(data, dict) else {}


def load_cache(path: Optional[str] = None) -> dict:
    return _read_json(cache_path(path))


def shipped_table(arch: str) -> dict:
    """The table tuned for arch that ships with the package ({} if none)."""
    return _read_json(os.path.join(SHIPPED, arch.split(":")[0] + ".json"))


def lookup(key: str, cache: Optional[str] = None) -> Optional[dict]:
    """The cache's entry for key, else the shipped table's, else None."""
    e = load_cache(cache).get(key)
    if e:
        return e
    return shipped_table(key.split("|")[0]).get(key)


def save_cache(data: dict, path: Optional[str] = None) -> None:
    p = cache_path(path)
    os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(p) or ".", suffix=".tmp")
    with os.fdopen(fd, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, p)  # atomic: concurrent readers see the old or the new file


def search(run: Callable[[Candidate], tuple], candidates: Iterable[Candidate], repeats: int = 1):
    """Time every candidate with ``run(c) -> (ms, fingerprint)``.

    Returns (best candidate, table of (candidate, ms)).  Raises TuneError if
    two candidates disagree on the fingerprint of the result.
    """
    table = []
    ref = None
    for c in candidates:
        best = math.inf
        for _ in range(max(1, repeats)):
            ms, fp = run(c)
            if ref is None:
                ref = (c, fp)
            elif fp != ref[1]:
                raise TuneError("candidate %s changed the result (vs %s)" % (c, ref[0]))
            best = min(best, ms)
        table.append((c, best))
    if not table:
        raise TuneError("empty search space")
    return min(table, key=lambda t: t[1])[0], table


def _fingerprint(g_out, cnt, res) -> tuple:
    import hashlib
    h = hashlib.sha256()
    h.update(g_out.contiguous().view(-1).cpu().numpy().tobytes())
    h.update(cnt.contiguous().view(-1).cpu().numpy().tobytes())
    return (h.hexdigest(), res["iterations"], res["edit_ops"], res["status"])


def device_arch(device: int = 0) -> str:
    import torch
    return torch.cuda.get_device_properties(device).gcnArchName


def tune(ctx, f, g_hat, xi, n_steps: int = 5, quick: bool = False, repeats: int = 1,
         cache: Optional[str] = None, candidates=None, log=None) -> dict:
    """Tune the options for f's class on (f, g_hat, xi); store and return them."""
    import torch
    ndim = field_ndim(f.shape)
    dtype = "f32" if f.dtype == torch.float32 else "f64"
    key = make_key(device_arch(f.device.index or 0), ndim, dtype, f.numel())
    cands = list(candidates) if candidates is not None else search_space(ndim, quick)
    g_out = torch.empty_like(f)
    cnt = torch.empty(f.shape, dtype=torch.uint8, device=f.device)
    saved = {"profile": 0}

    def run(c: Candidate):
        for k, v in c.options().items():
            ctx.set_option(k, v)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out, cn, res = ctx.correct(f, g_hat, xi, n_steps=n_steps, g_out=g_out, cnt=cnt)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        if log:
            log("tune %s %s: %.3f ms" % (key, c, ms))
        return ms, _fingerprint(out, cn, res)

    try:
        run(cands[0])  # warm the workspace and the code paths
        best, table = search(run, cands, repeats)
    finally:
        for k, v in Candidate(0, -1, 1, 0).options().items():
            ctx.set_option(k, v)
        ctx.set_option("profile", saved["profile"])
    entry = dict(best.options())
    entry["ms"] = min(ms for _, ms in table)
    entry["default_ms"] = next((ms for c, ms in table if c == Candidate(0, -1, 1, 0)), None)
    entry["candidates"] = len(table)
    data = load_cache(cache)
    data[key] = entry
    save_cache(data, cache)
    return {"key": key, **entry}


def options_for(arch: str, ndim: int, dtype: str, n: int, cache: Optional[str] = None):
    """Cached (or shipped) options for a field class, or None."""
    e = lookup(make_key(arch, ndim, dtype, n), cache)
    if not e:
        return None
    return {k: e[k] for k in ("tile", "grid", "frontier", "poll") if k in e}


def apply_options(ctx, f, cache: Optional[str] = None) -> Optional[dict]:
    """Set the cached options for f's class on ctx (the defaults if none)."""
    import torch
    dtype = "f32" if f.dtype == torch.float32 else "f64"
    opts = options_for(device_arch(f.device.index or 0), field_ndim(f.shape), dtype, f.numel(), cache)
    chosen = opts or Candidate(0, -1, 1, 0).options()
    for k, v in chosen.items():
        ctx.set_option(k, v)
    return opts


# ----------------------------------------------------------------------------
# batched calls and job steps


@dataclass(frozen=True)
class BatchCandidate:
    btile3: int       # box of the 3D members (tile_y * 100 + tile_z), 0 = default
    btile2: int       # box of the 1D / 2D members (tile_y * 100 + 1), 0 = default
    bgrid_box: int    # work-group cap of the batched check, 0 = default
    bgrid_apply: int  # work-group cap of the batched apply, 0 = default
    bitem: int        # apply item in quads per thread, 0 = default

    def options(self) -> dict:
        return {"btile3": self.btile3, "btile2": self.btile2, "bgrid_box": self.bgrid_box,
                "bgrid_apply": self.bgrid_apply, "bitem": self.bitem}


BATCH_DEFAULT = BatchCandidate(0, 0, 0, 0, 0)
BATCH_KEYS = ("btile3", "btile2", "bgrid_box", "bgrid_apply", "bitem")

# values tried per axis (the first is the library's default)
BATCH_AXES = {
    "btile3": [0, 804, 404, 802, 402, 1602],
    "btile2": [0, 801, 401, 101],
    "bgrid_box": [0, 1024, 2048, 8192, 16384],
    "bgrid_apply": [0, 1024, 2048, 8192, 16384],
    "bitem": [0, 4, 8, 32, 64],
}


def batch_signature(shapes_dtypes) -> tuple:
    """(dimensionalities, dtypes, total vertices) of a batch's members."""
    dims, dts, n = set(), set(), 0
    for shape, dt in shapes_dtypes:
        dims.add(field_ndim(shape))
        dts.add(dt)
        nv = 1
        for d in shape:
            nv *= int(d)
        n += nv
    return tuple(sorted(dims)), tuple(sorted(dts)), n


def make_batch_key(arch: str, dims, dtypes, n: int) -> str:
    arch = arch.split(":")[0]
    return "%s|batch|%s|%s|2^%d" % (arch, "+".join("%dd" % d for d in dims), "+".join(dtypes),
                                    size_class(n))


def _dtype_name(t) -> str:
    import torch
    return "f32" if t.dtype == torch.float32 else "f64"


def make_serving_key(arch: str) -> str:
    """Key of the options a serving executor sets once, before its first job
    (jobs keep the box shape they were created with, and one step's jobs
    must share it)."""
    return "%s|serving" % arch.split(":")[0]


def batch_key_of(items, device: int = 0) -> str:
    dims, dts, n = batch_signature([(it["f"].shape, _dtype_name(it["f"])) for it in items])
    return make_batch_key(device_arch(device), dims, dts, n)


def coordinate_search(run: Callable[[BatchCandidate], tuple], axes: dict, start: BatchCandidate,
                      repeats: int = 1):
    """One pass of coordinate descent: for each axis in turn, time every value
    with the other axes at their best so far, keep the fastest.  Every result
    must equal the first one.  Returns (best, table of (candidate, ms))."""
    table, ref, seen = [], None, {}

    def timed(c):
        if c in seen:
            return seen[c]
        nonlocal ref
        best = math.inf
        for _ in range(max(1, repeats)):
            ms, fp = run(c)
            if ref is None:
                ref = (c, fp)
            elif fp != ref[1]:
                raise TuneError("candidate %s changed the result (vs %s)" % (c, ref[0]))
            best = min(best, ms)
        seen[c] = best
        table.append((c, best))
        return best

    cur = start
    timed(cur)
    for key, values in axes.items():
        for v in values:
            c = BatchCandidate(**{**cur.options(), key: v})
            timed(c)
        cur = min((c for c in seen if all(getattr(c, k) == getattr(cur, k)
                                          for k in BATCH_KEYS if k != key)),
                  key=lambda c: seen[c])
    return cur, table


def _batch_fingerprint(out) -> tuple:
    return tuple(_fingerprint(g, c, r) for g, c, r in out)


def tune_batch(ctx, items, repeats: int = 1, cache: Optional[str] = None, axes=None,
               log=None, key: Optional[str] = None) -> dict:
    """Tune the batched options on ``items`` (as for Context.correct_batch);
    store and return them under the batch's key (or ``key``)."""
    import torch
    key = key or batch_key_of(items, items[0]["f"].device.index or 0)
    axes = axes or BATCH_AXES
    work = [dict(it, g_out=torch.empty_like(it["f"]),
                 cnt=torch.empty(it["f"].shape, dtype=torch.uint8, device=it["f"].device))
            for it in items]

    def run(c: BatchCandidate):
        for k, v in c.options().items():
            ctx.set_option(k, v)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = ctx.correct_batch(work)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        if log:
            log("tune %s %s: %.3f ms" % (key, c, ms))
        return ms, _batch_fingerprint(out)

    try:
        run(BATCH_DEFAULT)  # warm the workspace and the code paths
        best, table = coordinate_search(run, axes, BATCH_DEFAULT, repeats)
    finally:
        for k, v in BATCH_DEFAULT.options().items():
            ctx.set_option(k, v)
    entry = dict(best.options())
    entry["ms"] = min(ms for _, ms in table)
    entry["default_ms"] = next((ms for c, ms in table if c == BATCH_DEFAULT), None)
    entry["candidates"] = len(table)
    data = load_cache(cache)
    data[key] = entry
    save_cache(data, cache)
    return {"key": key, **entry}


def batch_options_for(key: str, cache: Optional[str] = None) -> Optional[dict]:
    e = lookup(key, cache)
    if not e:
        return None
    return {k: e[k] for k in BATCH_KEYS if k in e}


def apply_batch_options(ctx, key: str, cache: Optional[str] = None) -> Optional[dict]:
    """Set the tuned batched options for key on ctx (the defaults if none)."""
    opts = batch_options_for(key, cache)
    for k, v in (opts or BATCH_DEFAULT.options()).items():
        ctx.set_option(k, v)
    return opts


class TunedContext:
    """A Context whose options follow the autotune table per field class
    (single fields) and per batch class (batched calls)."""

    def __init__(self, device: int = 0, cache: Optional[str] = None, **options):
        from . import exactz
        self.ctx = exactz.Context(device, **options)
        self.cache = cache
        self.device = device

    def correct(self, f, g_hat, xi, **kw):
        apply_options(self.ctx, f, self.cache)
        return self.ctx.correct(f, g_hat, xi, **kw)

    def correct_batch(self, items, **kw):
        apply_batch_options(self.ctx, batch_key_of(items, self.device), self.cache)
        return self.ctx.correct_batch(items, **kw)

    def close(self):
        self.ctx.close()


# ----------------------------------------------------------------------------
# the shipped table: tuning runs on the benchmark's workload classes


def _table_workloads(quick: bool):
    """(label, kind, payload) of the classes the shipped table covers: the
    plain single-field classes of the benchmark's configurations and the
    batched classes of its 96-field set and of a serving step."""
    import numpy as np
    import torch

    from . import synth

    def dev(c):
        return torch.from_numpy(np.ascontiguousarray(c.f)).cuda(), \
            torch.from_numpy(np.ascontiguousarray(c.g_hat)).cuda(), c.xi

    yield "128^3 f32 (uniform, 1e-3)", "single", lambda: dev(synth.config1())
    yield "512^3 f32 (Lorenzo, 1e-4)", "single", lambda: dev(synth.config2(512))
    if not quick:
        yield "256^3 f32 (Lorenzo, 1e-4)", "single", lambda: dev(synth.config2(256))
        yield "512^3 f64 (Lorenzo, 1e-4)", "single", lambda: dev(
            synth.case_grf3d(512, seed=2, slope=-11.0 / 3.0, rel=1e-4, dtype=np.float64,
                             quantizer="lorenzo"))
        yield "256^2 f32 (Gaussians, 1e-3)", "single", lambda: dev(synth.case_gauss2d(256))

    def c3():
        items = []
        for s in synth.config3_specs(96):
            f, g, xi = dev(synth.config3_field(s))
            items.append({"f": f, "g_hat": g, "xi": xi})
        return items
    yield "96-field batch", "batch", c3

    def c4(active=32):
        # a serving step's active set: the first jobs of the serving trace,
        # cut from a device-synthesised source (timing only)
        src = synth.grf3d_device(512, seed=4, slope=-3.0)
        items = []
        for s in synth.config4_specs(active, 200.0):
            e = min(s["edge"], 256)
            off = [int(v) for v in np.random.default_rng(s["seed"]).integers(0, 512 - e, 3)]
            f = src[off[0]:off[0] + e, off[1]:off[1] + e, off[2]:off[2] + e].contiguous()
            eps = synth.eps_for_device(f, 1e-3)
            items.append({"f": f, "g_hat": synth.quantize_uniform_device(f, eps), "xi": eps})
        return items
    yield "serving step (32 jobs)", "serving", c4


def build_table(path: str, quick: bool = False, repeats: int = 2, log=print) -> dict:
    """Tune every class of _table_workloads on this GPU into a fresh table at
    path (the per-user cache is not touched)."""
    from . import exactz
    ctx = exactz.Context(0)
    report = {}
    try:
        for label, kind, make in _table_workloads(quick):
            log("tuning %s" % label)
            if kind == "single":
                f, g, xi = make()
                e = tune(ctx, f, g, xi, quick=quick, repeats=repeats, cache=path, log=None)
                del f, g
            else:
                items = make()
                key = make_serving_key(device_arch(0)) if kind == "serving" else None
                e = tune_batch(ctx, items, repeats=repeats, cache=path, log=None, key=key)
                del items
            log("  %s: %s" % (e["key"], {k: v for k, v in e.items() if k != "key"}))
            report[label] = e
    finally:
        ctx.close()
    return report


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="tune the launch options on this GPU")
    ap.add_argument("--table", required=True, help="write the table to this JSON file")
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--repeats", type=int, default=2)
    args = ap.parse_args(argv)
    if os.path.exists(args.table):
        os.remove(args.table)
    build_table(args.table, quick=args.quick, repeats=args.repeats)


if __name__ == "__main__":
    main()
