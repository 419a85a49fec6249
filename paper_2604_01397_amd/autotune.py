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


def load_cache(path: Optional[str] = None) -> dict:
    p = cache_path(path)
    if not os.path.exists(p):
        return {}
    with open(p) as fh:
        try:
            data = json.load(fh)
        except json.JSONDecodeError:
            return {}
    return data if isinstance(data, dict) else {}


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
    """Cached options for a field class, or None."""
    e = load_cache(cache).get(make_key(arch, ndim, dtype, n))
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


class TunedContext:
    """A Context whose options follow the autotune cache per field class."""

    def __init__(self, device: int = 0, cache: Optional[str] = None, **options):
        from . import exactz
        self.ctx = exactz.Context(device, **options)
        self.cache = cache

    def correct(self, f, g_hat, xi, **kw):
        apply_options(self.ctx, f, self.cache)
        return self.ctx.correct(f, g_hat, xi, **kw)

    def close(self):
        self.ctx.close()
