"""TEST INFRASTRUCTURE ONLY -- Python access to the CPU oracle and checker.

The oracle (``exactz_oracle.cpp``) is a plain, sequential C++ rendering of the
EXaCTz correction loop (Algorithm 1 with the constraint checks of Secs. 4.1-4.3
and the monotone edit of Sec. 3.3).  It exists so that the GPU library can be
compared with something obviously correct.  Only ``tests/``, the smoke check
in ``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import
this package; the library itself never does.

``checker.py`` holds brute-force topology (union-find merge trees, contour
tree, extremum graph, vulnerability graph) used to pin the oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "exactz_oracle.cpp")
_SO = os.path.join(_HERE, "_exactz_oracle.so")

REFORMULATED, ORIGINAL = 0, 1
OK, STUCK, MAX_ITERS = 0, 1, 2
E_INVALID, E_NONFINITE, E_BOUND = -1, -2, -3
TYPE_REGULAR, TYPE_MIN, TYPE_MAX, TYPE_SADDLE = 0, 1, 2, 3

STAT_KEYS = ("iterations", "edited_vertices", "edit_ops", "lossless_vertices",
             "floor_vertices", "residual_violations", "num_critical", "status")


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (-O2, no FMA contraction, rounding-mode aware)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-ffp-contract=off",
                               "-frounding-math", "-fno-fast-math", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        # EXACTZ_ORACLE_SO lets the mutation test load a deliberately broken
        # copy of the oracle to show that the pins catch it.
        path = os.environ.get("EXACTZ_ORACLE_SO") or _SO
        if path == _SO and not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(path)
        p, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.oref_correct.argtypes = [i32, p, i32, p, p, p, p, i32, d, i32, i32, i64,
                                   ctypes.c_uint64, p, i64, p]
        L.oref_correct.restype = i32
        L.oref_targets.argtypes = [i32, p, i32, p, p, i32, p]
        L.oref_targets.restype = i64
        L.oref_topology.argtypes = [i32, p, i32, p, p, p, p, p, p, p]
        L.oref_topology.restype = i32
        L.oref_critical_order.argtypes = [i32, p, i32, p, p, i64]
        L.oref_critical_order.restype = i64
        L.oref_offsets.argtypes = [i32, p]
        L.oref_offsets.restype = i32
        L.oref_bounds.argtypes = [i32, i64, p, d, i32, p, p, p, p]
        L.oref_bounds.restype = i32
        _lib = L
    return _lib


def _dtype_code(a: np.ndarray) -> int:
    if a.dtype == np.float32:
        return 0
    if a.dtype == np.float64:
        return 1
    raise TypeError("oracle fields must be float32 or float64")


def _dims(f: np.ndarray):
    d = list(reversed(f.shape)) + [1] * (3 - f.ndim)
    return np.array(d, dtype=np.int64), f.ndim


def _ptr(a):
    return a.ctypes.data if a is not None else None


def correct(f, g_hat, xi, n_steps=5, mode=REFORMULATED, max_iters=0, cnt=None,
            shuffle_seed=0, trace_cap=0):
    """Run the oracle loop.  Returns (g_out, cnt, stats dict, trace array or None).

    ``cnt`` (uint8, same shape) resumes from earlier edit counts; ``g_hat`` is
    then the current state.
    """
    f = np.ascontiguousarray(f)
    g_hat = np.ascontiguousarray(g_hat, dtype=f.dtype)
    assert f.shape == g_hat.shape
    dims, ndim = _dims(f)
    g_out = np.empty_like(f)
    resume = cnt is not None
    c = np.ascontiguousarray(cnt, dtype=np.uint8).copy() if resume else np.zeros(f.shape, np.uint8)
    stats = np.zeros(8, np.int64)
    trace = np.zeros(2 * trace_cap, np.int64) if trace_cap else None
    lib().oref_correct(ndim, dims.ctypes.data, _dtype_code(f), f.ctypes.data,
                       g_hat.ctypes.data, g_out.ctypes.data, c.ctypes.data, int(resume),
                       float(xi), int(n_steps), int(mode), int(max_iters),
                       int(shuffle_seed), _ptr(trace), int(trace_cap), stats.ctypes.data)
    st = dict(zip(STAT_KEYS, (int(v) for v in stats)))
    if trace is not None:
        trace = trace.reshape(-1, 2)[: min(trace_cap, st["iterations"] + (st["status"] == STUCK))]
    return g_out, c, st, trace


def targets(f, g, mode=REFORMULATED):
    """One CheckConstraints pass: boolean array of vertices to decrease."""
    f = np.ascontiguousarray(f)
    g = np.ascontiguousarray(g, dtype=f.dtype)
    dims, ndim = _dims(f)
    mark = np.zeros(f.shape, np.uint8)
    r = lib().oref_targets(ndim, dims.ctypes.data, _dtype_code(f), f.ctypes.data,
                           g.ctypes.data, int(mode), mark.ctypes.data)
    if r < 0:
        raise ValueError("bad arguments")
    return mark.astype(bool)


def topology(h):
    """Per-vertex asc, desc (flat vertex ids), lower mask, lc, uc, type."""
    h = np.ascontiguousarray(h)
    dims, ndim = _dims(h)
    n = h.size
    asc = np.zeros(n, np.int64)
    desc = np.zeros(n, np.int64)
    lower = np.zeros(n, np.uint32)
    lc = np.zeros(n, np.int8)
    uc = np.zeros(n, np.int8)
    ty = np.zeros(n, np.int8)
    lib().oref_topology(ndim, dims.ctypes.data, _dtype_code(h), h.ctypes.data,
                        asc.ctypes.data, desc.ctypes.data, lower.ctypes.data,
                        lc.ctypes.data, uc.ctypes.data, ty.ctypes.data)
    return {"asc": asc, "desc": desc, "lower": lower, "lc": lc, "uc": uc, "type": ty}


def critical_order(h):
    h = np.ascontiguousarray(h)
    dims, ndim = _dims(h)
    out = np.zeros(h.size, np.int64)
    k = lib().oref_critical_order(ndim, dims.ctypes.data, _dtype_code(h), h.ctypes.data,
                                  out.ctypes.data, h.size)
    return out[:k].copy()


def offsets(ndim):
    out = np.zeros(3 * 26, np.int32)
    k = lib().oref_offsets(ndim, out.ctypes.data)
    return out[: 3 * k].reshape(k, 3)


def bounds(f, xi, n_steps=5):
    """(L, U, xi_T, Delta) as the oracle computes them."""
    f = np.ascontiguousarray(f)
    L = np.empty_like(f)
    U = np.empty_like(f)
    xiT = ctypes.c_double()
    dl = ctypes.c_double()
    lib().oref_bounds(_dtype_code(f), f.size, f.ctypes.data, float(xi), int(n_steps),
                      L.ctypes.data, U.ctypes.data, ctypes.byref(xiT), ctypes.byref(dl))
    return L, U, xiT.value, dl.value
