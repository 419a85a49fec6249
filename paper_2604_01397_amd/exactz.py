"""ctypes binding of libexactz.so (include/exactz.h).

Argument marshalling only: every step of the correction runs in the HIP
library.  Tensors are torch CUDA (ROCm) tensors used as plain device
buffers; streams are torch streams.  There is no CPU fallback: without the
built library or a GPU every call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libexactz.so")

F32, F64 = 0, 1
REFORMULATED, ORIGINAL = 0, 1
OK, W_STUCK, W_MAX_ITERS = 0, 1, 2
E_INVALID, E_NONFINITE, E_BOUND, E_NOMEM, E_HIP, E_BUSY = -1, -2, -3, -4, -5, -6

EXPORTS = (
    "exz_ctx_create", "exz_ctx_destroy", "exz_ctx_set_option", "exz_ctx_bytes_in_use",
    "exz_workspace_bytes", "exz_workspace_bytes_k", "exz_correct", "exz_correct_host",
    "exz_correct_noalloc",
    "exz_correct_batch",
    "exz_job_create", "exz_job_submit", "exz_step", "exz_job_poll", "exz_job_query",
    "exz_job_release", "exz_job_bytes",
    "exz_status_string", "exz_last_error", "exz_debug_bounds", "exz_debug_targets",
)


class Params(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("dims", ctypes.c_int64 * 3), ("xi", ctypes.c_double),
                ("n_steps", ctypes.c_int32), ("event_mode", ctypes.c_int32),
                ("max_iters", ctypes.c_int64), ("certify", ctypes.c_int32),
                ("resume", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("edited_vertices", ctypes.c_int64),
                ("edit_ops", ctypes.c_int64), ("lossless_vertices", ctypes.c_int64),
                ("floor_vertices", ctypes.c_int64), ("residual_violations", ctypes.c_int64),
                ("num_critical", ctypes.c_int64), ("status", ctypes.c_int32),
                ("certified", ctypes.c_int32), ("setup_ms", ctypes.c_double),
                ("loop_ms", ctypes.c_double), ("check_launches", ctypes.c_int64),
                ("check_ms", ctypes.c_double), ("check_vertices", ctypes.c_int64),
                ("targets_total", ctypes.c_int64)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Field(ctypes.Structure):
    _fields_ = [("params", Params), ("f", ctypes.c_void_p), ("g_hat", ctypes.c_void_p),
                ("g_out", ctypes.c_void_p), ("cnt_io", ctypes.c_void_p)]


class ExactzError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("exactz status %d: %s" % (status, msg))
        self.status = status


_lib = None


def load(path: str | None = None):
    """Load libexactz.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError("libexactz.so not built: run __graft_entry__.build() (expected %s)" % path)
    # torch ships its own HIP runtime under the same soname; loading torch
    # first makes the library bind to that one copy (loaded the other way
    # round, the process holds two runtimes and only one of them sees the GPU)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(path)
    p, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.exz_ctx_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(p)]
    L.exz_ctx_bytes_in_use.argtypes = [p]
    L.exz_ctx_bytes_in_use.restype = ctypes.c_size_t
    L.exz_correct_host.argtypes = [p, p, p, p, p, ctypes.POINTER(Params), ctypes.POINTER(Result)]
    L.exz_correct_noalloc.argtypes = [p, p, p, p, p, ctypes.POINTER(Params),
                                      ctypes.POINTER(Result), p]
    L.exz_ctx_destroy.argtypes = [p]
    L.exz_ctx_set_option.argtypes = [p, ctypes.c_char_p, i64]
    L.exz_workspace_bytes.argtypes = [ctypes.POINTER(Params)]
    L.exz_workspace_bytes.restype = ctypes.c_size_t
    L.exz_workspace_bytes_k.argtypes = [ctypes.POINTER(Params), ctypes.c_int64]
    L.exz_workspace_bytes_k.restype = ctypes.c_size_t
    L.exz_correct.argtypes = [p, p, p, p, p, ctypes.POINTER(Params), ctypes.POINTER(Result), p]
    L.exz_correct_batch.argtypes = [p, ctypes.POINTER(Field), i32, ctypes.POINTER(Result), p]
    L.exz_job_create.argtypes = [p, ctypes.POINTER(Field), p, ctypes.POINTER(p)]
    L.exz_job_submit.argtypes = [p, ctypes.POINTER(Field), p, ctypes.POINTER(p)]
    L.exz_job_query.argtypes = [p, ctypes.POINTER(i32), ctypes.POINTER(Result)]
    L.exz_step.argtypes = [p, ctypes.POINTER(p), i32, i32, p]
    L.exz_job_poll.argtypes = [p, ctypes.POINTER(i32), ctypes.POINTER(Result)]
    L.exz_job_release.argtypes = [p]
    L.exz_job_bytes.argtypes = [ctypes.POINTER(Params)]
    L.exz_job_bytes.restype = ctypes.c_size_t
    L.exz_status_string.argtypes = [ctypes.c_int]
    L.exz_status_string.restype = ctypes.c_char_p
    L.exz_last_error.argtypes = [p]
    L.exz_last_error.restype = ctypes.c_char_p
    L.exz_debug_bounds.argtypes = [p, i32, p, i64, ctypes.c_double, p, p, p]
    L.exz_debug_targets.argtypes = [p, p, p, ctypes.POINTER(Params), p, ctypes.POINTER(i64), p]
    for name in ("exz_ctx_create", "exz_ctx_destroy", "exz_ctx_set_option", "exz_correct",
                 "exz_correct_host", "exz_correct_noalloc",
                 "exz_correct_batch", "exz_job_create", "exz_job_submit", "exz_step",
                 "exz_job_poll", "exz_job_query", "exz_job_release", "exz_debug_bounds",
                 "exz_debug_targets"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError("fields must be float32 or float64")


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_params(f, xi, n_steps=5, mode=REFORMULATED, max_iters=0, certify=False, resume=False):
    """Params for a C-ordered tensor f of shape ([nz,] [ny,] nx)."""
    p = Params()
    p.ndim = f.dim()
    p.dtype = _dtype_code(f)
    dims = list(reversed(f.shape)) + [1] * (3 - f.dim())
    for k in range(3):
        p.dims[k] = int(dims[k])
    p.xi = float(xi)
    p.n_steps = int(n_steps)
    p.event_mode = int(mode)
    p.max_iters = int(max_iters)
    p.certify = int(bool(certify))
    p.resume = int(bool(resume))
    return p


def _check_tensor(t, like=None):
    if not t.is_cuda:
        raise ValueError("tensors must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    if like is not None and (t.shape != like.shape or t.dtype != like.dtype or t.device != like.device):
        raise ValueError("shape/dtype/device mismatch")


class Context:
    """A library context on one device (owns the device workspace).

    ``budget`` caps the device bytes the context and its jobs may hold
    (0 = no cap); a call that would exceed it raises with E_NOMEM.
    """

    def __init__(self, device: int = 0, budget: int = 0, **options):
        self.lib = load()
        h = ctypes.c_void_p()
        st = self.lib.exz_ctx_create(int(device), int(budget), ctypes.byref(h))
        if st != OK:
            raise ExactzError(st, "exz_ctx_create failed")
        self.h = h
        self.device = device
        for k, v in options.items():
            self.set_option(k, v)

    def set_option(self, key, value):
        st = self.lib.exz_ctx_set_option(self.h, key.encode(), int(value))
        if st != OK:
            raise ExactzError(st, self.last_error())

    def last_error(self):
        return (self.lib.exz_last_error(self.h) or b"").decode()

    def bytes_in_use(self):
        """Device bytes the context and its live jobs hold (what the budget counts)."""
        return int(self.lib.exz_ctx_bytes_in_use(self.h))

    def close(self):
        if self.h:
            self.lib.exz_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def correct(self, f, g_hat, xi, n_steps=5, mode=REFORMULATED, max_iters=0,
                certify=False, g_out=None, cnt=None, resume=False, stream=None,
                raise_on_error=True):
        """Run the correction loop; returns (g_out, cnt, result dict).

        ``g_out`` may be ``g_hat`` (in place).  ``cnt`` (uint8, same shape)
        receives the per-vertex edit counts; with ``resume`` it holds the
        counts of an earlier call and ``g_hat`` the state that call left.
        """
        import torch
        _check_tensor(f)
        _check_tensor(g_hat, f)
        if g_out is None:
            g_out = torch.empty_like(f)
        _check_tensor(g_out, f)
        if cnt is None:
            cnt = torch.zeros(f.shape, dtype=torch.uint8, device=f.device)
        elif cnt.dtype != torch.uint8 or cnt.shape != f.shape:
            raise ValueError("cnt must be uint8 of f's shape")
        p = make_params(f, xi, n_steps, mode, max_iters, certify, resume)
        r = Result()
        st = self.lib.exz_correct(self.h, ctypes.c_void_p(f.data_ptr()),
                                  ctypes.c_void_p(g_hat.data_ptr()),
                                  ctypes.c_void_p(g_out.data_ptr()),
                                  ctypes.c_void_p(cnt.data_ptr()), ctypes.byref(p),
                                  ctypes.byref(r), _stream_ptr(stream))
        if st < 0 and raise_on_error:
            raise ExactzError(st, self.last_error())
        return g_out, cnt, r.to_dict()

    def correct_noalloc(self, f, g_hat, xi, n_steps=5, mode=REFORMULATED, max_iters=0,
                        certify=False, g_out=None, cnt=None, resume=False, stream=None,
                        raise_on_error=True):
        """exz_correct_noalloc: like correct(), but the library allocates nothing
        (its workspace is a static per-GPU buffer); the caller's tensors are
        allocated here, before the call."""
        import torch
        _check_tensor(f)
        _check_tensor(g_hat, f)
        if g_out is None:
            g_out = torch.empty_like(f)
        _check_tensor(g_out, f)
        if cnt is None:
            cnt = torch.zeros(f.shape, dtype=torch.uint8, device=f.device)
        elif cnt.dtype != torch.uint8 or cnt.shape != f.shape:
            raise ValueError("cnt must be uint8 of f's shape")
        p = make_params(f, xi, n_steps, mode, max_iters, certify, resume)
        r = Result()
        st = self.lib.exz_correct_noalloc(self.h, ctypes.c_void_p(f.data_ptr()),
                                          ctypes.c_void_p(g_hat.data_ptr()),
                                          ctypes.c_void_p(g_out.data_ptr()),
                                          ctypes.c_void_p(cnt.data_ptr()), ctypes.byref(p),
                                          ctypes.byref(r), _stream_ptr(stream))
        if st < 0 and raise_on_error:
            raise ExactzError(st, self.last_error())
        return g_out, cnt, r.to_dict()

    def correct_host(self, f, g_hat, xi, n_steps=5, mode=REFORMULATED, max_iters=0,
                     certify=False, cnt=None, resume=False, raise_on_error=True):
        """exz_correct_host on numpy arrays: returns (g_out, cnt, result dict)."""
        import numpy as np
        f = np.ascontiguousarray(f)
        g_hat = np.ascontiguousarray(g_hat)
        if f.dtype not in (np.float32, np.float64) or g_hat.dtype != f.dtype or g_hat.shape != f.shape:
            raise ValueError("f and g_hat must be float32/float64 arrays of one shape")
        g_out = np.empty_like(f)
        if cnt is None:
            cnt = np.zeros(f.shape, np.uint8)
        cnt = np.ascontiguousarray(cnt, dtype=np.uint8).copy()
        p = Params()
        p.ndim = f.ndim
        p.dtype = F32 if f.dtype == np.float32 else F64
        dims = list(reversed(f.shape)) + [1] * (3 - f.ndim)
        for k in range(3):
            p.dims[k] = int(dims[k])
        p.xi, p.n_steps, p.event_mode = float(xi), int(n_steps), int(mode)
        p.max_iters, p.certify, p.resume = int(max_iters), int(bool(certify)), int(bool(resume))
        r = Result()
        st = self.lib.exz_correct_host(self.h, f.ctypes.data, g_hat.ctypes.data, g_out.ctypes.data,
                                       cnt.ctypes.data, ctypes.byref(p), ctypes.byref(r))
        if st < 0 and raise_on_error:
            raise ExactzError(st, self.last_error())
        return g_out, cnt, r.to_dict()

    def correct_batch(self, items, stream=None, raise_on_error=False):
        """Correct many fields together.

        ``items``: list of dicts with keys f, g_hat, xi and optional n_steps,
        mode, max_iters, certify, g_out, cnt, resume.  Returns a list of
        (g_out, cnt, result dict) in the same order.
        """
        import torch
        n = len(items)
        arr = (Field * max(n, 1))()
        outs = []
        for k, it in enumerate(items):
            f, g = it["f"], it["g_hat"]
            _check_tensor(f)
            _check_tensor(g, f)
            g_out = it.get("g_out")
            if g_out is None:
                g_out = torch.empty_like(f)
            cnt = it.get("cnt")
            if cnt is None:
                cnt = torch.zeros(f.shape, dtype=torch.uint8, device=f.device)
            arr[k].params = make_params(f, it["xi"], it.get("n_steps", 5),
                                        it.get("mode", REFORMULATED), it.get("max_iters", 0),
                                        it.get("certify", False), it.get("resume", False))
            arr[k].f = f.data_ptr()
            arr[k].g_hat = g.data_ptr()
            arr[k].g_out = g_out.data_ptr()
            arr[k].cnt_io = cnt.data_ptr()
            outs.append((g_out, cnt))
        res = (Result * max(n, 1))()
        st = self.lib.exz_correct_batch(self.h, arr, n, res, _stream_ptr(stream))
        if st < 0 and raise_on_error:
            raise ExactzError(st, self.last_error())
        return [(outs[k][0], outs[k][1], res[k].to_dict()) for k in range(n)]

    # ------------------------------------------------------------------
    # serving primitives: jobs whose state stays on the device between steps

    def job_create(self, f, g_hat, xi, n_steps=5, max_iters=0, g_out=None, cnt=None,
                   stream=None):
        """Validate a field and build its reference topology; returns a Job.

        The job keeps references to its tensors until it is released.
        ``g_out`` may be ``g_hat`` (in place)."""
        return self._job("exz_job_create", f, g_hat, xi, n_steps, max_iters, g_out, cnt, stream)

    def job_submit(self, f, g_hat, xi, n_steps=5, max_iters=0, g_out=None, cnt=None,
                   stream=None):
        """job_create without waiting for the set-up (exz_job_submit): a bad
        field is reported later, by Job.query / Job.poll."""
        return self._job("exz_job_submit", f, g_hat, xi, n_steps, max_iters, g_out, cnt, stream)

    def _job(self, entry, f, g_hat, xi, n_steps, max_iters, g_out, cnt, stream):
        import torch
        _check_tensor(f)
        _check_tensor(g_hat, f)
        if g_out is None:
            g_out = torch.empty_like(f)
        _check_tensor(g_out, f)
        if cnt is None:
            cnt = torch.zeros(f.shape, dtype=torch.uint8, device=f.device)
        fl = Field()
        fl.params = make_params(f, xi, n_steps, REFORMULATED, max_iters)
        fl.f = f.data_ptr()
        fl.g_hat = g_hat.data_ptr()
        fl.g_out = g_out.data_ptr()
        fl.cnt_io = cnt.data_ptr()
        h = ctypes.c_void_p()
        st = getattr(self.lib, entry)(self.h, ctypes.byref(fl), _stream_ptr(stream),
                                      ctypes.byref(h))
        if st != OK:
            raise ExactzError(st, self.last_error())
        return Job(self, h, (f, g_hat, g_out, cnt))

    def step(self, jobs, iters=1, stream=None):
        """Advance every listed job by up to ``iters`` rounds (stream-ordered)."""
        n = len(jobs)
        if n == 0:
            return
        arr = (ctypes.c_void_p * n)(*[j.h for j in jobs])
        st = self.lib.exz_step(self.h, arr, n, int(iters), _stream_ptr(stream))
        if st != OK:
            raise ExactzError(st, self.last_error())

    def debug_bounds(self, f, xi, stream=None):
        import torch
        _check_tensor(f)
        L = torch.empty_like(f)
        U = torch.empty_like(f)
        st = self.lib.exz_debug_bounds(self.h, _dtype_code(f), ctypes.c_void_p(f.data_ptr()),
                                       f.numel(), float(xi), ctypes.c_void_p(L.data_ptr()),
                                       ctypes.c_void_p(U.data_ptr()), _stream_ptr(stream))
        if st != OK:
            raise ExactzError(st, self.last_error())
        return L, U

    def debug_targets(self, f, g, xi, n_steps=5, stream=None):
        import torch
        _check_tensor(f)
        _check_tensor(g, f)
        p = make_params(f, xi, n_steps)
        mark = torch.empty(f.shape, dtype=torch.uint8, device=f.device)
        cnt = ctypes.c_int64()
        st = self.lib.exz_debug_targets(self.h, ctypes.c_void_p(f.data_ptr()),
                                        ctypes.c_void_p(g.data_ptr()), ctypes.byref(p),
                                        ctypes.c_void_p(mark.data_ptr()), ctypes.byref(cnt),
                                        _stream_ptr(stream))
        if st != OK:
            raise ExactzError(st, self.last_error())
        return mark.bool(), cnt.value


class Job:
    """A correction job resident on the device (see Context.job_create)."""

    def __init__(self, ctx, handle, tensors):
        self.ctx = ctx
        self.h = handle
        self.f, self.g_hat, self.g_out, self.cnt = tensors

    def poll(self):
        """(done, result dict); waits for the work issued for this job."""
        return self._state("exz_job_poll")

    def query(self):
        """(done, result dict) after the job's latest step whose work has
        ended; never waits (exz_job_query)."""
        return self._state("exz_job_query")

    def _state(self, entry):
        done = ctypes.c_int32()
        r = Result()
        st = getattr(self.ctx.lib, entry)(self.h, ctypes.byref(done), ctypes.byref(r))
        if st != OK:
            raise ExactzError(st, self.ctx.last_error())
        return bool(done.value), r.to_dict()

    def release(self):
        if self.h:
            self.ctx.lib.exz_job_release(self.h)
            self.h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def job_bytes(shape_xyz, dtype=F32, xi=1e-3, n_steps=5):
    """exz_job_bytes: device workspace of a job on a (nx[, ny[, nz]]) field."""
    lib = load()
    p = Params()
    p.ndim = len(shape_xyz)
    p.dtype = dtype
    d = list(shape_xyz) + [1] * (3 - len(shape_xyz))
    for k in range(3):
        p.dims[k] = int(d[k])
    p.xi = xi
    p.n_steps = n_steps
    p.event_mode = REFORMULATED
    return int(lib.exz_job_bytes(ctypes.byref(p)))


def workspace_bytes(shape_xyz, dtype=F32, xi=1e-3, n_steps=5, mode=REFORMULATED, certify=False,
                    num_critical=None):
    """exz_workspace_bytes for a field of the given (nx[, ny[, nz]]) shape
    (exz_workspace_bytes_k when num_critical is given)."""
    lib = load()
    p = Params()
    p.ndim = len(shape_xyz)
    p.dtype = dtype
    d = list(shape_xyz) + [1] * (3 - len(shape_xyz))
    for k in range(3):
        p.dims[k] = int(d[k])
    p.xi = xi
    p.n_steps = n_steps
    p.event_mode = mode
    p.certify = int(certify)
    if num_critical is not None:
        return int(lib.exz_workspace_bytes_k(ctypes.byref(p), int(num_critical)))
    return int(lib.exz_workspace_bytes(ctypes.byref(p)))


_default_ctx = {}


def default_context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def correct(f, g_hat, xi, **kw):
    """Module-level convenience: correct(f, g_hat, xi) -> (g_out, cnt, result)."""
    return default_context(f.device.index or 0).correct(f, g_hat, xi, **kw)
