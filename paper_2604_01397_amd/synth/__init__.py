"""Seeded synthetic inputs (f, g_hat, xi) for the correction loop.

The paper evaluates on simulation outputs compressed by SZ3/ZFP/cuSZp/...; none
of those are available, so these generators stand in for them with fields of
the same shapes, spectra and error structure:

* ``gaussians2d`` -- sum of random 2D Gaussians plus white noise;
* ``grf3d`` -- isotropic Gaussian random field with power spectrum P(k) ~ k^slope;
* ``quantize_uniform`` -- mid-tread uniform quantiser with bin width 2*eps;
* ``quantize_lorenzo`` -- Lorenzo predictor + bin-2*eps residual quantiser
  (SZ-like, spatially correlated errors).

Every decompressed field satisfies |f - g_hat| <= eps exactly (checked in
float64 arithmetic, in which the difference of two float32 values is exact).
``eps`` is returned as a value representable in the field dtype, so that the
error bound handed to the correction loop is the same number in both
precisions.

This module holds no part of the correction method; both the GPU path and the
CPU oracle consume its outputs.  Arrays are C-ordered (z, y, x): x is the
fastest index, matching vertex index i = x + nx*(y + ny*z).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LORENZO_SO = os.path.join(_HERE, "_lorenzo.so")


def build_lorenzo(force: bool = False) -> str:
    """Compile the Lorenzo quantiser helper (plain C, host only)."""
    src = os.path.join(_HERE, "lorenzo.c")
    if force or not os.path.exists(_LORENZO_SO) or (
        os.path.getmtime(_LORENZO_SO) < os.path.getmtime(src)
    ):
        tmp = _LORENZO_SO + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", src, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LORENZO_SO)
    return _LORENZO_SO


_lorenzo_lib = None


def _lorenzo():
    global _lorenzo_lib
    if _lorenzo_lib is None:
        if not os.path.exists(_LORENZO_SO):
            build_lorenzo()
        lib = ctypes.CDLL(_LORENZO_SO)
        lib.synth_lorenzo3d.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_int64, ctypes.c_double,
        ]
        lib.synth_lorenzo3d.restype = None
        _lorenzo_lib = lib
    return _lorenzo_lib


# ----------------------------------------------------------------------------
# fields


def gaussians2d(nx: int, ny: int, seed: int, n_gauss: int = 32,
                sigma=(4.0, 24.0), noise: float = 0.01,
                dtype=np.float32) -> np.ndarray:
    """Sum of ``n_gauss`` random Gaussians A*exp(-r^2/(2 sigma^2)) + N(0, noise^2).

    Centres are uniform over the domain, sigma uniform in ``sigma`` (pixels),
    amplitudes +-U[0.5, 1] with a fair sign.  Returned shape (ny, nx).
    """
    rng = np.random.default_rng(seed)
    cx = rng.uniform(0, nx, n_gauss)
    cy = rng.uniform(0, ny, n_gauss)
    sg = rng.uniform(sigma[0], sigma[1], n_gauss)
    amp = rng.uniform(0.5, 1.0, n_gauss) * np.where(rng.random(n_gauss) < 0.5, -1.0, 1.0)
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    f = np.zeros((ny, nx), dtype=np.float64)
    for k in range(n_gauss):
        r2 = (x - cx[k]) ** 2 + (y - cy[k]) ** 2
        f += amp[k] * np.exp(-r2 / (2.0 * sg[k] ** 2))
    f += rng.normal(0.0, noise, size=(ny, nx))
    return f.astype(dtype)


def grf3d(n: int | tuple, seed: int, slope: float, dtype=np.float32,
          workers: int | None = None) -> np.ndarray:
    """Periodic Gaussian random field with P(k) ~ |k|^slope, zero mean, unit variance.

    White N(0,1) noise is filtered in Fourier space by sqrt(P(|k|)) with k in
    integer cycles per box and P(0) = 0.  ``n`` is an edge or (nz, ny, nx).
    """
    import scipy.fft as sfft

    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape, dtype=np.float32)
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    W = sfft.rfftn(w, workers=workers)
    del w
    kz = np.fft.fftfreq(shape[0]) * shape[0]
    ky = np.fft.fftfreq(shape[1]) * shape[1]
    kx = np.fft.rfftfreq(shape[2]) * shape[2]
    k2 = (kz[:, None] ** 2 + ky[None, :] ** 2).astype(np.float32)
    for ix in range(kx.shape[0]):
        kk = k2 + np.float32(kx[ix] ** 2)
        with np.errstate(divide="ignore"):
            amp = np.where(kk > 0, kk ** np.float32(slope / 4.0), np.float32(0.0))
        W[:, :, ix] *= amp
    f = sfft.irfftn(W, s=shape, workers=workers)
    del W
    f = f.astype(np.float64)
    f -= f.mean()
    sd = f.std()
    if sd > 0:
        f /= sd
    return f.astype(dtype)


# ----------------------------------------------------------------------------
# error bound and quantisers


def eps_for(f: np.ndarray, rel: float) -> float:
    """rel * (max f - min f), rounded down to a value of f's dtype (float)."""
    lo = float(np.min(f))
    hi = float(np.max(f))
    e = rel * (hi - lo)
    if f.dtype == np.float32:
        e32 = np.float32(e)
        if float(e32) > e:
            e32 = np.nextafter(e32, np.float32(0))
        return float(e32)
    return float(e)


def _enforce_band(f: np.ndarray, g: np.ndarray, eps: float) -> np.ndarray:
    """Move g one ulp towards f wherever |g - f| > eps (exact for float32)."""
    if f.dtype == np.float32:
        for _ in range(8):
            d = g.astype(np.float64) - f.astype(np.float64)
            bad = np.abs(d) > eps
            if not bad.any():
                return g
            g[bad] = np.nextafter(g[bad], f[bad])
        raise RuntimeError("band enforcement did not converge")
    # float64: the quantisers used a bin shrunk by 2^-20, so the computed
    # difference plus its rounding error stays well inside the band.
    d = np.abs(g - f)
    if not np.all(d <= eps * (1.0 - 2.0 ** -21)):
        raise RuntimeError("float64 quantiser left the band")
    return g


def _bin(eps: float, dtype) -> float:
    return 2.0 * eps * (1.0 - 2.0 ** -20) if dtype == np.float64 else 2.0 * eps


def quantize_uniform(f: np.ndarray, eps: float) -> np.ndarray:
    """Mid-tread uniform quantiser, bin 2*eps, ties to even, in float64."""
    b = _bin(eps, f.dtype)
    q = np.rint(f.astype(np.float64) / b) * b
    g = q.astype(f.dtype)
    return _enforce_band(f, g, eps)


def quantize_lorenzo(f: np.ndarray, eps: float) -> np.ndarray:
    """3D Lorenzo predictor on reconstructed values + bin-2*eps residual quantiser."""
    f3 = f.reshape((1,) * (3 - f.ndim) + f.shape)
    nz, ny, nx = f3.shape
    src = np.ascontiguousarray(f3, dtype=np.float64)
    out = np.empty_like(src)
    _lorenzo().synth_lorenzo3d(src.ctypes.data, out.ctypes.data, nx, ny, nz,
                               _bin(eps, f.dtype) / 2.0)
    g = out.astype(f.dtype).reshape(f.shape)
    return _enforce_band(f, g, eps)


# ----------------------------------------------------------------------------
# the workloads


@dataclass
class Case:
    """One correction problem: original f, decompressed g_hat, absolute bound xi."""
    name: str
    f: np.ndarray
    g_hat: np.ndarray
    xi: float
    meta: dict = field(default_factory=dict)

    @property
    def dims(self):
        return tuple(reversed(self.f.shape))  # (nx, ny[, nz])

    @property
    def ndim(self):
        return self.f.ndim


def case_gauss2d(n: int = 256, seed: int = 0, rel: float = 1e-3, dtype=np.float32,
                 ny: int | None = None) -> Case:
    """2D Gaussians + noise, uniform quantiser (the 256x256 float32 workload)."""
    ny = n if ny is None else ny
    scale = max(n, ny) / 256.0
    f = gaussians2d(n, ny, seed, sigma=(4.0 * scale, 24.0 * scale), dtype=dtype)
    eps = eps_for(f, rel)
    return Case(f"gauss2d_{n}x{ny}_s{seed}", f, quantize_uniform(f, eps), eps,
                {"rel": rel, "quantizer": "uniform"})


def case_grf3d(n: int = 128, seed: int = 1, slope: float = -3.0, rel: float = 1e-3,
               quantizer: str = "uniform", dtype=np.float32) -> Case:
    """3D GRF, P(k) ~ k^slope, uniform or Lorenzo quantiser."""
    f = grf3d(n, seed, slope, dtype=dtype)
    eps = eps_for(f, rel)
    g = quantize_uniform(f, eps) if quantizer == "uniform" else quantize_lorenzo(f, eps)
    edge = n if np.isscalar(n) else "x".join(str(v) for v in reversed(n))
    return Case(f"grf3d_{edge}_k{slope:g}_{quantizer}_s{seed}", f, g, eps,
                {"rel": rel, "quantizer": quantizer, "slope": slope})


def config0() -> Case:
    """2D float32 256x256, 32 Gaussians + N(0, 0.01) noise, eps = 1e-3 range."""
    return case_gauss2d(256, seed=0, rel=1e-3)


def config1() -> Case:
    """3D float32 128^3 GRF k^-3, uniform quantiser, eps = 1e-3 range."""
    return case_grf3d(128, seed=1, slope=-3.0, rel=1e-3, quantizer="uniform")


def config2(edge: int = 512) -> Case:
    """3D float32 512^3 GRF k^-11/3, Lorenzo quantiser, eps = 1e-4 range."""
    return case_grf3d(edge, seed=2, slope=-11.0 / 3.0, rel=1e-4, quantizer="lorenzo")


def config3_specs(nfields: int = 96, seed: int = 3):
    """Shapes/dtypes/bounds of the 96-field batched workload (no data)."""
    rng = np.random.default_rng(seed)
    specs = []
    for j in range(nfields):
        is2d = rng.random() < 0.5
        if is2d:
            edge = int(round(math.exp(rng.uniform(math.log(128), math.log(2048)))))
        else:
            edge = int(round(math.exp(rng.uniform(math.log(32), math.log(256)))))
        dtype = np.float32 if rng.random() < 0.8 else np.float64
        rel = [1e-2, 1e-3, 1e-4][int(rng.integers(0, 3))]
        specs.append({"j": j, "ndim": 2 if is2d else 3, "edge": edge,
                      "dtype": dtype, "rel": rel, "seed": 3000 + j})
    return specs


def config3_field(spec: dict) -> Case:
    if spec["ndim"] == 2:
        c = case_gauss2d(spec["edge"], seed=spec["seed"], rel=spec["rel"], dtype=spec["dtype"])
    else:
        c = case_grf3d(spec["edge"], seed=spec["seed"], slope=-3.0, rel=spec["rel"],
                       quantizer="uniform", dtype=spec["dtype"])
    c.name = f"batch{spec['j']:02d}_" + c.name
    return c


def config4_specs(njobs: int = 1000, rate: float = 200.0, seed: int = 4,
                  lo: int = 64, hi: int = 1024):
    """Poisson arrival times and block edges L (log-uniform) of the serving trace.

    Each job is an (L+2)^3 float32 block (1-voxel ghost layer) with GRF k^-3
    content, eps = 1e-3 range, seed 4000 + j.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, njobs)
    t = np.cumsum(gaps) - gaps[0]
    edges = np.exp(rng.uniform(math.log(lo), math.log(hi), njobs)).round().astype(int)
    return [{"j": j, "arrival": float(t[j]), "edge": int(edges[j]) + 2,
             "seed": 4000 + j, "rel": 1e-3} for j in range(njobs)]


def config4_source(edge: int = 1024, seed: int = 4) -> np.ndarray:
    """The periodic volume the serving jobs are cut from: GRF k^-3, float32,
    edge^3, synthesised on the host (so every job's input can be rebuilt on
    the CPU bit for bit)."""
    return grf3d(edge, seed, -3.0, dtype=np.float32)


def config4_offsets(spec: dict, src_edge: int = 1024):
    """(z, y, x) corner of job spec's block in the periodic source volume."""
    return [int(v) for v in np.random.default_rng(spec["seed"]).integers(0, src_edge, 3)]


def config4_job(source: np.ndarray, spec: dict) -> Case:
    """Job spec's (L+2)^3 block (wrapping around the periodic source), its
    eps = rel * range of the block and the uniform quantisation."""
    e = spec["edge"]
    n = source.shape[0]
    idx = [(np.arange(e) + o) % n for o in config4_offsets(spec, n)]
    f = np.ascontiguousarray(source[np.ix_(idx[0], idx[1], idx[2])])
    eps = eps_for(f, spec["rel"])
    return Case("job%04d_%d" % (spec["j"], e), f, quantize_uniform(f, eps), eps,
                {"rel": spec["rel"], "quantizer": "uniform", "edge": e})


def config4_job_device(source, spec: dict):
    """config4_job() on a device copy of the source volume: the same block,
    eps and quantisation bit for bit (exact min / max, the same rounding).
    Returns (f, g_hat, eps)."""
    import torch
    e = spec["edge"]
    n = source.shape[0]
    off = config4_offsets(spec, n)
    idx = [(torch.arange(e, device=source.device) + o) % n for o in off]
    f = source.index_select(0, idx[0]).index_select(1, idx[1]).index_select(2, idx[2])
    f = f.contiguous()
    eps = eps_for_device(f, spec["rel"])
    return f, quantize_uniform_device(f, eps), eps


# ----------------------------------------------------------------------------
# device-side generation for the serving workload (blocks appear in HBM, as
# an in-situ simulation would leave them); same rules as the host versions


def grf3d_device(n: int, seed: int, slope: float, device="cuda:0"):
    """Periodic GRF (P(k) ~ |k|^slope, zero mean, unit variance) of edge n,
    float32, synthesised on the device with torch's FFT (seeded)."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    w = torch.randn((n, n, n), generator=gen, device=device, dtype=torch.float32)
    W = torch.fft.rfftn(w)
    del w
    k = torch.fft.fftfreq(n, d=1.0 / n, device=device, dtype=torch.float32)
    kx = torch.fft.rfftfreq(n, d=1.0 / n, device=device, dtype=torch.float32)
    for iz in range(n):  # one plane at a time keeps the temporaries small
        kk = k[iz] ** 2 + k[:, None] ** 2 + kx[None, :] ** 2
        amp = torch.where(kk > 0, kk.clamp_min(1e-30) ** (slope / 4.0), torch.zeros_like(kk))
        W[iz] *= amp
    f = torch.fft.irfftn(W, s=(n, n, n))
    del W
    f -= f.mean(dtype=torch.float64).to(torch.float32)
    sd = f.std()
    if sd > 0:
        f /= sd
    return f.contiguous()


def eps_for_device(f, rel: float) -> float:
    """eps_for() of a device tensor: rel * range, rounded down to f's dtype."""
    import torch

    lo = float(f.min().double())
    hi = float(f.max().double())
    e = rel * (hi - lo)
    if f.dtype == torch.float32:
        e32 = np.float32(e)
        if float(e32) > e:
            e32 = np.nextafter(e32, np.float32(0))
        return float(e32)
    return e


def quantize_uniform_device(f, eps: float, checked: bool = True):
    """quantize_uniform() of a float32 device tensor (same rounding, same band
    enforcement: |g - f| <= eps exactly).

    With ``checked=False`` nothing waits for the device: two rounds of band
    enforcement run unconditionally (a round that finds nothing outside the
    band changes nothing, so the result equals the checked one whenever two
    rounds suffice, which one ulp of float32 rounding always does; a value
    still outside the band would be rejected by the library's validation).

    The arithmetic is elementwise; it runs over chunks of 2^25 values, so
    its float64 temporaries stay small whatever the block size."""
    import torch

    if f.dtype != torch.float32:
        raise TypeError("device quantiser handles float32 blocks")
    # the bin as a device tensor: torch divides by a Python scalar through its
    # reciprocal, which can round differently from numpy's true division
    b = torch.full((), 2.0 * eps, dtype=torch.float64, device=f.device)
    flat = f.reshape(-1)
    out = torch.empty_like(flat)
    chunk = 1 << 25
    for k0 in range(0, flat.numel(), chunk):
        fc = flat[k0:k0 + chunk]
        fd = fc.double()
        g = (torch.round(fd / b) * b).to(torch.float32)  # round half to even, as np.rint
        for _ in range(8 if checked else 2):
            bad = (g.double() - fd).abs() > eps
            if checked and not bool(bad.any()):
                break
            g = torch.where(bad, torch.nextafter(g, fc), g)
        else:
            if checked:
                raise RuntimeError("band enforcement did not converge")
        out[k0:k0 + chunk] = g
    return out.reshape(f.shape)
