"""The synthetic inputs are inside the error band and have the stated shapes."""
import numpy as np
import pytest

from paper_2604_01397_amd import synth


def _in_band(f, g, eps):
    return np.all(np.abs(g.astype(np.float64) - f.astype(np.float64)) <= eps)


def test_config0_shape_and_band():
    c = synth.config0()
    assert c.f.shape == (256, 256) and c.f.dtype == np.float32
    assert _in_band(c.f, c.g_hat, c.xi)
    assert np.float32(c.xi) == c.xi  # representable in the field dtype
    rng = float(c.f.max()) - float(c.f.min())
    assert c.xi <= 1e-3 * rng < c.xi * (1 + 1e-6)


@pytest.mark.parametrize("quant", ["uniform", "lorenzo"])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_grf_quantizers_band(quant, dtype):
    c = synth.case_grf3d(24, seed=5, slope=-11 / 3, rel=1e-3, quantizer=quant, dtype=dtype)
    assert c.f.shape == (24, 24, 24) and c.f.dtype == dtype
    assert abs(float(c.f.mean())) < 1e-5 and abs(float(c.f.std()) - 1) < 1e-4
    assert _in_band(c.f, c.g_hat, c.xi)
    assert np.any(c.g_hat != c.f)


def test_lorenzo_stays_on_the_quantisation_lattice():
    # The 7-point Lorenzo stencil has integer weights, so a prediction from
    # reconstructed values (all multiples of 2*eps) is itself a multiple of
    # 2*eps and p + 2*eps*round((f - p)/(2*eps)) = 2*eps*round(f/(2*eps)):
    # the reconstruction equals the uniform quantiser's up to rounding.
    a = synth.case_grf3d(16, seed=2, slope=-3, rel=1e-2, quantizer="uniform")
    b = synth.case_grf3d(16, seed=2, slope=-3, rel=1e-2, quantizer="lorenzo")
    assert np.array_equal(a.f, b.f)
    assert np.mean(a.g_hat != b.g_hat) < 1e-3


def test_generators_are_seeded():
    a = synth.case_gauss2d(64, seed=3)
    b = synth.case_gauss2d(64, seed=3)
    assert np.array_equal(a.f, b.f) and np.array_equal(a.g_hat, b.g_hat)


def test_batched_specs():
    specs = synth.config3_specs()
    assert len(specs) == 96
    assert {s["ndim"] for s in specs} == {2, 3}
    for s in specs:
        lo, hi = (128, 2048) if s["ndim"] == 2 else (32, 256)
        assert lo <= s["edge"] <= hi
        assert s["rel"] in (1e-2, 1e-3, 1e-4)
    n64 = sum(s["dtype"] == np.float64 for s in specs)
    assert 5 <= n64 <= 40


def test_serving_specs():
    specs = synth.config4_specs(njobs=1000)
    t = np.array([s["arrival"] for s in specs])
    assert np.all(np.diff(t) >= 0)
    assert 3.5 < len(t) / t[-1] / 50 < 4.5  # ~200 jobs/s
    assert all(66 <= s["edge"] <= 1026 for s in specs)
