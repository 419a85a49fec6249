"""Edit stream: the decompressor's rebuild of g' from g_hat, Delta and the
stream equals the corrected field bit for bit (oracle corrections with many
(N+1)-th edits), and the sizes add up."""
import numpy as np
import pytest

import oracle
from paper_2604_01397_amd import editcodec, synth


def _bits(a):
    return a.view(np.uint32 if a.dtype == np.float32 else np.uint64)


@pytest.mark.parametrize("make,n_steps", [
    (lambda: synth.case_grf3d(24, seed=81, rel=1e-3), 2),
    (lambda: synth.case_grf3d(20, seed=82, rel=1e-4, quantizer="lorenzo"), 5),
    (lambda: synth.case_gauss2d(64, seed=83, rel=1e-3, dtype=np.float64), 3),
])
def test_round_trip(make, n_steps):
    c = make()
    g_out, cnt, st, _ = oracle.correct(c.f, c.g_hat, c.xi, n_steps=n_steps)
    d = editcodec.step(c.xi, c.f.dtype, n_steps)
    es = editcodec.encode(c.g_hat, g_out, cnt, d, n_steps)
    assert es.edited == int(np.count_nonzero(cnt)) == st["edited_vertices"]
    # every (N+1)-th edit is stored exactly (it holds the lower bound)
    assert es.exact >= int(np.count_nonzero(cnt == n_steps + 1))
    assert es.value_bytes == es.exact * c.f.itemsize
    assert len(es.data) == editcodec._HEADER.size + es.record_bytes + es.value_bytes
    g2, cnt2 = editcodec.decode(es.data, c.g_hat, d)
    assert np.array_equal(_bits(g2), _bits(g_out.ravel()))
    assert np.array_equal(cnt2, cnt.ravel())
    assert 0 < es.compressed() <= len(es.data) + 64


def test_no_edits_and_varints():
    g = np.linspace(0, 1, 50, dtype=np.float32)
    es = editcodec.encode(g, g, np.zeros(50, np.uint8), np.float32(0.01), 5)
    assert es.edited == 0 and es.exact == 0 and len(es.data) == editcodec._HEADER.size
    g2, c2 = editcodec.decode(es.data, g, np.float32(0.01))
    assert np.array_equal(g2, g) and not c2.any()
    v = np.array([0, 1, 127, 128, 300, 2 ** 35 + 7], dtype=np.uint64)
    out, pos = editcodec._read_varints(editcodec._varints(v), v.size, 0)
    assert np.array_equal(out, v)


def test_step_matches_band_rounding():
    # xi_T is the largest float32 not above xi; Delta rounds xi_T / N
    xi = 0.1
    d = editcodec.step(xi, np.float32, 5)
    x = np.float32(xi)
    x = np.nextafter(x, np.float32(-np.inf)) if float(x) > xi else x
    assert float(x) <= xi and d == np.float32(x / np.float32(5))
    assert editcodec.step(xi, np.float64, 4) == 0.1 / 4
