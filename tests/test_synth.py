"""The seeded input generators draw what their docstrings state."""
import numpy as np

from paper_1705_06284_amd import synth


def test_gaussian_field_variance_and_spectrum_slope():
    g = synth.gaussian_field(32, 2.0, 0.7, 1)
    assert abs(g.mean()) < 1e-12 and np.isclose(g.std(), 0.7)
    G = np.abs(np.fft.fftn(g)) ** 2
    f = np.fft.fftfreq(32, 1 / 32)
    r = np.sqrt(f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2)
    p1 = G[(r >= 2) & (r < 3)].mean()
    p2 = G[(r >= 8) & (r < 9)].mean()
    assert 0.5 < (p1 / p2) / ((8.5 / 2.5) ** 2) < 2.0        # P ~ k^-2


def test_lognormal_and_seeds():
    a = synth.lognormal_field(16, 1.5, 1.0, 2)
    b = synth.lognormal_field(16, 1.5, 1.0, 2)
    c = synth.lognormal_field(16, 1.5, 1.0, 3)
    assert a.dtype == np.float32 and np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() > -1.0


def test_toy_bubbles_fraction():
    d, st = synth.toy_bubbles(64, 4.0, 0.5, 3, return_stats=True)
    assert d.dtype == np.float32
    assert 0.5 <= st["ionized_fraction"] < 0.55
    vals = np.unique(np.round(d, 5))
    assert len(vals) == 2                                      # binary x_HI, mean removed


def test_bins():
    lo, hi = synth.linear_bins(128, 16)
    assert lo[0] == 0 and hi[-1] == 64 and np.allclose(hi - lo, 4)
    lo, hi = synth.unit_bins(1, 8)
    assert np.allclose(lo, np.arange(1, 9) - 0.5)
