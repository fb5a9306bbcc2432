"""Pins of the ionised-sphere model (oracle/toymodel.py; Section 3.3,
Eqs. BharPk and BharBk) and of its bin averages.

* W is the Fourier transform of the unit top hat: checked against the radial
  integral evaluated by quadrature, its first zero tan x = x and its series.
* The bin average over closed triangles (FFT form on the model spectrum)
  equals a brute-force average over closed mode triples on small grids.
* The model itself: P and B follow from the window with the stated powers of
  the ionised fraction and the sphere density.
"""
import numpy as np
import pytest
from scipy import integrate, optimize

import oracle
from oracle import toymodel


def test_window_is_the_top_hat_transform():
    R = 1.7
    for k in (1e-4, 0.05, 0.29, 0.3, 0.9, 2.3, 4.0, 7.5):
        # (3 / (4 pi R^3)) int_0^R 4 pi r^2 sin(kr) / (kr) dr
        v, _ = integrate.quad(lambda r: r * r * np.sin(k * r) / (k * r), 0.0, R, epsabs=1e-14, epsrel=1e-13)
        assert toymodel.window(k * R) == pytest.approx(3.0 * v / R ** 3, rel=1e-10, abs=1e-13)


def test_window_first_zero_and_series():
    x0 = optimize.brentq(lambda x: np.tan(x) - x, 4.0, 4.6)
    assert abs(toymodel.window(x0)) < 1e-12
    assert toymodel.window(0.0) == 1.0
    x = 1e-3
    assert toymodel.window(x) == pytest.approx(1.0 - x ** 2 / 10.0 + x ** 4 / 280.0, rel=1e-15)
    # both sides of the switch from the series to the closed form
    R = 1.0
    for k in (0.4999999, 0.5000001):
        v, _ = integrate.quad(lambda r: r * r * np.sin(k * r) / (k * r), 0.0, R, epsabs=1e-14, epsrel=1e-13)
        assert toymodel.window(k) == pytest.approx(3.0 * v, rel=1e-12)


def test_model_powers():
    R, nbar, x = 10.0, 2e-6, 0.01
    k = np.array([0.01, 0.2, 0.3])           # k R below the first zero of W
    w = toymodel.window(k * R)
    assert np.allclose(toymodel.power(k, R, nbar, x), x * x * w * w / nbar, rtol=1e-14)
    b = toymodel.bispectrum(k[0], k[1], k[2], R, nbar, x)
    assert b == pytest.approx(-(x ** 3) * np.prod(w) / nbar ** 2, rel=1e-14)
    assert b < 0        # a neutral field punctured by spheres: negative skewness


@pytest.mark.parametrize("shape,L", [((16, 16, 16), 16.0), ((12, 16, 20), 30.0)])
def test_bin_averages_match_brute_force(shape, L):
    R = 1.5 * L / shape[2]
    lo = np.array([1.0, 2.5, 4.0])
    hi = np.array([2.5, 4.0, 6.0])
    trip = np.array([(0, 0, 0), (0, 1, 1), (0, 1, 2), (1, 1, 2)])
    w2, www, cnt = toymodel.binned_window_moments(shape, lo, hi, L, R, trip)
    # brute force: direct sum over closed triples of the real spectrum W(|k| R)
    kk = toymodel.kmod_grid(shape, L)
    W = toymodel.window(kk * R)
    res = oracle.bispectrum(np.zeros(shape, np.float32), lo, hi, trip, box_len=L, delta_k=W.astype(complex))
    assert np.array_equal(cnt.astype(np.int64), res.count)
    assert np.allclose(www, res.s.real / res.count, rtol=1e-12, atol=1e-15)
    # the same with the counts given (the sums of W1 W2 W3 alone)
    w2g, wwwg, _ = toymodel.binned_window_moments(shape, lo, hi, L, R, trip, counts=res.count)
    assert np.allclose(wwwg, www, rtol=1e-13, atol=1e-16) and np.array_equal(w2g, w2)
    # shell means of W^2 by enumeration of the shell modes
    for b in range(3):
        md = oracle.shell_modes(shape, lo, hi, b)
        k = np.sqrt(sum(((2 * np.pi / (L * shape[a] / shape[2])) * md[:, a]) ** 2 for a in range(3)))
        assert w2[b] == pytest.approx(np.mean(toymodel.window(k * R) ** 2), rel=1e-12)
