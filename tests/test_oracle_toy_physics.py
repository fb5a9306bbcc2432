"""The estimator on the ionised-sphere boxes of Section 3.3 against the
bin-averaged Bharadwaj-Pandey model (Eqs. BharPk, BharBk; Figs. powerSpec and
xH_bi), on the FP64 values the oracle stored for the two 600^3 boxes
(tests/golden/toy600_*.fftref.npz; the GPU matches them in
test_gpu_fullsets.py).

The model is averaged over the same configurations as the estimate: W^2
over the modes of each shell, W1 W2 W3 over the closed triangles of each
triplet (oracle/toymodel.py), with the box's sphere density and ionised
fraction.  Differences are measured against the window's envelope
(max of the bin average and the large-kR envelope 4.5 / (kR)^4 for W^2,
(min(1, 3 / (kR)^2))^3 / 2 for the triple product), so that a zero of the
window does not blow up a relative error.  Sample variance makes k below
(100/6) k_f noisy (Section 3.3); those shells are left out.

* x_HI = 0.99 (522 spheres, overlap negligible): P within 10 % and B within
  15 % of the envelope everywhere, both with medians below 3 % -- the
  paper's "follows the theoretical predictions very closely".
* x_HI = 0.88 (6615 spheres, overlapping): the model, which has no overlap,
  fits worse below 0.2 Mpc^-1, as the paper finds at z = 11 on its
  equilateral configurations: there the median deviation is ten times the
  0.99 box's (0.42 against 0.04 of the envelope), while above 0.2 Mpc^-1
  the 0.88 box stays near the model (median 0.07).
"""
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _load(wl):
    path = os.path.join(HERE, "golden", "%s.fftref.npz" % wl)
    if not os.path.exists(path):
        pytest.skip("no stored values for %s" % wl)
    return np.load(path)


def _deviations(z):
    L, R = float(z["box_len"]), float(z["radius"])
    xion = float(z["ionized_fraction"])
    nbar = int(z["spheres"]) / L ** 3
    kf = 2.0 * np.pi / L
    kc = 0.5 * (z["k_lo"] + z["k_hi"])
    x = kc * kf * R
    t = z["triplets"]
    env_p = np.maximum(z["W2_bin"], 4.5 / x ** 4)
    dp = np.abs(z["P"] - xion ** 2 * z["W2_bin"] / nbar) / (xion ** 2 / nbar * env_p)
    env_w = np.minimum(1.0, 3.0 / x ** 2)
    env_b = np.maximum(np.abs(z["WWW_bin"]), 0.5 * env_w[t[:, 0]] * env_w[t[:, 1]] * env_w[t[:, 2]])
    db = np.abs(z["B"] + xion ** 3 * z["WWW_bin"] / nbar ** 2) / (xion ** 3 / nbar ** 2 * env_b)
    return kc, kf, t, dp, db


def test_toy_box_099_follows_the_model():
    z = _load("toy600_xhi099")
    assert int(z["spheres"]) == 522 and abs(float(z["ionized_fraction"]) - 0.01) < 1e-4
    kc, kf, t, dp, db = _deviations(z)
    sp = kc >= 100.0 / 6.0
    sb = kc[t].min(axis=1) >= 100.0 / 6.0
    assert sp.sum() == 53 and sb.sum() > 100
    assert dp[sp].max() <= 0.10 and np.median(dp[sp]) <= 0.03
    assert db[sb].max() <= 0.15 and np.median(db[sb]) <= 0.03
    # the sign: a neutral field punctured by spheres has negative skewness
    # where the window is positive (k R below its first zero, 4.49)
    low = (kc[t].max(axis=1) * kf * float(z["radius"]) < 4.0) & sb
    assert np.all(z["B"][low] < 0)


def test_overlap_at_088_departs_from_the_model_below_0p2():
    z99, z88 = _load("toy600_xhi099"), _load("toy600_xhi088")
    assert int(z88["spheres"]) == 6615 and abs(float(z88["ionized_fraction"]) - 0.12) < 1e-4
    kc, kf, t, _, db99 = _deviations(z99)
    _, _, t88, _, db88 = _deviations(z88)
    assert np.array_equal(t, t88)
    k = kc[t] * kf
    equilateral = (t[:, 0] == t[:, 1]) & (t[:, 1] == t[:, 2])
    low = equilateral & (k.max(axis=1) < 0.2)
    assert low.sum() == 9
    assert np.median(db88[low]) > 5.0 * np.median(db99[low])
    high = k.min(axis=1) >= 0.2
    assert high.sum() > 100
    assert np.median(db88[high]) < 0.1 < np.median(db88[low])
