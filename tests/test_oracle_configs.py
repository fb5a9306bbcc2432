"""Pins of the configuration-binning oracle (CPU).

The count-weighted group average of per-triplet B (oracle.configs.rebin over
oracle.polyspec.bispectrum) must equal a brute-force sum over the mode pairs
of the two fixed shells, grouped by the angle of the closing shell
(oracle.configs.theta_direct), which never forms a per-triplet sum.  The
angle groups are checked against closed-form triangles.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import configs as oc
from oracle import polyspec as ps
from paper_1705_06284_amd import synth


@pytest.fixture(scope="module")
def small():
    n = 16
    lo, hi = synth.unit_bins(1, 7)
    d = synth.lognormal_field(n, 1.5, 1.0, 7)
    tri, _ = ps.closed_triplets(n, lo, hi)
    return n, lo, hi, d, tri, ps.bispectrum(d, lo, hi, tri)


@pytest.mark.parametrize("b1,b2,n_cos", [(1, 3, 20), (2, 2, 20), (0, 6, 20), (4, 2, 7), (3, 3, 1)])
def test_rebin_equals_brute_force_over_mode_pairs(small, b1, b2, n_cos):
    n, lo, hi, d, tri, ref = small
    g, _ = oc.theta_groups(lo, hi, tri, b1, b2, n_cos)
    rb = oc.rebin(ref.value, ref.count, g, n_cos)[0]
    bd, cd = oc.theta_direct(d, lo, hi, b1, b2, n_cos)
    cg = np.array([ref.count[g == k].sum() for k in range(n_cos)])
    assert np.array_equal(cg, cd)                       # the same closed triangles
    assert np.array_equal(np.isfinite(rb), cd > 0)
    ok = cd > 0
    assert ok.any()
    assert np.max(np.abs(rb[ok] - bd[ok]) / np.abs(bd[ok])) < 1e-12


def test_angle_groups_of_closed_form_triangles():
    c = Fraction
    # equilateral: theta = pi/3, cos = 1/2, the lower edge of group 15 of 20
    assert oc.cos_group(c(5), c(5), c(5), 20) == (c(1, 2), 15)
    # 3-4-5: the angle between 3 and 4 is a right angle (cos 0: group 10)
    assert oc.cos_group(c(3), c(4), c(5), 20) == (c(0), 10)
    # collinear k3 = k1 + k2: cos = -1, group 0; folded k3 = k2 - k1: cos = 1, last group
    assert oc.cos_group(c(2), c(3), c(5), 20) == (c(-1), 0)
    assert oc.cos_group(c(2), c(3), c(1), 20) == (c(1), 19)
    # no triangle: k3 beyond k1 + k2
    assert oc.cos_group(c(2), c(3), c(6), 20)[1] == -1
    # an exact edge that FP64 division misses: cos = -4/5 starts group 2
    assert oc.cos_group(c(15), c(28), c(41), 20) == (c(-4, 5), 2)


def test_theta_groups_membership(small):
    n, lo, hi, d, tri, ref = small
    g, cos = oc.theta_groups(lo, hi, tri, 1, 3, 20)
    for t, (i, j, k) in enumerate(tri):
        ms = sorted((int(i), int(j), int(k)))
        holds = 1 in ms and (3 in ms[:ms.index(1)] + ms[ms.index(1) + 1:])
        assert (not np.isnan(cos[t])) == holds
        if holds:
            rest = list(ms)
            rest.remove(1)
            rest.remove(3)
            c1, c2, c3 = 2.0, 4.0, rest[0] + 1.0            # unit bins: centre = index + 1
            assert cos[t] == pytest.approx((c1 * c1 + c2 * c2 - c3 * c3) / (2 * c1 * c2), abs=1e-15)
        else:
            assert g[t] == -1


def test_rebin_weights_and_empty_groups():
    vals = np.array([[1.0, 2.0, 4.0, np.nan]])
    counts = np.array([1.0, 3.0, 0.0, 0.0])
    out = oc.rebin(vals, counts, np.array([0, 0, 1, 0]), 3)[0]
    assert out[0] == pytest.approx((1.0 + 6.0) / 4.0)
    assert np.isnan(out[1]) and np.isnan(out[2])       # only zero counts / no member
