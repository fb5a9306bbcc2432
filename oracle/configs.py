"""Configuration binning of narrow-shell bispectra (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the HIP path.

Watkinson et al. 2017 (arXiv:1705.06284) plot B against the angle theta
between the triangle sides k1 and k2 at fixed k1 and k2 = m k1 (Section 3,
Fig. theta_illus, Eqs. ratio and alpha), averaging over bins of cos theta of
half-width 0.05 (Section 3.2), and advise measuring with shells one k_f wide
and binning further afterwards (Section 3.2, Conclusion).  Readings used here:

* theta is the interior angle between sides k1 and k2, so by the law of
  cosines cos theta = (k1^2 + k2^2 - k3^2) / (2 k1 k2), evaluated at the bin
  centres (lo + hi) / 2 of the triplet's three bins;
* the cos theta bins are n_cos equal intervals [-1 + 2g/n_cos, -1 + 2(g+1)/n_cos)
  (the last one closed at 1); bin centres outside [-1, 1] form no triangle
  and join no group.  The decision is taken in exact rational arithmetic;
* the average over a group weights each triplet by its triangle count N_t,
  which is the estimator over the union of the group's closed triangles.

Functions:

* ``theta_groups``: the group of each triplet (exact rationals);
* ``rebin``: the count-weighted group average of given per-triplet values;
* ``theta_direct``: B per group by brute force over the mode pairs
  (m1 in S_b1, m2 in S_b2), m3 = -(m1 + m2) mod N, without the per-triplet
  sums -- the pin of the two above.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from . import polyspec as _ps


def _centre(k_lo, k_hi, b):
    return (Fraction(float(k_lo[b])) + Fraction(float(k_hi[b]))) / 2


def cos_group(c1, c2, c3, n_cos):
    """(cos theta as a Fraction, group or -1) for side centres c1, c2, c3."""
    c = (c1 * c1 + c2 * c2 - c3 * c3) / (2 * c1 * c2)
    if c < -1 or c > 1:
        return c, -1
    g = math.floor((c + 1) * n_cos / 2)
    return c, min(g, n_cos - 1)


def theta_groups(k_lo, k_hi, triplets, b1, b2, n_cos):
    """group[t] for B(theta) at k1 in bin b1, k2 in bin b2; -1 where the
    triplet does not hold b1 and b2 (as a multiset) or has no angle."""
    group = np.full(len(triplets), -1, dtype=np.int32)
    cos = np.full(len(triplets), np.nan)
    c1, c2 = _centre(k_lo, k_hi, b1), _centre(k_lo, k_hi, b2)
    for t, tri in enumerate(np.asarray(triplets).reshape(-1, 3)):
        rest = [int(b) for b in tri]
        ok = True
        for want in (b1, b2):
            if want in rest:
                rest.remove(want)
            else:
                ok = False
        if not ok:
            continue
        c, g = cos_group(c1, c2, _centre(k_lo, k_hi, rest[0]), n_cos)
        cos[t] = float(c)
        group[t] = g
    return group, cos


def rebin(values, counts, group, n_group):
    """sum_{t in g} N_t X_t / sum_{t in g} N_t per group (NaN if empty);
    values: [n_tri] or [batch, n_tri]."""
    v = np.atleast_2d(np.asarray(values, dtype=np.float64))
    counts = np.asarray(counts, dtype=np.float64)
    group = np.asarray(group)
    out = np.full((v.shape[0], n_group), np.nan)
    for g in range(n_group):
        sel = (group == g) & (counts > 0)
        if not sel.any():
            continue
        den = math.fsum(counts[sel])
        for m in range(v.shape[0]):
            out[m, g] = math.fsum(counts[sel] * v[m, sel]) / den
    return out


def theta_direct(delta, k_lo, k_hi, b1, b2, n_cos, box_len=None):
    """(B [n_cos], count [n_cos]) by brute force over the mode pairs of
    shells b1 and b2: for every m1 in S_b1 and m2 in S_b2 the closing mode is
    m3 = -(m1 + m2) wrapped into [-N/2, N/2)^3; every bin b3 that holds m3
    adds D(m1) D(m2) D(m3) and 1 to the group of (b1, b2, b3)."""
    d = _ps.prepare(delta)
    n = d.shape[0]
    dk = _ps.dft3(d)
    lo2, hi2 = _ps.squared_edges(k_lo, k_hi, n)
    nb = len(k_lo)
    c1, c2 = _centre(k_lo, k_hi, b1), _centre(k_lo, k_hi, b2)
    grp = [cos_group(c1, c2, _centre(k_lo, k_hi, b3), n_cos)[1] for b3 in range(nb)]
    s1 = _ps.shell_modes(n, k_lo, k_hi, b1).astype(np.int64)
    s2 = _ps.shell_modes(n, k_lo, k_hi, b2).astype(np.int64)
    h = n // 2
    S = np.zeros(n_cos, dtype=np.complex128)
    C = np.zeros(n_cos, dtype=np.int64)
    for m1 in s1:
        m3 = (-(m1[None, :] + s2) + h) % n - h                # wrapped closing modes
        r2 = (m3 * m3).sum(axis=1).astype(np.float64)
        idx = m3 % n
        d1 = dk[m1[0] % n, m1[1] % n, m1[2] % n]
        prod = d1 * dk[s2[:, 0] % n, s2[:, 1] % n, s2[:, 2] % n] * dk[idx[:, 0], idx[:, 1], idx[:, 2]]
        for b3 in range(nb):
            g = grp[b3]
            if g < 0:
                continue
            sel = (r2 > 0) & (r2 >= lo2[b3]) & (r2 < hi2[b3])
            if sel.any():
                S[g] += prod[sel].sum()
                C[g] += int(sel.sum())
    vol = float(n) ** 3 if (box_len is None or box_len <= 0) else float(box_len) ** 3
    npix = float(n) ** 3
    with np.errstate(invalid="ignore", divide="ignore"):
        B = (vol ** 2 / npix ** 3) * S.real / C
    return B, C
