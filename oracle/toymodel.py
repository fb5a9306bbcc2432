"""Randomly placed ionised spheres: the Bharadwaj & Pandey model of the
ionisation field (TEST INFRASTRUCTURE; Section 3.3, Eqs. BharPk, BharBk).

Only ``tests/`` may import this module.  It shares no code with the HIP path.

Spheres of one radius R at number density nbar, ionised fraction
x_ion = 1 - xbar_HI = (4 pi R^3 / 3) nbar in the model (no overlap).  With
W(kR) = 3 (sin kR - kR cos kR) / (kR)^3, the Fourier transform of the unit top
hat, the neutral-fraction field x_HI has

    P(k)          = x_ion^2 W^2(kR) / nbar                      (Eq. BharPk)
    B(k1, k2, k3) = -x_ion^3 W(k1 R) W(k2 R) W(k3 R) / nbar^2     (Eq. BharBk)

(the ionised field has the same P and the opposite B).  The paper compares its
estimates with the theory averaged over the same bins (Fig. xH_bi): P over the
modes of each shell, B over the closed triangles of each triplet of shells,
which is the FFT form of the estimator applied to the model spectrum W(|k| R)
(``fftref.FFTReference.from_spectrum``): the closed-triangle mean of
W1 W2 W3 is sum_n G1 G2 G3 / sum_n I1 I2 I3 with G_b the inverse transform of
the shell box filled with W.
"""
from __future__ import annotations

import numpy as np

from . import fftref, polyspec


def window(x):
    """W(x) = 3 (sin x - x cos x) / x^3.

    Below |x| = 1/2 the difference sin x - x cos x cancels (relative error
    about 1e-16 / x^2), so there the series is summed instead:
    W = 3 sum_{n >= 1} (-1)^(n+1) 2n x^(2n-2) / (2n+1)!  (terms to n = 9)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    small = np.abs(x) < 0.5
    x2 = x[small] ** 2
    acc = np.zeros_like(x2)
    fact = 6.0                                   # (2n+1)! at n = 1
    for n in range(1, 10):
        acc += (-1.0) ** (n + 1) * 6.0 * n * x2 ** (n - 1) / fact
        fact *= (2 * n + 2) * (2 * n + 3)
    out[small] = acc
    xl = x[~small]
    out[~small] = 3.0 * (np.sin(xl) - xl * np.cos(xl)) / xl ** 3
    return out


def power(k, R, nbar, x_ion):
    return x_ion ** 2 * window(np.asarray(k) * R) ** 2 / nbar


def bispectrum(k1, k2, k3, R, nbar, x_ion):
    return -x_ion ** 3 * window(np.asarray(k1) * R) * window(np.asarray(k2) * R) * window(np.asarray(k3) * R) / nbar ** 2


def kmod_grid(shape, box_len):
    """|k| of every grid mode (cubic cells, L_x = box_len) in inverse length units."""
    nz, ny, nx = shape
    s = polyspec.q_scales(shape)
    q = polyspec._q_of(*np.meshgrid(*[polyspec.freq(n) for n in shape], indexing="ij"), s)
    # |k| = (2 pi / L_x) sqrt(q) / s_x
    return (2.0 * np.pi / float(box_len)) * np.sqrt(q.astype(np.float64)) / s[2]


def binned_window_moments(shape, k_lo, k_hi, box_len, R, triplets, cache_bytes=16 << 30, counts=None):
    """<W^2> over the modes of each shell and <W1 W2 W3> over the closed
    triangles of each triplet (closure modulo N, as the estimator counts them),
    with the triangle counts (computed here unless given)."""
    kk = kmod_grid(shape, box_len)
    w = window(kk * R)
    lo2, hi2 = polyspec.squared_edges(k_lo, k_hi, shape)
    s = polyspec.q_scales(shape)
    q = (kk * float(box_len) / (2.0 * np.pi) * s[2]) ** 2
    qi = np.rint(q)
    w2 = np.zeros(len(k_lo))
    for b in range(len(k_lo)):
        m = (qi > 0) & (qi >= lo2[b]) & (qi < hi2[b])
        w2[b] = np.mean(w[m] ** 2)
    del q, qi, kk
    ref = fftref.FFTReference.from_spectrum(w.astype(np.complex128), k_lo, k_hi, box_len=box_len,
                                            cache_bytes=cache_bytes)
    del w
    if counts is None:
        sp = ref.bispectrum(triplets)
        return w2, sp.s / sp.count, sp.count
    # the sums of W1 W2 W3 alone, in bin order so the field cache is reused
    t = np.asarray(triplets, dtype=np.int64).reshape(-1, 3)
    s = np.zeros(len(t))
    for i in sorted(range(len(t)), key=lambda i: tuple(sorted(t[i]))):
        s[i] = ref.grid_sum("F", t[i]) / ref.npix
    return w2, s / np.asarray(counts, dtype=np.float64), np.asarray(counts, dtype=np.float64)
