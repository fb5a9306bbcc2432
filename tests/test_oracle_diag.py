"""Pins of the oracle's diagonal-binned trispectrum (CPU).

T(a, b, c, d; e) sums D(k1) D(k2) D(k3) D(k4) over closed quadruples with
k_i in the four shells and the diagonal k1 + k2 (reduced modulo N) in shell
e (Section 2, Eq. Jeong_gen with p = 4; four shells leave the diagonal free).

* Enumeration: on 8^3 every combination of modes of the four shells is
  tested for closure and for the diagonal; the sum, the count and the paired
  part (two pairs k_i = -k_j) match trispectrum_diag and
  diag_disconnected_sums.
* Sum over diagonals: with shells e tiling every |q| > 0, the diagonal sums
  add up to the plain p = 4 sum (pinned elsewhere) when a != b (no closed
  quadruple then has q = 0), and the paired sums of (a, b, a, b) add up to
  X_a X_b = sum |D1|^2 sum |D2|^2.
* Plane wave: D = A at +-k0 only; the quad (a, a, a, a) with |2 k0| in e has
  S = 2 A^4 and a connected part of zero.
"""
import numpy as np

import oracle
from oracle import polyspec


def _wrap(c, n):
    return ((c + n // 2) % n) - n // 2


def test_diag_sums_match_enumeration_8():
    rng = np.random.default_rng(41)
    n = 8
    d = rng.standard_normal((n, n, n)).astype(np.float32)
    lo = np.array([0.9, 1.9, 0.9, 1.5])
    hi = np.array([1.9, 2.6, 2.3, 2.9])
    # shells 0, 1 for the quads; 2 and 3 as diagonal shells (overlapping is fine)
    dq = np.array([(0, 1, 0, 1, 2), (0, 0, 1, 1, 3), (1, 0, 0, 1, 2), (0, 0, 0, 0, 3), (0, 1, 1, 1, 3)])
    res = oracle.trispectrum_diag(d, lo, hi, dq)
    sd = polyspec.diag_disconnected_sums(d, lo, hi, dq)
    D = np.fft.fftn(oracle.prepare(d))
    amp = lambda m: D[m[0] % n, m[1] % n, m[2] % n]
    sh = [oracle.shell_modes(n, lo, hi, b).astype(np.int64) for b in range(len(lo))]
    for t, (a, b, c, dd, e) in enumerate(dq):
        ks = [sh[a][:, None, None, None, :], sh[b][None, :, None, None, :],
              sh[c][None, None, :, None, :], sh[dd][None, None, None, :, :]]
        closed = np.all(_wrap(ks[0] + ks[1] + ks[2] + ks[3], n) == 0, axis=-1)
        q = _wrap(ks[0] + ks[1], n)
        qq = np.sum(q * q, axis=-1).astype(np.float64)
        inside = (qq > 0) & (qq >= lo[e] ** 2) & (qq < hi[e] ** 2)
        sel = closed & inside
        amps = [amp(sh[x].T) for x in (a, b, c, dd)]
        p = (amps[0][:, None, None, None] * amps[1][None, :, None, None]
             * amps[2][None, None, :, None] * amps[3][None, None, None, :])
        pair = lambda i, j: np.all(_wrap(ks[i] + ks[j], n) == 0, axis=-1)
        is_paired = (pair(0, 1) & pair(2, 3)) | (pair(0, 2) & pair(1, 3)) | (pair(0, 3) & pair(1, 2))
        cnt, tot, paired = int(sel.sum()), p[sel].sum(), p[sel & is_paired].sum()
        assert res.count[t] == cnt, t
        assert cnt > 0
        assert abs(res.s[t] - tot) <= 1e-10 * (1 + abs(tot)), t
        assert abs(sd[t] - paired) <= 1e-10 * (1 + abs(paired)), t


def test_diagonal_shells_add_up_to_the_plain_sum():
    rng = np.random.default_rng(42)
    n = 12
    d = rng.standard_normal((n, n, n)).astype(np.float32)
    quad_lo, quad_hi = [1.0, 2.0, 3.0], [2.0, 3.0, 4.5]
    # diagonal shells tiling 0 < |q| <= sqrt(3) n / 2
    dl = np.arange(0.5, 11.0, 1.0)
    lo = np.concatenate([quad_lo, dl])
    hi = np.concatenate([quad_hi, dl + 1.0])
    assert hi[-1] ** 2 > 3 * (n / 2) ** 2
    diag = range(3, len(lo))
    for quad in [(0, 1, 0, 1), (0, 1, 1, 2), (0, 2, 1, 1), (1, 2, 2, 1)]:
        dq = np.array([quad + (e,) for e in diag])
        res = oracle.trispectrum_diag(d, lo, hi, dq)
        plain = oracle.trispectrum(d, lo, hi, np.array([quad]))
        assert res.count.sum() == plain.count[0]
        assert abs(res.s.sum() - plain.s[0]) <= 1e-10 * np.abs(res.s).sum()
    # paired parts of (a, b, a, b): every pair (k1, k2) with k3 = -k1, k4 = -k2
    dq = np.array([(0, 1, 0, 1, e) for e in diag])
    sd = polyspec.diag_disconnected_sums(d, lo, hi, dq)
    D = np.fft.fftn(oracle.prepare(d))
    x = [np.sum(np.abs(D[m[:, 0] % n, m[:, 1] % n, m[:, 2] % n]) ** 2)
         for m in (oracle.shell_modes(n, lo, hi, 0), oracle.shell_modes(n, lo, hi, 1))]
    assert abs(sd.sum() - x[0] * x[1]) <= 1e-10 * x[0] * x[1]


def test_plane_wave_closed_form_and_zero_connected_part():
    n = 16
    k0 = np.array([1, 2, 2])                     # |k0| = 3, |2 k0| = 6
    g = np.indices((n, n, n)).reshape(3, -1).T
    A = 0.5 * n ** 3
    d = np.cos(2 * np.pi * (g @ k0) / n).reshape(n, n, n)
    lo = np.array([2.5, 5.5])
    hi = np.array([3.5, 6.5])
    val, res, sd = oracle.trispectrum_diag_connected(d, lo, hi, [(0, 0, 0, 0, 1)])
    vol, npix = float(n) ** 3, float(n) ** 3
    assert abs(res.s[0] - 2 * A ** 4) <= 1e-9 * A ** 4
    assert abs(res.value[0] - vol ** 3 / npix ** 4 * 2 * A ** 4 / res.count[0]) <= 1e-9 * abs(res.value[0])
    assert abs(sd[0] - 2 * A ** 4) <= 1e-9 * A ** 4
    assert abs(val[0]) <= 1e-9 * abs(res.value[0])
