"""Pins of the oracle on non-cubic and odd-sided grids (mixed-radix sizes).

Section 2 (footnote to the pixel coordinates): with a non-cubic box each axis
has its own fundamental k_f,i = 2 pi / L_i, and the estimator's normalisation
still reduces to 1/V.  Reading: cubic cells, L_i = L_x N_i / N_x, shell edges
in units of the x-axis fundamental.  The brute force below forms |k| / k_f,x
directly from the physical wave vector, not through the oracle's integer q.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import fftref, polyspec


def _modes(shape):
    f = [polyspec.freq(n) for n in shape]
    mz, my, mx = np.meshgrid(*f, indexing="ij")
    return np.stack([mz.ravel(), my.ravel(), mx.ravel()], axis=1).astype(np.int64)


def _kmod(m, shape):
    """|k| / k_f,x = sqrt(sum (m_i N_x / N_i)^2) with cubic cells."""
    nz, ny, nx = shape
    return np.sqrt((m[..., 0] * nx / nz) ** 2 + (m[..., 1] * nx / ny) ** 2 + (m[..., 2] * 1.0) ** 2)


def _wrap(u, shape):
    out = np.empty_like(u)
    for a, n in enumerate(shape):
        r = np.mod(u[..., a], n)
        out[..., a] = np.where(r >= n - n // 2, r - n, r)
    return out


def brute(delta64, shape, lo, hi):
    """S[i,j,k], C[i,j,k] and Q[i,j,k] over every ordered closed pair of grid modes."""
    D = np.fft.fftn(delta64)
    m = _modes(shape)
    k = _kmod(m, shape)
    nb = len(lo)
    mem = ((k[:, None] >= lo) & (k[:, None] < hi) & (k[:, None] > 0)).astype(float)
    keep = mem.sum(1) > 0
    m, mem = m[keep], mem[keep]
    amp = D[m[:, 0] % shape[0], m[:, 1] % shape[1], m[:, 2] % shape[2]]
    S = np.zeros((nb,) * 3, complex)
    C = np.zeros((nb,) * 3)
    Q = np.zeros((nb,) * 3)
    for a0 in range(0, len(m), 64):
        u = -(m[a0:a0 + 64, None, :] + m[None, :, :])
        w = _wrap(u, shape)
        kw = _kmod(w, shape)
        m3 = ((kw[..., None] >= lo) & (kw[..., None] < hi) & (kw[..., None] > 0)).astype(float)
        a3 = D[w[..., 0] % shape[0], w[..., 1] % shape[1], w[..., 2] % shape[2]]
        prod = amp[a0:a0 + 64, None] * amp[None, :] * a3
        S += np.einsum("ai,bj,abk,ab->ijk", mem[a0:a0 + 64], mem, m3, prod)
        C += np.einsum("ai,bj,abk->ijk", mem[a0:a0 + 64], mem, m3)
        Q += np.einsum("ai,bj,abk,ab->ijk", mem[a0:a0 + 64], mem, m3, np.abs(prod) ** 2)
    return S, C, Q


@pytest.mark.parametrize("shape,lo,hi", [
    ((6, 8, 10), [0.93, 1.71, 2.63, 3.57], [1.71, 2.63, 3.57, 4.93]),
    ((15, 15, 15), [0.93, 2.11, 3.57, 5.13], [2.11, 3.57, 5.13, 7.49]),
])
def test_noncubic_and_odd_grids_match_bruteforce(shape, lo, hi):
    rng = np.random.default_rng(11)
    d = rng.standard_normal(shape).astype(np.float32)
    lo, hi = np.array(lo), np.array(hi)
    trip = np.array(list(itertools.combinations_with_replacement(range(len(lo)), 3)))
    L = 4.5
    res = oracle.bispectrum(d, lo, hi, trip, box_len=L)
    S, C, Q = brute(oracle.prepare(d), shape, lo, hi)
    nz, ny, nx = shape
    V = L ** 3 * (nz / nx) * (ny / nx)
    norm = V ** 2 / float(np.prod(shape)) ** 3
    assert any(round(C[tuple(t)]) > 0 for t in trip)
    for t, (i, j, k) in enumerate(trip):
        assert res.count[t] == round(C[i, j, k])
        if C[i, j, k] > 0:
            scale = np.sqrt(Q[i, j, k])
            assert abs(res.s[t] - S[i, j, k]) <= 1e-9 * scale
            assert np.isclose(res.noise[t], norm * scale / C[i, j, k], rtol=1e-10)
    # mode counts from the physical |k|
    k = _kmod(_modes(shape), shape)
    want = [int(np.sum((k >= lo[b]) & (k < hi[b]) & (k > 0))) for b in range(len(lo))]
    assert list(oracle.mode_counts(shape, lo, hi)) == want


def test_noncubic_planewave_closed_form():
    shape = (12, 16, 20)
    nz, ny, nx = shape
    A = 0.3
    m1, m2 = np.array([1, 0, 2]), np.array([0, 3, -1])
    m3 = -(m1 + m2)
    ph = np.array([0.4, -0.9, 1.2])
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = sum(A * np.cos(2 * np.pi * (m[0] * z / nz + m[1] * y / ny + m[2] * x / nx) + p) for m, p in zip((m1, m2, m3), ph))
    d = d.astype(np.float32)
    kk = [_kmod(m, shape) for m in (m1, m2, m3)]
    lo = np.array([v - 1e-3 for v in kk])
    hi = np.array([v + 1e-3 for v in kk])
    L = 3.0
    res = oracle.bispectrum(d, lo, hi, [(0, 1, 2)], box_len=L)
    V = L ** 3 * (nz / nx) * (ny / nx)
    assert res.count[0] >= 2
    assert np.isclose(res.value[0], V ** 2 * A ** 3 * np.cos(ph.sum()) / (4 * res.count[0]), rtol=3e-6)
    P, M = oracle.power_spectrum(d, lo, hi, box_len=L)
    assert np.allclose(P * M, V * A ** 2 * 2 / 4, rtol=3e-6)


def test_noncubic_dft_is_numpy_fft():
    rng = np.random.default_rng(4)
    d = rng.standard_normal((6, 10, 15))
    assert np.allclose(oracle.dft3(d), np.fft.fftn(d), rtol=0, atol=1e-10 * np.abs(np.fft.fftn(d)).max())


@pytest.mark.parametrize("shape", [(12, 16, 20), (15, 15, 15), (24, 24, 24)])
def test_fft_form_equals_direct_sums_noncubic(shape):
    rng = np.random.default_rng(5)
    d = (rng.standard_normal(shape) ** 2).astype(np.float32)
    nx = shape[2]
    e = np.linspace(0.8, nx / 2.0, 7)
    lo, hi = e[:-1], e[1:]
    trip, _ = oracle.closed_triplets(shape, lo, hi)
    R = fftref.FFTReference(d, lo, hi, box_len=6.0)
    fb = R.bispectrum(trip)
    ref = oracle.bispectrum(d, lo, hi, trip, box_len=6.0)
    assert np.array_equal(fb.count, ref.count)
    err = np.abs(fb.value - ref.value) / np.maximum(np.abs(ref.value), ref.noise)
    assert err.max() <= 1e-12
    p, m = R.power_spectrum()
    pr, mr = oracle.power_spectrum(d, lo, hi, box_len=6.0)
    assert np.array_equal(m, mr) and np.max(np.abs(p - pr) / pr) <= 1e-12
    quads = np.array([(0, 0, 1, 1), (1, 1, 2, 2), (0, 1, 1, 2)], np.int32)
    ft = R.trispectrum(quads)
    rt = oracle.trispectrum(d, lo, hi, quads, box_len=6.0)
    assert np.array_equal(ft.count, rt.count)
    assert np.max(np.abs(ft.value - rt.value) / np.maximum(np.abs(rt.value), rt.noise)) <= 1e-12
