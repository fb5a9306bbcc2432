"""Pins of the oracle's direct closed-tuple sums (B, T, counts, P).

* Brute force: on 8^3 / 16^3 grids every ordered pair (triple) of grid modes
  is enumerated with numpy, the closing mode found by index arithmetic modulo
  N, and the sums compared with the oracle's shell-list loops (the check of
  triangle counts against the FFT count, Section 3 after Eq. nyqvist).
* Plane-wave closed forms: delta = A sum_a cos(2 pi m_a.n / N + phi_a) gives
  B, P and T in closed form (Eqs. Jeong_PS, Jeong_BI, Jeong_gen).
* Parseval: P equals the shell average of |Delta|^2 and the direct pair sum.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import polyspec


def _grid_modes(n, hi_max):
    f = oracle.freq(n)
    mz, my, mx = np.meshgrid(f, f, f, indexing="ij")
    m = np.stack([mz.ravel(), my.ravel(), mx.ravel()], axis=1).astype(np.int64)
    r2 = np.sum(m * m, axis=1)
    keep = (r2 > 0) & (r2 < hi_max * hi_max)
    return m[keep]


def _membership(m, lo, hi):
    r2 = np.sum(m * m, axis=-1).astype(np.float64)
    lo2, hi2 = np.asarray(lo) ** 2, np.asarray(hi) ** 2
    inside = (r2[..., None] >= lo2) & (r2[..., None] < hi2) & (r2[..., None] > 0)
    return inside


def _wrap(c, n):
    return ((c + n // 2) % n) - n // 2


def brute_bispectrum_sums(delta64, lo, hi, want_sq=False):
    """S[i,j,k] (ordered slots, mod-N closure) and strict S by full enumeration;
    with want_sq also Q[i,j,k] = sum |D1 D2 D3|^2 over the same closed triples."""
    n = delta64.shape[0]
    D = np.fft.fftn(delta64)                  # library FFT, not the oracle's DFT
    m = _grid_modes(n, max(hi))
    amp = D[m[:, 0] % n, m[:, 1] % n, m[:, 2] % n]
    mem = _membership(m, lo, hi).astype(np.float64)
    nb = len(lo)
    S = np.zeros((nb, nb, nb), complex)
    Ss = np.zeros((nb, nb, nb), complex)
    C = np.zeros((nb, nb, nb))
    Cs = np.zeros((nb, nb, nb))
    Q = np.zeros((nb, nb, nb))
    chunk = 64
    for a0 in range(0, len(m), chunk):
        m1 = m[a0:a0 + chunk]
        u = -(m1[:, None, :] + m[None, :, :])          # unreduced closing vector
        w = _wrap(u, n)
        strict = np.all(u == w, axis=-1)
        a3 = D[w[..., 0] % n, w[..., 1] % n, w[..., 2] % n]
        prod = amp[a0:a0 + chunk, None] * amp[None, :] * a3
        m3 = _membership(w, lo, hi).astype(np.float64)
        m1m = mem[a0:a0 + chunk]
        S += np.einsum("ai,bj,abk,ab->ijk", m1m, mem, m3, prod)
        C += np.einsum("ai,bj,abk->ijk", m1m, mem, m3)
        Ss += np.einsum("ai,bj,abk,ab->ijk", m1m, mem, m3, prod * strict)
        Cs += np.einsum("ai,bj,abk,ab->ijk", m1m, mem, m3, strict.astype(float))
        if want_sq:
            Q += np.einsum("ai,bj,abk,ab->ijk", m1m, mem, m3, np.abs(prod) ** 2)
    if want_sq:
        return S, C, Ss, Cs, Q
    return S, C, Ss, Cs


def test_counts_and_sums_match_bruteforce_8():
    rng = np.random.default_rng(5)
    n = 8
    d = rng.standard_normal((n, n, n)).astype(np.float32)
    lo, hi = np.array([0.5, 1.5, 2.5]), np.array([1.5, 2.5, 4.0])
    trip = np.array(list(itertools.combinations_with_replacement(range(3), 3)))
    res = oracle.bispectrum(d, lo, hi, trip)
    S, C, Ss, Cs = brute_bispectrum_sums(oracle.prepare(d), lo, hi)
    for t, (i, j, k) in enumerate(trip):
        assert res.count[t] == round(C[i, j, k])
        assert res.count_strict[t] == round(Cs[i, j, k])
        assert abs(res.s[t] - S[i, j, k]) <= 1e-9 * (1 + np.abs(S).max())
        assert abs(res.s_strict[t] - Ss[i, j, k]) <= 1e-9 * (1 + np.abs(S).max())
    # 8^3 with hi = N/2 = 4 aliases: at least one triplet has count != strict
    assert np.any(res.count != res.count_strict)


def test_noise_level_matches_bruteforce_8():
    """The noise level of every parity bar, norm sqrt(sum |D1 D2 D3|^2) / N_t
    (the random-phase spread of the mean over closed triples), against the
    full-grid enumeration of the closed triples and their squared products."""
    rng = np.random.default_rng(6)
    n = 8
    d = rng.standard_normal((n, n, n)).astype(np.float32)
    lo, hi = np.array([0.5, 1.5, 2.5]), np.array([1.5, 2.5, 4.0])
    trip = np.array(list(itertools.combinations_with_replacement(range(3), 3)))
    L = 5.0
    res = oracle.bispectrum(d, lo, hi, trip, box_len=L)
    S, C, _, _, Q = brute_bispectrum_sums(oracle.prepare(d), lo, hi, want_sq=True)
    norm = (L ** 3) ** 2 / float(n) ** 9
    for t, (i, j, k) in enumerate(trip):
        want = norm * np.sqrt(Q[i, j, k]) / C[i, j, k]
        assert np.isclose(res.noise[t], want, rtol=1e-10), (t, res.noise[t], want)
        # and B itself, with the box length entering as V^2
        assert np.isclose(res.value[t], norm * S[i, j, k].real / C[i, j, k], rtol=1e-9,
                          atol=1e-9 * norm * np.sqrt(Q[i, j, k]) / C[i, j, k])


def test_candidate_filter_keeps_every_closed_triplet():
    """Every bin triplet with a non-zero brute-force count (closure modulo N,
    aliasing included) passes the candidate filter, and the filter drops
    some triplets on a layout with a gap between shells."""
    n = 8
    lo, hi = np.array([0.5, 1.2, 2.0, 3.0]), np.array([1.2, 2.0, 3.0, 4.0])
    _, C, _, Cs = brute_bispectrum_sums(np.ones((n, n, n)), lo, hi)
    assert np.any(np.round(C) != np.round(Cs))          # aliased closures occur
    cand = {tuple(t) for t in oracle.candidate_triplets(lo, hi)}
    full = list(itertools.combinations_with_replacement(range(4), 3))
    assert len(cand) < len(full)
    for t in full:
        if round(C[t]) > 0:
            assert t in cand, t
    closed, cnt = oracle.closed_triplets(n, lo, hi)
    assert {tuple(t) for t in closed} == {t for t in full if round(C[t]) > 0}
    assert all(c == round(C[tuple(t)]) for t, c in zip(closed, cnt))
    # a gapped layout: (0, 0, 2) fails the triangle test and has no closure
    n = 16
    lo, hi = np.array([1.0, 2.0, 6.0]), np.array([2.0, 3.0, 7.5])
    _, C, _, _ = brute_bispectrum_sums(np.ones((n, n, n)), lo, hi)
    cand = {tuple(t) for t in oracle.candidate_triplets(lo, hi)}
    assert (0, 0, 2) not in cand and round(C[0, 0, 2]) == 0
    for t in itertools.combinations_with_replacement(range(3), 3):
        if round(C[t]) > 0:
            assert t in cand, t


def test_counts_match_bruteforce_16_linear_bins():
    n = 16
    lo, hi = np.arange(4) * 2.0, np.arange(1, 5) * 2.0
    trip = oracle.candidate_triplets(lo, hi)
    cnt, cnt_strict = oracle.triangle_counts(n, lo, hi, trip)
    d = np.ones((n, n, n))
    _, C, _, Cs = brute_bispectrum_sums(d, lo, hi)   # counts do not use amplitudes
    for t, (i, j, k) in enumerate(trip):
        assert cnt[t] == round(C[i, j, k])
        assert cnt_strict[t] == round(Cs[i, j, k])
        # slot symmetry of the count
        assert round(C[i, j, k]) == round(C[k, i, j]) == round(C[j, k, i])


def test_pair_loop_slot_order_invariance():
    """S(i,j,k) computed with the loops over (i,j) or over (j,k) agree."""
    rng = np.random.default_rng(9)
    n = 16
    d = oracle.prepare(rng.standard_normal((n, n, n)).astype(np.float32))
    D = oracle.dft3(d)
    lo, hi = np.array([1.0, 2.5, 4.0]), np.array([2.5, 4.0, 6.0])
    mask = oracle.bin_mask_table(n, lo, hi)
    sh = [oracle.shell_modes(n, lo, hi, b) for b in range(3)]
    re, im = np.ascontiguousarray(D.real), np.ascontiguousarray(D.imag)
    a = polyspec._pair_sums(n, re, im, sh[0], sh[1], mask, 1 << 2, 3)[2]
    b = polyspec._pair_sums(n, re, im, sh[1], sh[2], mask, 1 << 0, 3)[0]
    c = polyspec._pair_sums(n, re, im, sh[2], sh[0], mask, 1 << 1, 3)[1]
    assert a[2] == b[2] == c[2]
    for x in (b, c):
        assert abs(complex(a[0], a[1]) - complex(x[0], x[1])) < 1e-9 * abs(complex(a[0], a[1]))


def _waves(n, amp, vecs, phases):
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    d = np.zeros((n, n, n))
    for m, ph in zip(vecs, phases):
        d += amp * np.cos(2 * np.pi * (m[0] * z + m[1] * y + m[2] * x) / n + ph)
    return d


def test_planewave_three_shells_closed_form():
    n = 16
    A = 0.3
    m1, m2 = np.array([1, 0, 0]), np.array([0, 2, 1])
    m3 = -(m1 + m2)                                     # |m|^2 = 1, 5, 6
    ph = np.array([0.3, -1.1, 0.7])
    d = _waves(n, A, [m1, m2, m3], ph).astype(np.float32)
    lo, hi = np.sqrt([0.5, 4.5, 5.5]), np.sqrt([1.5, 5.5, 6.5])   # one |m|^2 per bin
    res = oracle.bispectrum(d, lo, hi, [(0, 1, 2)])
    V = float(n) ** 3
    want = V ** 2 * A ** 3 * np.cos(ph.sum()) / (4 * res.count[0])
    assert np.isclose(res.value[0], want, rtol=2e-6)    # FP32 input rounding
    # noise level: of the N_t closed triples only (m1, m2, m3) and its
    # negative carry amplitude, each |product| = (A N_pix / 2)^3
    assert res.count[0] > 2
    assert np.isclose(res.noise[0], V ** 2 * A ** 3 * np.sqrt(2.0) / (8 * res.count[0]), rtol=2e-6)
    # B(alpha delta) = alpha^3 B
    res2 = oracle.bispectrum((2.0 * d).astype(np.float32), lo, hi, [(0, 1, 2)])
    assert np.isclose(res2.value[0], 8 * res.value[0], rtol=1e-12)
    # P_b = V A^2 (number of +-m_a in S_b) / (4 M_b), with box length L != N
    P, M = oracle.power_spectrum(d, lo, hi, box_len=3.0)
    assert np.allclose(P, 27.0 * A ** 2 * 2 / (4 * M), rtol=2e-6)


def test_planewave_equilateral_single_shell():
    n = 32
    A, c = 0.2, 3
    v = [c * np.array([1, -1, 0]), c * np.array([0, 1, -1]), c * np.array([-1, 0, 1])]
    ph = np.array([0.4, 0.25, -1.3])
    d = _waves(n, A, v, ph).astype(np.float32)
    r = np.sqrt(2.0) * c
    lo, hi = np.array([r - 0.3]), np.array([r + 0.3])
    L = 7.5
    res = oracle.bispectrum(d, lo, hi, [(0, 0, 0)], box_len=L)
    want = 3 * (L ** 3) ** 2 * A ** 3 * np.cos(ph.sum()) / (2 * res.count[0])
    assert np.isclose(res.value[0], want, rtol=2e-6)


def test_planewave_aliased_closure_counts_only_mod_n():
    """m1+m2+m3 = (0,0,N): closed modulo N only; the strict sum is empty."""
    n = 16
    A = 0.5
    vecs = [np.array([0, 0, 7]), np.array([0, 0, 6]), np.array([0, 0, 3])]
    ph = np.array([0.1, 0.2, 0.3])
    d = _waves(n, A, vecs, ph).astype(np.float32)
    lo, hi = np.array([2.5, 5.5, 6.5]), np.array([3.5, 6.5, 7.5])
    res = oracle.bispectrum(d, lo, hi, [(0, 1, 2)])
    V = float(n) ** 3
    assert abs(res.s_strict[0]) < 1e-6 * abs(res.s[0])
    assert np.isclose(res.value[0], V ** 2 * A ** 3 * np.cos(ph.sum()) / (4 * res.count[0]), rtol=2e-6)


def _enumerate_sparse_tuple_sum(modes, amps, shells, n):
    """Sum over ordered tuples drawn from a sparse spectrum, closure mod N."""
    tot = 0j
    for pick in itertools.product(range(len(modes)), repeat=len(shells)):
        if not all(shells[s](modes[p]) for s, p in enumerate(pick)):
            continue
        ssum = np.sum([modes[p] for p in pick], axis=0)
        if np.all(ssum % n == 0):
            tot += np.prod([amps[p] for p in pick])
    return tot


def test_planewave_collapsed_trispectrum_closed_form():
    n = 16
    A = 0.4
    m1, m2 = np.array([1, 2, 0]), np.array([2, -1, 0])      # |m|^2 = 5
    m3 = np.array([-1, -2, 2])
    m4 = -(m1 + m2 + m3)                                     # |m|^2 = 9
    assert m4 @ m4 == 9 and m3 @ m3 == 9
    ph = np.array([0.5, -0.2, 1.0, 0.3])
    d = _waves(n, A, [m1, m2, m3, m4], ph).astype(np.float32)
    lo, hi = np.array([2.2, 2.95]), np.array([2.3, 3.05])   # |m|^2 = 5 and 9 only
    res = oracle.trispectrum(d, lo, hi, [(0, 0, 1, 1)])
    V = float(n) ** 3
    # connected closures: 8 ordered assignments (4 with +phi, 4 with -phi);
    # disconnected pairings (x, -x, y, -y): 4 x 4 = 16.
    want_s = (A * n ** 3 / 2) ** 4 * (8 * np.cos(ph.sum()) + 16)
    # check the combinatorics of the construction by direct enumeration of the
    # eight non-zero modes of the sparse spectrum
    modes = [m1, m2, m3, m4, -m1, -m2, -m3, -m4]
    amps = [A * n ** 3 / 2 * np.exp(1j * p) for p in ph] + [A * n ** 3 / 2 * np.exp(-1j * p) for p in ph]
    in_a = lambda m: int(m @ m) == 5
    in_b = lambda m: int(m @ m) == 9
    enum = _enumerate_sparse_tuple_sum(modes, amps, [in_a, in_a, in_b, in_b], n)
    assert np.isclose(enum, want_s, rtol=1e-12)
    assert np.isclose(res.s[0].real, want_s, rtol=2e-6)
    assert np.isclose(res.value[0], V ** 3 * A ** 4 * (8 * np.cos(ph.sum()) + 16) / (16 * res.count[0]),
                      rtol=2e-6)


def test_trispectrum_sums_match_bruteforce_8():
    rng = np.random.default_rng(21)
    n = 8
    d = rng.standard_normal((n, n, n)).astype(np.float32)
    lo, hi = np.array([0.5, 1.5]), np.array([1.5, 2.5])
    quads = np.array([(0, 0, 1, 1), (0, 1, 1, 1), (0, 0, 0, 0), (1, 1, 1, 1)])
    res = oracle.trispectrum(d, lo, hi, quads)
    D = np.fft.fftn(oracle.prepare(d))
    m = _grid_modes(n, hi.max())
    amp = D[m[:, 0] % n, m[:, 1] % n, m[:, 2] % n]
    mem = _membership(m, lo, hi)
    for q, quad in enumerate(quads):
        idx = [np.flatnonzero(mem[:, b]) for b in quad]
        tot, cnt = 0j, 0
        for a in idx[0]:
            for b in idx[1]:
                s12 = m[a] + m[b]
                m3 = m[idx[2]]
                u = -(s12[None, :] + m3)
                w = _wrap(u, n)
                ok = _membership(w, lo, hi)[:, quad[3]]
                a4 = D[w[:, 0] % n, w[:, 1] % n, w[:, 2] % n]
                tot += np.sum(amp[a] * amp[b] * amp[idx[2]] * a4 * ok)
                cnt += int(ok.sum())
        assert res.count[q] == cnt
        assert abs(res.s[q] - tot) < 1e-9 * (1 + abs(tot))


def test_power_spectrum_parseval_and_pair_sum():
    rng = np.random.default_rng(2)
    n = 16
    d = rng.standard_normal((n, n, n)).astype(np.float32)
    lo, hi = np.array([1.0, 3.0, 5.0]), np.array([3.0, 5.0, 8.0])
    P, M = oracle.power_spectrum(d, lo, hi)
    D = np.fft.fftn(oracle.prepare(d))
    f = oracle.freq(n)
    r = np.sqrt(f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2)
    for b in range(3):
        sel = (r >= lo[b]) & (r < hi[b]) & (r > 0)
        assert M[b] == sel.sum()
        assert np.isclose(P[b], np.mean(np.abs(D[sel]) ** 2) / n ** 3, rtol=1e-12)
    # the p = 2 closed-pair sum over (S_b, S_b) is sum |Delta|^2 with M_b pairs
    mask = oracle.bin_mask_table(n, lo, hi)
    Dg = oracle.dft3(oracle.prepare(d))
    for b in range(3):
        sh = oracle.shell_modes(n, lo, hi, b)
        s = 0j
        for v in sh:
            w = (-v) % n
            s += Dg[v[0] % n, v[1] % n, v[2] % n] * Dg[w[0], w[1], w[2]]
        assert np.isclose(s.real / M[b] / n ** 3, P[b], rtol=1e-12)
    assert mask.dtype == np.uint64


def test_more_than_64_bins_match_per_triplet_bruteforce():
    """Plans beyond 64 bins: the direct sums take a bin-mask table per group
    of closing bins.  96 narrow bins on 8^3 (one per sixteenth of k_f between
    1 and 7, most of them empty); 40 closed and 10 open triplets whose bins
    include one above 64, checked against an enumeration of their mode
    triples."""
    rng = np.random.default_rng(11)
    n = 8
    d = rng.standard_normal((n, n, n)).astype(np.float32)
    edges = 1.0 + np.arange(97) / 16.0
    lo, hi = edges[:-1], edges[1:]
    D = np.fft.fftn(oracle.prepare(d))
    m = _grid_modes(n, hi[-1])
    mem = _membership(m, lo, hi)
    occupied = [b for b in range(len(lo)) if mem[:, b].any()]
    assert max(occupied) > 64

    def brute(i, j, k):
        a, b = m[mem[:, i]], m[mem[:, j]]
        u = _wrap(-(a[:, None, :] + b[None, :, :]), n).reshape(-1, 3)
        r2 = np.sum(u * u, axis=1).astype(np.float64)
        inside = (r2 > 0) & (r2 >= lo[k] ** 2) & (r2 < hi[k] ** 2)
        prod = (D[a[:, 0] % n, a[:, 1] % n, a[:, 2] % n][:, None]
                * D[b[:, 0] % n, b[:, 1] % n, b[:, 2] % n][None, :]).ravel()
        prod = prod * D[u[:, 0] % n, u[:, 1] % n, u[:, 2] % n]
        return int(inside.sum()), prod[inside].sum(), np.abs(prod[inside]).sum()

    closed, open_, ref = [], [], {}
    for t in itertools.combinations_with_replacement(occupied, 3):
        if t[2] <= 64 or (t[0] + 7 * t[1] + 13 * t[2]) % 3:
            continue
        c = brute(*t)
        if c[0] > 0 and len(closed) < 40:
            closed.append(t)
            ref[t] = c
        elif c[0] == 0 and len(open_) < 10:
            open_.append(t)
            ref[t] = c
    assert len(closed) == 40 and len(open_) == 10
    trip = closed + open_
    res = oracle.bispectrum(d, lo, hi, trip)
    for t, key in enumerate(trip):
        cnt, s, mag = ref[key]
        assert res.count[t] == cnt, key
        assert abs(res.s[t] - s) <= 1e-12 * max(1.0, mag), key
