"""Pins of the oracle's connected collapsed trispectrum (CPU).

* Brute force: on an 8^3 grid every closed quadruple of the two shells is
  enumerated and classified as paired (the four modes split into two pairs
  k_i = -k_j) or not; the paired part must equal oracle.disconnected_sums,
  which builds the three pairing sets mode by mode instead.
* Wick's theorem: for a Gaussian field the expectation of D1 D2 D3 D4 over a
  closed quadruple vanishes unless it is paired, so the connected T has
  zero mean (t-test over seeds), while the raw T does not.
"""
import itertools

import numpy as np

import oracle
from oracle import polyspec
from paper_1705_06284_amd import synth


def _wrap(c, n):
    return ((c + n // 2) % n) - n // 2


def test_disconnected_sums_match_bruteforce_8():
    rng = np.random.default_rng(31)
    n = 8
    d = rng.standard_normal((n, n, n)).astype(np.float32)
    lo, hi = np.array([0.5, 1.5]), np.array([1.5, 2.5])
    quads = np.array([(0, 0, 1, 1), (0, 0, 0, 0), (1, 1, 0, 0)])
    sd = polyspec.disconnected_sums(d, lo, hi, quads)
    D = np.fft.fftn(oracle.prepare(d))
    for q, (a, _, b, _) in enumerate(quads):
        sa = oracle.shell_modes(n, lo, hi, a).astype(np.int64)
        sb = oracle.shell_modes(n, lo, hi, b).astype(np.int64)
        inb = {tuple(m) for m in sb}
        amp = lambda m: D[m[0] % n, m[1] % n, m[2] % n]
        tot_paired, tot_all = 0j, 0j
        for k1, k2, k3 in itertools.product(sa, sa, sb):
            k4 = _wrap(-(k1 + k2 + k3), n)
            if tuple(k4) not in inb:
                continue
            ks = (k1, k2, k3, k4)
            p = amp(k1) * amp(k2) * amp(k3) * amp(k4)
            tot_all += p
            paired = any(np.all(ks[i] + ks[j] == 0) and np.all(ks[k] + ks[l] == 0)
                         for (i, j), (k, l) in (((0, 1), (2, 3)), ((0, 2), (1, 3)), ((0, 3), (1, 2))))
            if paired:
                tot_paired += p
        assert abs(sd[q] - tot_paired) < 1e-9 * (1 + abs(tot_paired))
        full = oracle.trispectrum(d, lo, hi, quads[q:q + 1])
        assert abs(full.s[0] - tot_all) < 1e-9 * (1 + abs(tot_all))


def test_connected_trispectrum_of_gaussian_fields_has_zero_mean():
    n = 16
    lo, hi = np.array([1.0, 2.0]), np.array([2.0, 3.0])
    quads = np.array([(0, 0, 1, 1), (0, 0, 0, 0), (1, 1, 1, 1)])
    conn, raw = [], []
    for seed in range(16):
        d = synth.gaussian_field(n, 1.0, 1.0, 300 + seed).astype(np.float32)
        val, full, _ = polyspec.trispectrum_connected(d, lo, hi, quads)
        conn.append(val)
        raw.append(full.value)
    conn, raw = np.array(conn), np.array(raw)
    t_conn = conn.mean(0) / (conn.std(0, ddof=1) / np.sqrt(len(conn)))
    t_raw = raw.mean(0) / (raw.std(0, ddof=1) / np.sqrt(len(raw)))
    assert np.all(np.abs(t_conn) < 4.0), t_conn
    assert np.all(np.abs(t_raw) > 5.0), t_raw           # the disconnected part dominates the raw mean
