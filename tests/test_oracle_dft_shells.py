"""Pins of the oracle's forward DFT and shell construction.

The DFT is the unnormalised forward transform of Eq. (DeltaFFTtoDelta); the
shells follow the spherical reading of the bin rule of Eq. (gen_Nspec3) with
the Nyquist cut of Eq. (nyqvist).  Each test checks the oracle against an
independent computation: a brute-force sum, a library FFT, Parseval, or a
plain enumeration of integer vectors.
"""
import itertools

import numpy as np
import pytest

import oracle


def test_dft_matches_bruteforce_sum():
    rng = np.random.default_rng(11)
    n = 4
    d = rng.standard_normal((n, n, n))
    got = oracle.dft3(d)
    for mz, my, mx in itertools.product(range(n), repeat=3):
        s = 0j
        for z, y, x in itertools.product(range(n), repeat=3):
            s += d[z, y, x] * np.exp(-2j * np.pi * (mz * z + my * y + mx * x) / n)
        assert abs(got[mz, my, mx] - s) < 1e-12 * (1 + abs(s))


@pytest.mark.parametrize("n", [8, 16, 32])
def test_dft_matches_numpy_fft(n):
    rng = np.random.default_rng(n)
    d = rng.standard_normal((n, n, n))
    got = oracle.dft3(d)
    ref = np.fft.fftn(d)
    assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref))


def test_dft_parseval_and_hermitian():
    rng = np.random.default_rng(3)
    n = 16
    d = rng.standard_normal((n, n, n))
    D = oracle.dft3(d)
    assert np.isclose(np.sum(np.abs(D) ** 2), n ** 3 * np.sum(d * d), rtol=1e-12)
    # real input: Delta(-m) = conj Delta(m)
    idx = (-np.arange(n)) % n
    Dm = D[idx][:, idx][:, :, idx]
    assert np.max(np.abs(Dm - np.conj(D))) < 1e-10


def _brute_shell(n, lo, hi):
    """Enumerate integer vectors directly: lo <= |m| < hi, m != 0, components in [-N/2, N/2)."""
    out = []
    r = range(-(n // 2), n // 2)
    for z in r:
        for y in r:
            for x in r:
                q = z * z + y * y + x * x
                if q > 0 and lo * lo <= q < hi * hi:
                    out.append((z, y, x))
    return sorted(out)


def test_unit_bin_mode_counts_32():
    lo = np.arange(1, 9) - 0.5
    hi = np.arange(1, 9) + 0.5
    got = oracle.mode_counts(32, lo, hi)
    # brute-force enumeration with a different loop structure
    ref = [len(_brute_shell(32, lo[b], hi[b])) for b in range(8)]
    assert list(got) == ref
    # |m|^2 in {1, 2} for the first shell: 6 axis + 12 face-diagonal vectors
    assert got[0] == 18


@pytest.mark.parametrize("n,nb", [(16, 4), (16, 8), (32, 6)])
def test_linear_bins_modes_match_enumeration(n, nb):
    e = np.arange(nb + 1) * (n / 2) / nb
    lo, hi = e[:-1], e[1:]
    for b in range(nb):
        got = sorted(map(tuple, oracle.shell_modes(n, lo, hi, b).tolist()))
        assert got == _brute_shell(n, lo[b], hi[b])


def test_shells_exclude_dc_and_nyquist():
    n = 16
    lo, hi = np.array([0.0, 4.0]), np.array([4.0, 8.0])
    for b in range(2):
        m = oracle.shell_modes(n, lo, hi, b)
        assert not np.any(np.all(m == 0, axis=1))
        assert not np.any(m == -n // 2)
    # together the two shells tile every mode with 0 < |m| < N/2
    tot = sum(len(oracle.shell_modes(n, lo, hi, b)) for b in range(2))
    assert tot == len(_brute_shell(n, 0.0, 8.0))


def test_mask_table_agrees_with_shells():
    n = 16
    lo, hi = np.array([0.5, 2.0, 2.5]), np.array([1.5, 3.0, 5.0])  # overlapping bins allowed
    mask = oracle.bin_mask_table(n, lo, hi)
    for b in range(3):
        m = oracle.shell_modes(n, lo, hi, b).astype(np.int64)
        r2 = np.sum(m * m, axis=1)
        assert np.all((mask[r2] >> np.uint64(b)) & np.uint64(1))
        f = oracle.freq(n).astype(np.int64)
        all_r2 = np.unique(f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2)
        flagged = all_r2[((mask[all_r2] >> np.uint64(b)) & np.uint64(1)).astype(bool)]
        assert np.array_equal(flagged, np.unique(r2))
