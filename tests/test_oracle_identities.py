"""Identity and statistical pins of the oracle.

* Discrete skewness (Eq. skew, Section 1): with bins tiling every mode
  0 < |m| < N/2 of a band-limited field, the ordered sum of all triplet sums
  S_ijk equals N_pix^2 sum_n delta(n)^3.
* Invariances: periodic translation, axis permutation and reflection.
* Below N/3 the modulo-N and the strict closures coincide (Section 3,
  the k_max = N k_f / 3 argument around Eq. delta_sefusatti).
* A Gaussian field has zero bispectrum on average (Section 3.1).
* The local quadratic field delta = g + f (g^2 - <g^2>) has the tree-level
  bispectrum 2 f (P1 P2 + P2 P3 + P3 P1), averaged over the triangles of the
  bin as the paper does for theory curves (Section 3.3, bin-averaged theory).
"""
import itertools

import numpy as np

import oracle
from paper_1705_06284_amd import synth


def _bandlimited(n, seed, kmax):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, n, n))
    D = np.fft.fftn(d)
    f = np.fft.fftfreq(n, 1.0 / n)
    r2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2
    D[r2 >= kmax ** 2] = 0
    D[0, 0, 0] = 0
    return np.fft.ifftn(D).real


def test_discrete_skewness_identity():
    n = 16
    d = _bandlimited(n, 4, n / 2)
    # fields used by the oracle are FP32: band-limit the rounded field again
    d32 = d.astype(np.float32)
    edges = np.array([0.5, 1.5, 2.5, 3.5, 4.5, 5.5, 6.5, 7.5, 8.0])
    lo, hi = edges[:-1], edges[1:]
    nb = len(lo)
    trip = np.array(list(itertools.combinations_with_replacement(range(nb), 3)))
    res = oracle.bispectrum(d32, lo, hi, trip)
    ordered = 0.0
    for t, (i, j, k) in enumerate(trip):
        ordered += len(set(itertools.permutations((i, j, k)))) * res.s[t]
    x = oracle.prepare(d32)
    X = np.fft.fftn(x)
    f = np.fft.fftfreq(n, 1.0 / n)
    r2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2
    X[r2 >= (n / 2) ** 2] = 0
    xt = np.fft.ifftn(X).real
    rhs = float(n) ** 6 * np.sum(xt ** 3)
    assert abs(ordered.imag) < 1e-9 * abs(rhs)
    assert np.isclose(ordered.real, rhs, rtol=1e-9)


def _some_triplets():
    lo, hi = np.array([1.0, 2.5, 4.0, 5.5]), np.array([2.5, 4.0, 5.5, 7.0])
    return lo, hi, oracle.candidate_triplets(lo, hi)


def test_translation_rotation_reflection_invariance():
    n = 16
    d = synth.lognormal_field(n, 1.5, 0.8, 7)
    lo, hi, trip = _some_triplets()
    base = oracle.bispectrum(d, lo, hi, trip)
    for g in (np.roll(d, (3, -5, 7), axis=(0, 1, 2)),
              np.transpose(d, (2, 0, 1)),
              d[::-1, :, :],
              d[:, :, ::-1]):
        r = oracle.bispectrum(np.ascontiguousarray(g), lo, hi, trip)
        assert np.array_equal(r.count, base.count)
        scale = np.max(np.abs(base.value))
        assert np.max(np.abs(r.value - base.value)) < 1e-9 * scale


def test_strict_equals_mod_n_below_third():
    n = 24
    lo, hi = np.array([1.0, 3.0, 5.0]), np.array([3.0, 5.0, 8.0])    # hi <= N/3
    trip = oracle.candidate_triplets(lo, hi)
    d = synth.lognormal_field(n, 1.0, 0.5, 3)
    r = oracle.bispectrum(d, lo, hi, trip)
    assert np.array_equal(r.count, r.count_strict)
    assert np.allclose(r.s, r.s_strict, rtol=0, atol=1e-12 * np.abs(r.s).max())
    # and with hi up to N/2 aliasing appears
    lo2, hi2 = np.array([4.0, 8.0]), np.array([8.0, 12.0])
    c, cs = oracle.triangle_counts(n, lo2, hi2, [(1, 1, 1)])
    assert c[0] > cs[0]


def test_gaussian_field_has_zero_mean_bispectrum():
    n = 16
    lo, hi, trip = _some_triplets()
    vals = []
    for seed in range(24):
        g = synth.gaussian_field(n, 2.0, 1.0, 100 + seed).astype(np.float32)
        vals.append(oracle.bispectrum(g, lo, hi, trip).value)
    vals = np.array(vals)
    t = vals.mean(0) / (vals.std(0, ddof=1) / np.sqrt(len(vals)))
    assert np.max(np.abs(t)) < 4.5


def _tree_level_bin_average(G, n, lo, hi, b):
    """avg over closed ordered triples of bin (b,b,b) of P1P2 + P2P3 + P3P1,
    with P(m) = |G(m)|^2 / N_pix, enumerated directly."""
    f = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    mz, my, mx = np.meshgrid(f, f, f, indexing="ij")
    r2 = mz ** 2 + my ** 2 + mx ** 2
    sel = (r2 > 0) & (r2 >= lo[b] ** 2) & (r2 < hi[b] ** 2)
    m = np.stack([mz[sel], my[sel], mx[sel]], 1)
    P = np.abs(G[sel]) ** 2 / n ** 3
    m3 = -(m[:, None, :] + m[None, :, :])
    m3 = ((m3 + n // 2) % n) - n // 2
    q = np.sum(m3 * m3, -1)
    ok = (q > 0) & (q >= lo[b] ** 2) & (q < hi[b] ** 2)
    P3 = np.abs(G[m3[..., 0] % n, m3[..., 1] % n, m3[..., 2] % n]) ** 2 / n ** 3
    tot = (P[:, None] * P[None, :] + P[None, :] * P3 + P3 * P[:, None])[ok]
    return tot.mean()


def test_local_quadratic_tree_level():
    """B(f) - B(-f) on one Gaussian g isolates the O(f) term, whose
    expectation is 2 * 2 f (P1P2 + P2P3 + P3P1) bin-averaged (Wick).

    The realisation-to-realisation scatter of the O(f) term is large at these
    mode counts (the small-N_tri sample-variance regime of Section 3.2), so
    the check is statistical: 16 seeds, each bin within 4 standard errors
    and the mean over bins within 8 %.  A lost factor of 2 or a wrong
    normalisation power fails it.
    """
    n, f_nl, sigma = 32, 0.5, 0.1
    lo = np.array([2.0, 4.0, 6.0])
    hi = lo + 2.0
    trip = [(b, b, b) for b in range(len(lo))]
    ratios = []
    for seed in range(16):
        g = synth.gaussian_field(n, 1.5, sigma, seed)
        G = np.fft.fftn(g)
        g2 = g * g - np.mean(g * g)
        bp = oracle.bispectrum(g + f_nl * g2, lo, hi, trip).value
        bm = oracle.bispectrum(g - f_nl * g2, lo, hi, trip).value
        want = np.array([2 * f_nl * _tree_level_bin_average(G, n, lo, hi, b) for b in range(len(lo))])
        ratios.append(0.5 * (bp - bm) / want)
    ratios = np.array(ratios)
    mean = ratios.mean(0)
    sem = ratios.std(0, ddof=1) / np.sqrt(len(ratios))
    assert np.all(np.abs(mean - 1) < 4 * sem + 0.02), (mean, sem)
    assert abs(mean.mean() - 1) < 0.08, mean
