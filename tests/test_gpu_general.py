"""GPU parity on grids that are not cubic powers of two (mixed-radix
Stockham transforms, non-cubic boxes of cubic cells), through the C ABI.

References: the FP64 direct sums over closed tuples (oracle/polyspec.py,
pinned on non-cubic and odd grids in test_oracle_noncubic.py).  Metric per
result: |X - X_ref| / max(|X_ref|, X_noise); FP32 1e-5, split-BF16 1e-4; P
plain relative error; counts exact.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1705_06284_amd import synth  # noqa: E402

TOL = {"fp32": 1e-5, "split_bf16": 1e-4}


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_06284_amd import binding as b
    return b


def _say(msg):
    print(msg, flush=True)


def _err(got, ref):
    return np.abs(got - ref.value) / np.maximum(np.abs(ref.value), ref.noise)


def _field(shape, seed):
    """A lognormal-like field on any grid (exp of smoothed white noise)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal(shape)
    k2 = sum(np.meshgrid(*[np.fft.fftfreq(n) ** 2 for n in shape], indexing="ij"))
    g = np.fft.ifftn(np.fft.fftn(w) * np.exp(-k2 * 40.0)).real
    g *= 1.0 / g.std()
    return (np.exp(g - 0.5) - 1.0).astype(np.float32)


CASES = [
    ((24, 24, 24), np.linspace(1.0, 12.0, 9)),
    ((30, 30, 30), np.linspace(0.5, 15.0, 9)),
    ((40, 48, 60), np.linspace(1.0, 30.0, 11)),
    ((14, 21, 28), np.linspace(1.0, 14.0, 8)),
]


@pytest.mark.parametrize("shape,edges", CASES, ids=["24cube", "30cube", "40x48x60", "14x21x28"])
@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_every_triplet_power_and_collapsed_quads(binding, shape, edges, prec):
    lo, hi = edges[:-1], edges[1:]
    d = _field(shape, seed=sum(shape))
    L = 0.75 * shape[2]
    _say("general grid %s, %d bins, %s" % (shape, len(lo), prec))
    plan = binding.Plan(shape, lo, hi, precision=prec, box_len=L)
    trip = plan.triplets
    want, cnt = oracle.closed_triplets(shape, lo, hi)
    assert np.array_equal(trip, want) and np.array_equal(plan.counts.astype(np.int64), cnt)
    assert np.array_equal(plan.mode_counts, oracle.mode_counts(shape, lo, hi))
    P, B, T = plan.polyspec(d)
    ref = oracle.bispectrum(d, lo, hi, trip, box_len=L)
    e = _err(B.cpu().numpy()[0], ref)
    refp, _ = oracle.power_spectrum(d, lo, hi, box_len=L)
    ep = np.abs(P.cpu().numpy()[0] - refp) / refp
    quads = plan.quads
    sel = [q for q in range(len(quads)) if quads[q][2] <= 2]
    reft = oracle.trispectrum(d, lo, hi, quads[sel], box_len=L)
    assert np.array_equal(plan.quad_counts[sel].astype(np.int64), reft.count)
    et = _err(T.cpu().numpy()[0][sel], reft)
    _say("  %d triplets max err %.2e, P %.2e, %d quads %.2e" % (len(trip), e.max(), ep.max(), len(sel), et.max()))
    assert e.max() <= TOL[prec] and ep.max() <= TOL[prec] and et.max() <= TOL[prec]


@pytest.mark.parametrize("shape", [(30, 30, 30), (12, 20, 28)])
def test_bin_fields_match_masked_inverse_fft(binding, shape):
    d = _field(shape, seed=7)
    nx = shape[2]
    edges = np.linspace(1.0, nx / 2.0, 4)
    lo, hi = edges[:-1], edges[1:]
    _say("general bin fields %s" % (shape,))
    plan = binding.Plan(shape, lo, hi, precision="fp32")
    F = plan.bin_fields(d).cpu().numpy()[0].astype(np.float64)
    D = np.fft.fftn(oracle.prepare(d))
    s = oracle.polyspec.q_scales(shape)
    f = [oracle.freq(n) for n in shape]
    q = ((s[0] * f[0])[:, None, None] ** 2 + (s[1] * f[1])[None, :, None] ** 2 + (s[2] * f[2])[None, None, :] ** 2)
    lo2, hi2 = oracle.squared_edges(lo, hi, shape)
    for b in range(3):
        M = (q > 0) & (q >= lo2[b]) & (q < hi2[b])
        ref = np.fft.ifftn(D * M).real * np.prod(shape)
        assert np.max(np.abs(F[b] - ref)) <= 2e-6 * np.max(np.abs(ref)), b


def test_batch_equals_single_maps(binding):
    shape = (20, 24, 30)
    edges = np.linspace(1.0, 15.0, 7)
    lo, hi = edges[:-1], edges[1:]
    maps = np.stack([_field(shape, seed=s) for s in (1, 2)])
    _say("general batch of 2 vs single")
    for prec in ("fp32", "split_bf16"):
        plan = binding.Plan(shape, lo, hi, precision=prec, max_batch=2)
        P, B, T = plan.polyspec(maps)
        for i in range(2):
            p1, b1, t1 = plan.polyspec(maps[i])
            assert torch.equal(B[i], b1[0]) and torch.equal(P[i], p1[0]) and torch.equal(T[i], t1[0]), prec


def test_connected_trispectrum_is_refused_on_general_grids(binding):
    shape = (24, 24, 24)
    edges = np.linspace(1.0, 12.0, 4)
    plan = binding.Plan(shape, edges[:-1], edges[1:], quads=[(0, 0, 1, 1)])
    with pytest.raises(binding.BispecError) as ei:
        plan.trispec_connected(_field(shape, 3))
    assert ei.value.code == -2
