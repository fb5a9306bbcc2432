"""GPU parity of plans with more than 64 bins (narrow shells; the paper's
advice of one-k_f shells, Section 3.2 and the Conclusion, gives 127 shells
at 256^3), through the C ABI.

The triplets run on the product-Gram over the bin fields in HBM, one pass per
group of 64 columns; P and the collapsed quads on the pass over the squared
fields (P and T on the vector ALUs when n_bins is a multiple of 64).
References: the FP64 direct sums (oracle/polyspec.py; beyond 64 bins pinned
in test_oracle_sums.py).  Metric per result: |X - X_ref| / max(|X_ref|,
X_noise); split-BF16 1e-4; FP32 1e-5 up to kappa 40 (beyond it the FP32 FFTs'
own rounding, about 2.5e-7 kappa, passes 1e-5) and 1e-4 for every triplet; P
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


def _field(shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal(shape)
    k2 = sum(np.meshgrid(*[np.fft.fftfreq(n) ** 2 for n in shape], indexing="ij"))
    g = np.fft.ifftn(np.fft.fftn(w) * np.exp(-k2 * 40.0)).real
    g *= 1.0 / g.std()
    return (np.exp(g - 0.5) - 1.0).astype(np.float32)


def _one_radius_bins(n, nb):
    """One bin per occupied |m|^2 of the cubic grid, the nb smallest:
    [sqrt(q - 1/2), sqrt(q + 1/2)), the narrowest shells a grid has."""
    f = oracle.freq(n)
    q = np.unique((f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2).ravel())
    q = q[q > 0][:nb].astype(np.float64)
    assert len(q) == nb and q[-1] < (n / 2) ** 2
    return np.sqrt(q - 0.5), np.sqrt(q + 0.5)


CASES = [
    ((32, 32, 32), 96),      # two column groups, ones column in the second
    ((32, 32, 32), 128),     # two full groups: P and T on the vector ALUs
    ((24, 24, 24), 80),      # mixed-radix grid
]


@pytest.mark.parametrize("shape,nb", CASES, ids=["32cube-96", "32cube-128", "24cube-80"])
@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_every_triplet_power_and_collapsed_quads(binding, shape, nb, prec):
    lo, hi = _one_radius_bins(shape[0], nb)
    d = _field(shape, seed=nb + shape[0])
    _say("%s, %d one-radius bins up to %.2f k_f, %s" % (shape, nb, hi[-1], prec))
    plan = binding.Plan(shape, lo, hi, precision=prec)
    trip = plan.triplets
    want, cnt = oracle.closed_triplets(shape, lo, hi)
    assert np.array_equal(trip, want) and np.array_equal(plan.counts.astype(np.int64), cnt)
    assert np.array_equal(plan.mode_counts, oracle.mode_counts(shape, lo, hi))
    P, B, T = plan.polyspec(d)
    ref = oracle.bispectrum(d, lo, hi, trip)
    e = np.abs(B.cpu().numpy()[0] - ref.value) / np.maximum(np.abs(ref.value), ref.noise)
    kappa = plan.condition
    refp, _ = oracle.power_spectrum(d, lo, hi)
    ep = np.abs(P.cpu().numpy()[0] - refp) / refp
    quads = plan.quads
    rng = np.random.default_rng(nb)
    sel = np.sort(rng.choice(len(quads), size=min(60, len(quads)), replace=False))
    reft = oracle.trispectrum(d, lo, hi, quads[sel])
    assert np.array_equal(np.rint(plan.quad_counts[sel]).astype(np.int64), reft.count)
    et = np.abs(T.cpu().numpy()[0][sel] - reft.value) / np.maximum(np.abs(reft.value), reft.noise)
    w = int(np.argmax(e))
    _say("  %d triplets max err %.2e at %s (kappa %.1f), P %.2e, %d quads %.2e"
         % (len(trip), e[w], tuple(trip[w]), kappa[w], ep.max(), len(sel), et.max()))
    assert ep.max() <= TOL[prec] and et.max() <= TOL[prec]
    if prec == "split_bf16":
        assert e.max() <= TOL[prec]
    else:
        assert e[kappa <= 40.0].max() <= TOL["fp32"] and e.max() <= TOL["split_bf16"]


def test_bin_fields_beyond_64(binding):
    shape, nb = (32, 32, 32), 80
    lo, hi = _one_radius_bins(32, nb)
    d = _field(shape, seed=3)
    _say("bin fields, %d bins" % nb)
    plan = binding.Plan(shape, lo, hi, precision="split_bf16", triplets=[(70, 75, 79)])
    F = plan.bin_fields(d).cpu().numpy()[0].astype(np.float64)
    D = np.fft.fftn(oracle.prepare(d))
    f = oracle.freq(32)
    q = f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2
    for b in (0, 63, 64, 79):
        M = (q > 0) & (q >= lo[b] ** 2) & (q < hi[b] ** 2)
        ref = np.fft.ifftn(D * M).real * 32 ** 3
        assert np.max(np.abs(F[b] - ref)) <= 2e-6 * max(np.max(np.abs(ref)), 1e-30), b


def test_resident_bin_fields(binding):
    """bin_fields(keep=True) leaves the fields in the workspace and
    polyspec(None) contracts them: bitwise the same P, B, T as from the map;
    an estimate from a map leaves its fields resident too.  Plans whose
    contraction is fused with the last transform have no field region."""
    shape, nb = (32, 32, 32), 70
    lo, hi = _one_radius_bins(32, nb)
    maps = np.stack([_field(shape, seed=s) for s in (21, 22)])
    plan = binding.Plan(shape, lo, hi, precision="split_bf16", max_batch=2)
    ref = plan.polyspec(maps)
    plan.bin_fields(maps[:1], keep=True)
    with pytest.raises(binding.BispecError) as ei:
        plan.polyspec(None, batch=2)             # one map resident, not two
    assert ei.value.code == -1
    one = plan.polyspec(None, batch=1)
    plan.polyspec(maps)                           # leaves both maps' fields resident
    two = plan.polyspec(None, batch=2)
    for a, b, c in zip(ref, one, two):
        assert torch.equal(a[:1], b) and torch.equal(a, c)
    fused = binding.Plan(32, *synth.linear_bins(32, 8), precision="split_bf16")
    with pytest.raises(binding.BispecError) as ei:
        fused.bin_fields(maps[0], keep=True)
    assert ei.value.code == -5
    with pytest.raises(binding.BispecError) as ei:
        fused.polyspec(None)
    assert ei.value.code == -1


@pytest.mark.parametrize("shape,nb", [((32, 32, 32), 96), ((24, 24, 24), 80), ((64, 64, 64), 40)],
                         ids=["32cube-96", "24cube-80", "64cube-40-narrow"])
def test_batch_of_two_equals_single_maps(binding, shape, nb):
    """Every kernel indexes maps by grid.y and reduces each map in a fixed
    order, so a map's results do not depend on the batch it runs in: the
    column groups, the squares pass, the refinement of ill-conditioned
    triplets (40 shells of 0.75 k_f at 64^3 reach kappa ~ 100) and (24^3)
    the pruned mixed-radix transforms, bit for bit."""
    if nb == 40:
        lo = 1.0 + 0.75 * np.arange(nb)
        hi = lo + 0.75
    else:
        lo, hi = _one_radius_bins(shape[0], nb)
    maps = np.stack([_field(shape, seed=s) for s in (3, 4)])
    for prec in ("fp32", "split_bf16"):
        plan = binding.Plan(shape, lo, hi, precision=prec, max_batch=2)
        kappa = plan.condition
        _say("%s, %d bins, %s: batch of 2 vs single (%d triplets above kappa 2.5)"
             % (shape, nb, prec, int((kappa > 2.5).sum())))
        if nb == 40:
            assert (kappa > 2.5).sum() > 0          # the refinement runs
        P, B, T = plan.polyspec(maps)
        for i in range(2):
            p1, b1, t1 = plan.polyspec(maps[i])
            assert torch.equal(B[i], b1[0]) and torch.equal(P[i], p1[0]) and torch.equal(T[i], t1[0]), prec
