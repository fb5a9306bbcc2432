"""GPU parity of the diagonal-binned trispectrum and of the connected T of
general quads, through the C ABI.

References: the FP64 direct sums with the diagonal test and the paired
quadruples built mode by mode (oracle/polyspec.py; pinned in
test_oracle_diag.py), and the oracle's plain trispectrum.  Metric per
result: |X - X_ref| / max(|X_ref|, X_noise), X_noise the random-phase level
of the raw sum; the pair-product spectra are FP32 transforms of FP32 fields,
held to 1e-5.  Counts N_q(e) exact.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1705_06284_amd import synth  # noqa: E402

TOL = 1e-5


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
    g = np.fft.ifftn(np.fft.fftn(w) * np.exp(-k2 * 30.0)).real
    g *= 1.0 / g.std()
    return (np.exp(g - 0.5) - 1.0).astype(np.float32)


# quad shells 0..3 (disjoint), diagonal shells 4..7 (may overlap the quad shells)
LO = np.array([1.0, 2.0, 3.0, 4.0, 0.5, 1.5, 2.5, 4.0])
HI = np.array([2.0, 3.0, 4.0, 5.0, 1.5, 2.5, 4.0, 5.5])
DQ = [(0, 1, 0, 1, 5), (0, 1, 1, 0, 6), (1, 0, 0, 1, 4), (0, 0, 1, 1, 6), (1, 1, 1, 1, 7), (0, 0, 0, 0, 5),
      (0, 1, 2, 3, 6), (1, 2, 1, 2, 7), (2, 2, 3, 3, 4), (0, 2, 1, 1, 5), (3, 1, 2, 0, 7)]
SHAPES = [(16, 16, 16), (24, 24, 24), (12, 16, 20)]


@pytest.mark.parametrize("shape", SHAPES, ids=["16cube", "24cube", "12x16x20"])
def test_diag_trispectrum_raw_and_connected(binding, shape):
    d = _field(shape, seed=sum(shape))
    L = 0.8 * shape[2]
    _say("diagonal-binned T %s, %d configurations" % (shape, len(DQ)))
    plan = binding.Plan(shape, LO, HI, triplets=[(0, 1, 2)], quads=[(0, 0, 1, 1)], box_len=L, dquads=DQ,
                        precision="split_bf16")
    assert plan.n_dquad == len(DQ)
    Td, Tdc = plan.trispec_diag(d)
    val, ref, sd = oracle.trispectrum_diag_connected(d, LO, HI, DQ, box_len=L)
    assert np.array_equal(plan.dquad_counts.astype(np.int64), ref.count)
    assert np.all(ref.count > 0)
    e = np.abs(Td.cpu().numpy()[0] - ref.value) / np.maximum(np.abs(ref.value), ref.noise)
    ec = np.abs(Tdc.cpu().numpy()[0] - val) / np.maximum(np.abs(val), ref.noise)
    _say("  raw max err %.2e, connected max err %.2e (paired share up to %.2f)"
         % (e.max(), ec.max(), np.max(np.abs(sd.real) / np.maximum(np.abs(ref.s.real), 1e-300))))
    assert e.max() <= TOL and ec.max() <= TOL


def test_diag_batch_equals_single_maps(binding):
    shape = (16, 16, 16)
    maps = np.stack([_field(shape, seed=s) for s in (5, 6)])
    plan = binding.Plan(shape, LO, HI, triplets=[(0, 1, 2)], dquads=DQ, max_batch=2)
    Td, Tdc = plan.trispec_diag(maps)
    for i in range(2):
        t1, c1 = plan.trispec_diag(maps[i])
        assert torch.equal(Td[i], t1[0]) and torch.equal(Tdc[i], c1[0])


def test_connected_part_needs_disjoint_shells(binding):
    shape = (16, 16, 16)
    plan = binding.Plan(shape, LO, HI, triplets=[(0, 1, 2)], dquads=[(0, 6, 0, 6, 5)])   # 0 = [1,2), 6 = [2.5,4): disjoint
    plan.trispec_diag(_field(shape, 1))
    plan = binding.Plan(shape, LO, HI, triplets=[(0, 1, 2)], dquads=[(2, 6, 2, 6, 5)])   # 2 = [3,4), 6 = [2.5,4)
    Td, _ = plan.trispec_diag(_field(shape, 1), connected=False)
    assert torch.isfinite(Td).all()
    with pytest.raises(binding.BispecError) as ei:
        plan.trispec_diag(_field(shape, 1))
    assert ei.value.code == -1


def test_connected_t_of_general_quads_is_the_raw_t(binding):
    """With identical or disjoint shells only (a, a, b, b) has pairings: the
    connected T of any other quad equals its raw T, and the collapsed ones
    match the oracle's connected T."""
    n = 32
    lo, hi = synth.linear_bins(n, 6)
    d = synth.lognormal_field(n, 1.5, 1.0, seed=77)
    quads = [(0, 1, 2, 3), (0, 0, 1, 2), (1, 1, 2, 2), (2, 2, 2, 2), (0, 1, 1, 2)]
    plan = binding.Plan(n, lo, hi, quads=quads)
    T, Tc = plan.trispec_connected(d)
    T, Tc = T.cpu().numpy()[0], Tc.cpu().numpy()[0]
    for q in (0, 1, 4):
        assert Tc[q] == T[q]
    val, full, _ = oracle.polyspec.trispectrum_connected(d, lo, hi, np.array([quads[2], quads[3]]))
    ec = np.abs(Tc[[2, 3]] - val) / np.maximum(np.abs(val), full.noise)
    assert ec.max() <= 1e-4
