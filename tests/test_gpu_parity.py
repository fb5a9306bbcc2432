"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Metric (per result): err = |X_gpu - X_oracle| / max(|X_oracle|, X_noise),
with X_noise = norm * sqrt(sum |product|^2) / count from the oracle (the
random-phase noise level of the mean over closed tuples).  FP32 contraction:
err <= 1e-5; split-BF16 contraction: err <= 1e-4.  P is positive, so plain
relative error applies.  Tuple counts are integers and must match exactly.
"""
import itertools
import os

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


def _err(got, ref):
    return np.abs(got - ref.value) / np.maximum(np.abs(ref.value), ref.noise)


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_c1_equilateral_power_32(binding, prec):
    n = 32
    lo, hi = synth.unit_bins(1, 8)
    trip = np.array([(b, b, b) for b in range(8)], np.int32)
    d = synth.local_quadratic_field(n, 2.0, 0.1, 0.5, seed=1)
    _say("c1 32^3 equilateral %s" % prec)
    plan = binding.Plan(n, lo, hi, triplets=trip, precision=prec)
    B, P = plan.estimate(d)
    ref = oracle.bispectrum(d, lo, hi, trip)
    refp, m = oracle.power_spectrum(d, lo, hi)
    assert np.array_equal(plan.counts.astype(np.int64), ref.count)
    assert np.array_equal(plan.mode_counts, m)
    assert np.max(_err(B.cpu().numpy()[0], ref)) <= TOL[prec]
    assert np.max(np.abs(P.cpu().numpy()[0] - refp) / refp) <= TOL[prec]


@pytest.mark.parametrize("n,nb", [(16, 4), (32, 6), (32, 8)])
def test_auto_triplet_set_and_counts(binding, n, nb):
    lo, hi = synth.linear_bins(n, nb)
    _say("auto triplets n=%d nb=%d" % (n, nb))
    plan = binding.Plan(n, lo, hi, precision="fp32")
    want, cnt = oracle.closed_triplets(n, lo, hi)
    got = plan.triplets
    assert np.array_equal(got, want)
    assert np.array_equal(plan.counts.astype(np.int64), cnt)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_all_triplets_lognormal_32(binding, prec):
    n = 32
    lo, hi = synth.linear_bins(n, 8)
    d = synth.lognormal_field(n, 1.5, 1.0, seed=12)
    _say("all triplets 32^3 %s" % prec)
    plan = binding.Plan(n, lo, hi, precision=prec)
    P, B, T = plan.polyspec(d)
    ref = oracle.bispectrum(d, lo, hi, plan.triplets)
    e = _err(B.cpu().numpy()[0], ref)
    assert np.max(e) <= TOL[prec], (np.max(e), plan.triplets[np.argmax(e)])
    refp, _ = oracle.power_spectrum(d, lo, hi)
    assert np.max(np.abs(P.cpu().numpy()[0] - refp) / refp) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_collapsed_trispectrum_32(binding, prec):
    n = 32
    lo, hi = synth.linear_bins(n, 6)
    d = synth.lognormal_field(n, 1.5, 1.0, seed=5)
    _say("collapsed trispectrum 32^3 %s" % prec)
    plan = binding.Plan(n, lo, hi, precision=prec)
    quads = plan.quads
    assert len(quads) == 21
    T = plan.trispec(d).cpu().numpy()[0]
    sel = [q for q in range(len(quads)) if quads[q][0] <= 1 and quads[q][2] <= 2]
    ref = oracle.trispectrum(d, lo, hi, quads[sel])
    assert np.array_equal(plan.quad_counts[sel].astype(np.int64), ref.count)
    assert np.max(_err(T[sel], ref)) <= TOL[prec]


def test_bin_fields_match_masked_inverse_dft(binding):
    n = 32
    lo, hi = np.array([1.0, 4.0, 9.0]), np.array([4.0, 9.0, 16.0])     # odd bin count
    d = synth.lognormal_field(n, 1.0, 0.7, seed=8)
    _say("bin fields 32^3")
    plan = binding.Plan(n, lo, hi, precision="fp32")
    F = plan.bin_fields(d).cpu().numpy()[0].astype(np.float64)
    D = oracle.dft3(oracle.prepare(d))
    f = oracle.freq(n)
    r2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2
    for b in range(3):
        M = (r2 > 0) & (r2 >= lo[b] ** 2) & (r2 < hi[b] ** 2)
        ref = np.fft.ifftn(D * M).real * n ** 3       # unnormalised inverse
        assert np.max(np.abs(F[b] - ref)) <= 2e-6 * np.max(np.abs(ref))


def test_batch_equals_single_maps(binding):
    n = 32
    lo, hi = synth.linear_bins(n, 5)
    maps = np.stack([synth.lognormal_field(n, 1.5, 1.0, seed=s) for s in (1, 2, 3)])
    _say("batch of 3 vs single")
    for prec in ("fp32", "split_bf16"):
        plan = binding.Plan(n, lo, hi, precision=prec, max_batch=3)
        for shape in (binding.TAIL_WIDE, binding.TAIL_TWIN, binding.TAIL_DEEP):
            plan.set_tuning(32, shape)             # 32^3: 64 units of 512 points, 32 blocks
            P, B, T = plan.polyspec(maps)
            for i in range(3):
                p1, b1, t1 = plan.polyspec(maps[i])
                assert torch.equal(B[i], b1[0]) and torch.equal(P[i], p1[0]) and torch.equal(T[i], t1[0]), (prec, shape)


def test_overlapping_bins_and_explicit_zero_count(binding):
    """Squeezed configurations with a one-pixel k3 shell that overlaps bin 0,
    and an explicit triplet with no closed triangle (NaN)."""
    n = 64
    lo, hi = synth.linear_bins(n, 12)
    lo = np.append(lo, 0.5)
    hi = np.append(hi, 1.5)
    sq = 12
    trip = [(b, b, b) for b in range(12)] + [(b, b, sq) for b in range(12)] + [(0, 0, 11)]
    d = synth.lognormal_field(n, 1.5, 1.0, seed=5001)
    _say("squeezed + overlapping bins 64^3")
    plan = binding.Plan(n, lo, hi, triplets=trip, precision="fp32")
    B, P = plan.estimate(d)
    b = B.cpu().numpy()[0]
    assert np.isnan(b[-1]) and plan.counts[-1] == 0
    ref = oracle.bispectrum(d, lo, hi, trip[:-1])
    assert np.max(_err(b[:-1], ref)) <= TOL["fp32"]


def _cheap_triplets(n, lo, hi, trip, budget):
    """Triplets whose direct sum the oracle finishes within `budget` pair steps
    in total: the oracle loops over the two smallest shells of a triplet, and
    triplets sharing that pair share one loop."""
    m = oracle.mode_counts(n, lo, hi)
    pair = [tuple(sorted(t, key=lambda b: (m[b], b))[:2]) for t in trip]
    cost = {p: float(m[p[0]]) * float(m[p[1]]) for p in set(pair)}
    keep, used = set(), 0.0
    for p in sorted(cost, key=lambda p: cost[p]):
        if used + cost[p] > budget:
            break
        keep.add(p)
        used += cost[p]
    return trip[[p in keep for p in pair]]


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_c2_lognormal_128_sampled(binding, prec):
    n = 128
    lo, hi = synth.workload_bins("c2_128_lognormal")
    d = synth.workload_field("c2_128_lognormal")
    _say("c2 128^3 sampled %s" % prec)
    plan = binding.Plan(n, lo, hi, precision=prec)
    P, B, T = plan.polyspec(d, want_t=False)
    trip = plan.triplets
    assert len(trip) == 508
    sel = _cheap_triplets(n, lo, hi, trip, 2e9)
    idx = [int(np.flatnonzero((trip == t).all(1))[0]) for t in sel]
    Dk = oracle.dft3(oracle.prepare(d))
    ref = oracle.bispectrum(d, lo, hi, sel, delta_k=Dk)
    assert np.array_equal(plan.counts[idx].astype(np.int64), ref.count)
    e = _err(B.cpu().numpy()[0][idx], ref)
    _say("  %d sampled triplets, max err %.2e" % (len(sel), e.max()))
    assert np.max(e) <= TOL[prec]
    refp, _ = oracle.power_spectrum(d, lo, hi, delta_k=Dk)
    assert np.max(np.abs(P.cpu().numpy()[0] - refp) / refp) <= TOL[prec]


def test_valu_contraction_and_general_quads(binding):
    """The vector-ALU contraction (mode 2) and non-collapsed p = 4 configurations."""
    n = 32
    lo, hi = synth.linear_bins(n, 6)
    d = synth.lognormal_field(n, 1.5, 1.0, seed=9)
    trip = np.array([(0, 1, 1), (1, 2, 2), (0, 2, 2), (2, 2, 2)], np.int32)
    quads = np.array([(0, 1, 1, 2), (0, 0, 1, 1), (1, 1, 1, 1)], np.int32)
    _say("valu contraction + general quads 32^3")
    ref_b = oracle.bispectrum(d, lo, hi, trip)
    ref_t = oracle.trispectrum(d, lo, hi, quads)
    for prec in ("fp32_valu", "split_bf16"):
        plan = binding.Plan(n, lo, hi, triplets=trip, quads=quads, precision=prec)
        P, B, T = plan.polyspec(d)
        assert np.array_equal(plan.quad_counts.astype(np.int64), ref_t.count)
        assert np.max(_err(B.cpu().numpy()[0], ref_b)) <= TOL[prec if prec != "fp32_valu" else "fp32"]
        assert np.max(_err(T.cpu().numpy()[0], ref_t)) <= 1e-5   # general quads always take FP32


@pytest.mark.parametrize("n", [8, 16, 128])
def test_small_and_medium_grids(binding, n):
    """Every FFT length path (radix 8 with a 2- or 4-point tail) and tiny grids.
    Linear bins from 0 (from k_f/2 at 8^3, where [0, 1) holds no mode)."""
    e = np.linspace(0.5 if n == 8 else 0.0, n / 2, 5)
    lo, hi = e[:-1], e[1:]
    d = synth.lognormal_field(n, 1.0, 0.8, seed=n)
    _say("grid %d^3" % n)
    plan = binding.Plan(n, lo, hi, precision="split_bf16")
    P, B, T = plan.polyspec(d)
    trip = plan.triplets
    sel = _cheap_triplets(n, lo, hi, trip, 5e8)
    idx = [int(np.flatnonzero((trip == t).all(1))[0]) for t in sel]
    ref = oracle.bispectrum(d, lo, hi, sel)
    assert np.array_equal(plan.counts[idx].astype(np.int64), ref.count)
    assert np.max(_err(B.cpu().numpy()[0][idx], ref)) <= TOL["split_bf16"]
    refp, _ = oracle.power_spectrum(d, lo, hi)
    assert np.max(np.abs(P.cpu().numpy()[0] - refp) / refp) <= TOL["split_bf16"]


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_c3_bubbles_256_sampled(binding, prec):
    """The benchmark workload: 256^3 toy-reionisation map, 24 bins, every closed
    triplet and collapsed quad, in the bench launch configuration (batch 1)."""
    n = 256
    wl = "c3_256_bubbles"
    lo, hi = synth.workload_bins(wl)
    d = synth.workload_field(wl)
    _say("c3 256^3 sampled %s" % prec)
    plan = binding.Plan(n, lo, hi, precision=prec)
    trip = plan.triplets
    assert len(trip) == 1522 and plan.n_quad == 300
    sel = _cheap_triplets(n, lo, hi, trip, 2e9)
    idx = [int(np.flatnonzero((trip == t).all(1))[0]) for t in sel]
    Dk = oracle.dft3(oracle.prepare(d))
    ref = oracle.bispectrum(d, lo, hi, sel, delta_k=Dk)
    assert np.array_equal(plan.counts[idx].astype(np.int64), ref.count)
    refp, _ = oracle.power_spectrum(d, lo, hi, delta_k=Dk)
    quads = plan.quads
    qsel = [q for q in range(len(quads)) if quads[q][2] <= 1]
    reft = oracle.trispectrum(d, lo, hi, quads[qsel], delta_k=Dk)
    assert np.array_equal(plan.quad_counts[qsel].astype(np.int64), reft.count)
    # every tail launch shape the tuner can pick, at the default block count
    # (512: no block contracts more than 64 units of 512 points) and the largest
    for nblk, shape in ((512, binding.TAIL_WIDE), (512, binding.TAIL_TWIN), (2048, binding.TAIL_TWIN),
                        (512, binding.TAIL_DEEP)):
        plan.set_tuning(nblk, shape)
        P, B, T = plan.polyspec(d)
        e = _err(B.cpu().numpy()[0][idx], ref)
        _say("  shape %d, %d blocks: %d sampled triplets, max err %.2e" % (shape, nblk, len(sel), e.max()))
        assert np.max(e) <= TOL[prec]
        assert np.max(np.abs(P.cpu().numpy()[0] - refp) / refp) <= TOL[prec]
        assert np.max(_err(T.cpu().numpy()[0][qsel], reft)) <= TOL[prec]


def test_empty_shell_is_rejected(binding):
    """[0, 1) holds only the mean mode, which no shell contains."""
    with pytest.raises(binding.BispecError) as ei:
        binding.Plan(8, [0.0, 1.0], [1.0, 2.0])
    assert ei.value.code == -4


def test_graph_replay_matches_eager(binding):
    """Captured launch sequences replayed several times, with other device work
    and synchronisations in between, give the eager results bit for bit."""
    n = 64
    lo, hi = synth.linear_bins(n, 8)
    a = torch.from_numpy(synth.lognormal_field(n, 1.5, 1.0, 71)).cuda().unsqueeze(0)
    b = torch.from_numpy(synth.lognormal_field(n, 1.5, 1.0, 72)).cuda().unsqueeze(0)
    _say("graph replay 64^3")
    plan = binding.Plan(n, lo, hi, precision="split_bf16", stream=torch.cuda.Stream())
    ref = {}
    for name, m in (("a", a), ("b", b)):
        P, B, T = plan.polyspec(m)
        torch.cuda.synchronize()
        ref[name] = (P.clone(), B.clone(), T.clone())
    plan.graph(True)
    inp = a.clone()
    out = (torch.empty_like(ref["a"][0]), torch.empty_like(ref["a"][1]), torch.empty_like(ref["a"][2]))
    junk = torch.randn(1 << 20, device="cuda")
    for rep, name in enumerate(["a", "a", "b", "a", "b", "b"]):
        inp.copy_(a if name == "a" else b)
        torch.cuda.synchronize()
        with torch.cuda.stream(plan.stream):
            plan.polyspec(inp, out=out)
        torch.cuda.synchronize()
        for got, want in zip(out, ref[name]):
            assert torch.equal(got, want), (rep, name)
        junk.mul_(1.0001).add_(0.5)          # eager work between replays
        torch.cuda.synchronize()
    plan.graph(False)


def test_autotune_choices_agree_with_oracle(binding):
    """Every launch shape the tuner may pick gives oracle parity; the tuner's
    pick is one of them and out-of-range choices are refused."""
    n = 64
    lo, hi = synth.linear_bins(n, 8)
    d = synth.lognormal_field(n, 1.5, 1.0, seed=81)
    _say("autotune 64^3")
    plan = binding.Plan(n, lo, hi, precision="split_bf16")
    ref = oracle.bispectrum(d, lo, hi, plan.triplets)
    refp, _ = oracle.power_spectrum(d, lo, hi)
    assert plan.autotune()[0] in (256, 512)          # on zero rows
    nb, shape = plan.autotune(d)
    # 512 units of 512 points: at least 8 blocks (64 units each), default 256, at most 512
    assert nb in (256, 512) and shape in (binding.TAIL_WIDE, binding.TAIL_TWIN, binding.TAIL_DEEP)
    for blocks in (8, 100, 256, 512):
        for sh in (binding.TAIL_WIDE, binding.TAIL_TWIN, binding.TAIL_DEEP):
            plan.set_tuning(blocks, sh)
            P, B, T = plan.polyspec(d)
            assert np.max(_err(B.cpu().numpy()[0], ref)) <= TOL["split_bf16"], (blocks, sh)
            assert np.max(np.abs(P.cpu().numpy()[0] - refp) / refp) <= TOL["split_bf16"], (blocks, sh)
    for bad, sh in ((0, 1), (7, 1), (513, 1), (256, 3), (256, -1)):
        with pytest.raises(binding.BispecError) as ei:
            plan.set_tuning(bad, sh)
        assert ei.value.code == -1


def test_condition_numbers_match_counts(binding):
    """kappa_t = sqrt(M_i M_j M_k / (N_pix N_t)) from the oracle's exact counts."""
    n = 32
    lo, hi = synth.linear_bins(n, 8)
    plan = binding.Plan(n, lo, hi, precision="fp32")
    m = oracle.mode_counts(n, lo, hi)
    _, cnt = oracle.closed_triplets(n, lo, hi)
    t = plan.triplets.astype(np.int64)
    want = np.sqrt(m[t[:, 0]] * m[t[:, 1]] * m[t[:, 2]] / (float(n) ** 3 * cnt))
    assert np.allclose(plan.condition, want, rtol=1e-14, atol=0)


@pytest.mark.parametrize("prec", ["split_bf16"])
def test_c4_lognormal_512_sampled(binding, prec):
    """512^3 lognormal field, 32 bins: the full triplet set (3384), P, and the
    collapsed quads, checked on the triplets the oracle finishes quickly."""
    n = 512
    wl = "c4_512_lognormal"
    lo, hi = synth.workload_bins(wl)
    d = synth.workload_field(wl)
    _say("c4 512^3 sampled %s" % prec)
    plan = binding.Plan(n, lo, hi, precision=prec)
    P, B, T = plan.polyspec(d)
    trip = plan.triplets
    assert len(trip) == 3384 and plan.n_quad == 528
    sel = _cheap_triplets(n, lo, hi, trip, 1.5e9)
    idx = [int(np.flatnonzero((trip == t).all(1))[0]) for t in sel]
    _say("  oracle DFT 512^3")
    Dk = oracle.dft3(oracle.prepare(d))
    ref = oracle.bispectrum(d, lo, hi, sel, delta_k=Dk)
    assert np.array_equal(plan.counts[idx].astype(np.int64), ref.count)
    e = _err(B.cpu().numpy()[0][idx], ref)
    _say("  %d sampled triplets, max err %.2e" % (len(sel), e.max()))
    assert np.max(e) <= TOL[prec]
    refp, _ = oracle.power_spectrum(d, lo, hi, delta_k=Dk)
    assert np.max(np.abs(P.cpu().numpy()[0] - refp) / refp) <= TOL[prec]
