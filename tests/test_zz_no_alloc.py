"""polyspec_estimate_noalloc: the allocation-free variant of polyspec_estimate.

Called through the C ABI on the library's static device scratch, it must
give the results of polyspec_estimate on the plan's own workspace (the same
kernels and launch shapes: bit for bit) and meet the oracle bars, on two
calls in a row whose second has a smaller input, and it must refuse a plan
whose workspace is larger than the scratch.  Device memory in use does not
change across a call.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1705_06284_amd import synth  # noqa: E402


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_06284_amd import binding as b
    return b


def _noalloc(binding, plan, d, P, B, T):
    with torch.cuda.device(plan.device):
        return binding.polyspec_estimate_noalloc(plan.handle, binding._ptr(d), d.shape[0], binding._ptr(P),
                                                 binding._ptr(B), binding._ptr(T))


def _case(binding, n, nb, batch, seeds, prec):
    lo, hi = synth.linear_bins(n, nb)
    lo, hi = lo[1:], hi[1:]                      # [0, N/(2 nb)) may hold no mode at small N
    maps = np.stack([synth.lognormal_field(n, 1.5, 1.0, seed=s) for s in seeds])
    plan = binding.Plan(n, lo, hi, precision=prec, max_batch=batch)
    d = torch.from_numpy(maps).cuda()
    want = plan.polyspec(d)
    torch.cuda.synchronize()
    P = torch.full_like(want[0], np.nan)
    B = torch.full_like(want[1], np.nan)
    T = torch.full_like(want[2], np.nan)
    return plan, lo, hi, maps, d, want, (P, B, T)


@pytest.mark.parametrize("prec", ["split_bf16", "fp32"])
def test_noalloc_two_calls_match_workspace_path(binding, prec):
    print("noalloc %s: 64^3 batch 2, then 32^3 batch 1" % prec, flush=True)
    big = _case(binding, 64, 8, 2, (901, 902), prec)
    small = _case(binding, 32, 6, 1, (903,), prec)
    free0 = None
    for plan, lo, hi, maps, d, want, out in (big, small, big):
        torch.cuda.synchronize()
        rc = _noalloc(binding, plan, d, *out)
        assert rc == 0, binding.bispec_last_error()
        torch.cuda.synchronize()
        for got, ref in zip(out, want):
            assert torch.equal(got, ref)
        # the first call in the process may load the scratch (the device keeps
        # it until the process ends); later calls allocate nothing
        if free0 is None:
            free0 = torch.cuda.mem_get_info()[0]
        assert torch.cuda.mem_get_info()[0] == free0
        ref = oracle.bispectrum(maps[0], lo, hi, plan.triplets)
        e = np.abs(out[1].cpu().numpy()[0] - ref.value) / np.maximum(np.abs(ref.value), ref.noise)
        assert e.max() <= (1e-5 if prec == "fp32" else 1e-4)
        for t in out:
            t.fill_(np.nan)


def test_noalloc_refuses_a_plan_larger_than_the_scratch(binding):
    lo, hi = synth.linear_bins(128, 16)
    plan = binding.Plan(128, lo[1:], hi[1:], precision="split_bf16")
    assert plan.workspace_bytes > (64 << 20)
    d = torch.from_numpy(synth.lognormal_field(128, 1.5, 1.0, seed=904)).cuda().unsqueeze(0)
    P, B, T = plan.polyspec(d)
    rc = _noalloc(binding, plan, d, P, B, T)
    assert rc == -5 and b"static scratch" in binding.bispec_last_error()
    # the plan keeps working on its own workspace
    P2, B2, T2 = plan.polyspec(d)
    assert torch.equal(B2, B)
