"""The count pass under a memory limit (bispec_set_count_memory): the bins
taken in groups, the unit fields of each touched set of groups made in turn.
The integer counts, and so every normalised output, must not change.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1705_06284_amd import synth  # noqa: E402


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_06284_amd import binding as b
    return b


@pytest.mark.parametrize("shape,nb", [((64, 64, 64), 16), ((24, 30, 20), 9)], ids=["64cube", "24x30x20"])
def test_counts_under_a_memory_limit(binding, shape, nb):
    edges = np.linspace(1.0, shape[2] / 2.0, nb + 1)
    lo, hi = edges[:-1], edges[1:]
    d = synth.lognormal_field(shape[0], 1.5, 1.0, seed=9) if shape[0] == shape[1] == shape[2] else \
        np.random.default_rng(9).standard_normal(shape).astype(np.float32)
    print("count memory %s, %d bins" % (shape, nb), flush=True)
    free = binding.Plan(shape, lo, hi, precision="split_bf16")
    pair_bytes = 2 * 8 * int(np.prod(shape)) + 2 * 8 * 128
    try:
        for pairs in (3, 7):                 # room for 3 or 7 pairs: groups of one pair
            binding.check(binding.bispec_set_count_memory(pairs * pair_bytes), "bispec_set_count_memory")
            lim = binding.Plan(shape, lo, hi, precision="split_bf16")
            assert np.array_equal(lim.triplets, free.triplets)
            assert np.array_equal(lim.counts, free.counts)
            assert np.array_equal(lim.quad_counts, free.quad_counts)
            assert np.array_equal(lim.mode_counts, free.mode_counts)
            a, b = free.polyspec(d), lim.polyspec(d)
            for x, y in zip(a, b):
                assert torch.equal(x, y)
    finally:
        binding.check(binding.bispec_set_count_memory(0), "bispec_set_count_memory")
