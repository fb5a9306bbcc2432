"""The request loop on the GPU: every result of a mixed, batched stream is
bitwise the result of the same map estimated alone with the same tail launch
shape, and matches the oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1705_06284_amd import serving, synth  # noqa: E402


@pytest.fixture(scope="module")
def backend():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return serving.GpuBackend()


def test_mixed_stream_equals_alone(backend):
    from paper_1705_06284_amd import binding
    print("serving: mixed 32^3/64^3 stream", flush=True)
    sizes = [32, 64, 32, 32, 64, 32, 64, 32, 32, 64, 32, 32]
    fields = {i: synth.lognormal_field(n, 1.5, 1.0, 5000 + i) for i, n in enumerate(sizes)}
    reqs = [serving.Request(rid=i, n=n, field=backend.pinned(fields[i])) for i, n in enumerate(sizes)]
    srv = serving.Server(backend, sizes=(32, 64), slots_per_size=2, max_batch=3)
    arrivals = [0.0] * 6 + [2e-3] * 6                  # a burst, then arrivals while busy
    done = srv.run(reqs, arrivals)
    assert len(done) == len(reqs) and not srv.refused
    alone = {}
    for n in (32, 64):
        lo, hi = serving.standard_bins(n)
        alone[n] = binding.Plan(n, lo, hi, triplets=serving.standard_triplets(), quads=np.zeros((1, 4), np.int32))
        alone[n].set_tuning(*backend.tuning[n])          # the slots' tail launch shape
    for r in done:
        B, P = alone[r.n].estimate(fields[r.rid])
        assert np.array_equal(B.cpu().numpy()[0], r.result["B"], equal_nan=True)
        assert np.array_equal(P.cpu().numpy()[0], r.result["P"], equal_nan=True)
    # one request against the oracle
    r = [x for x in done if x.n == 32][0]
    lo, hi = serving.standard_bins(32)
    ref = oracle.bispectrum(fields[r.rid], lo, hi, serving.standard_triplets())
    ok = ref.count > 0
    assert np.all(np.isnan(r.result["B"][~ok]))
    err = np.abs(r.result["B"][ok] - ref.value[ok]) / np.maximum(np.abs(ref.value[ok]), ref.noise[ok])
    assert np.max(err) <= 1e-4


def test_tight_budget_refuses_large_maps(backend):
    print("serving: budget admission", flush=True)
    fp32 = backend.footprint(32, 2)
    srv = serving.Server(backend, sizes=(32, 64), slots_per_size=1, max_batch=2, hbm_budget=fp32 + 1024)
    assert srv.n_slots[32] == 1 and srv.n_slots[64] == 0
    reqs = [serving.Request(rid=0, n=64, field=synth.lognormal_field(64, 1.5, 1.0, 1)),
            serving.Request(rid=1, n=32, field=synth.lognormal_field(32, 1.5, 1.0, 2))]
    srv.run(reqs, [0.0, 0.0])
    assert [r.rid for r in srv.refused] == [0] and [r.rid for r in srv.finished] == [1]
