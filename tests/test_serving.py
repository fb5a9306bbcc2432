"""Scheduling logic of the request loop, on the CPU with a modelled backend.

The modelled backend stands in for the GPU: each launch finishes after a
duration proportional to the batch's grid points, on a simulated clock.
"""
import numpy as np
import pytest

from paper_1705_06284_amd import serving


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-5          # every query advances time a little
        return self.t


class ModelBackend:
    def __init__(self, clock, sec_per_point=1e-9):
        self.clock = clock
        self.k = sec_per_point
        self.launches = []

    def footprint(self, n, max_batch):
        return 10 * n ** 3 * max_batch

    def make_slot(self, n, max_batch):
        return {"n": n, "until": 0.0, "fields": []}

    def launch(self, slot, fields):
        assert len(fields) >= 1
        slot["fields"] = list(fields)
        slot["until"] = self.clock.t + self.k * sum(f.size for f in fields)
        self.launches.append((slot["n"], len(fields)))

    def ready(self, slot):
        return self.clock.t >= slot["until"]

    def collect(self, slot):
        return [{"sum": float(np.sum(f))} for f in slot["fields"]]


def _requests(sizes, seed=0):
    rng = np.random.default_rng(seed)
    return [serving.Request(rid=i, n=int(n), field=rng.standard_normal((n, n, n)).astype(np.float32))
            for i, n in enumerate(sizes)]


def test_every_request_is_served_with_its_own_result():
    clock = Clock()
    be = ModelBackend(clock)
    srv = serving.Server(be, sizes=(8, 16), slots_per_size=2, max_batch=3, clock=clock)
    reqs = _requests([8, 16, 8, 8, 16, 8, 8, 16, 16, 8])
    done = srv.run(reqs, list(np.linspace(0, 1e-3, len(reqs))))
    assert len(done) == len(reqs) and not srv.refused
    for r in done:
        assert r.result["sum"] == pytest.approx(float(np.sum(r.field)))
        assert r.done >= r.arrival
    assert all(k <= 3 for _, k in be.launches)


def test_requests_arriving_while_busy_join_later_batches():
    clock = Clock()
    be = ModelBackend(clock, sec_per_point=1e-6)      # slow device: queues build up
    srv = serving.Server(be, sizes=(16,), slots_per_size=1, max_batch=4, clock=clock)
    reqs = _requests([16] * 9)
    srv.run(reqs, [0.0] + [1e-4] * 8)                   # one early, eight while it runs
    assert be.launches[0] == (16, 1)
    assert [k for _, k in be.launches[1:]] == [4, 4]   # continuous batching of the waiting ones
    assert len(srv.finished) == 9


def test_admission_by_hbm_footprint():
    clock = Clock()
    be = ModelBackend(clock)
    budget = be.footprint(8, 2) * 2 + be.footprint(16, 2)   # room for 2 small slots and 1 medium
    srv = serving.Server(be, sizes=(8, 16, 32), slots_per_size=2, max_batch=2, hbm_budget=budget, clock=clock)
    assert len(srv.slots[8]) == 2 and len(srv.slots[16]) == 1 and len(srv.slots[32]) == 0
    assert srv.committed <= budget
    reqs = _requests([8, 32, 16])
    srv.run(reqs, [0.0, 0.0, 0.0])
    assert [r.rid for r in srv.refused] == [1]
    assert "HBM budget" in srv.refused[0].error
    assert sorted(r.rid for r in srv.finished) == [0, 2]


def test_fifo_within_a_size_class():
    clock = Clock()
    be = ModelBackend(clock, sec_per_point=1e-6)
    srv = serving.Server(be, sizes=(8,), slots_per_size=1, max_batch=2, clock=clock)
    reqs = _requests([8] * 6)
    srv.run(reqs, [0.0] * 6)
    order = [r.rid for r in srv.finished]
    assert order == sorted(order)


def test_arrival_and_size_generators():
    a = serving.poisson_arrivals(100.0, 2000, seed=5)
    assert np.all(np.diff(a) > 0) and abs(len(a) / a[-1] - 100.0) < 10.0
    s = serving.mixed_sizes(7000, seed=5)
    frac = np.array([np.mean(s == n) for n in (64, 128, 256)])
    assert np.allclose(frac, [4 / 7, 2 / 7, 1 / 7], atol=0.02)
    lo, hi = serving.standard_bins(64)
    assert len(lo) == 13 and lo[-1] == 0.5 and hi[-1] == 1.5
    t = serving.standard_triplets()
    assert len(t) == 24 and tuple(t[12]) == (0, 0, 12)
