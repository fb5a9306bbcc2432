"""Request loop for the estimator: continuous batching of mixed-size maps.

The paper notes that the FFT estimator's speed suits sampling applications
(Section 2, after Eq. Jeong_BI), where maps arrive one after another.  This
module serves such a stream on one GPU:

* Every size class (grid side N) owns a few *slots*.  A slot is one plan with
  its own HIP stream, workspace, input buffer of ``max_batch`` maps and output
  buffers; everything stays resident on the device.
* Slots are created at start-up while their HBM footprint fits the budget;
  requests of a size class without a slot are refused (admission by HBM
  footprint).
* Requests queue per size class.  Whenever a slot is free, the waiting
  requests of its class (up to ``max_batch``) are copied in and launched as one
  batch on the slot's stream, so work of several slots overlaps on the device
  and requests that arrive while others run join the next free slot
  (continuous batching, not a queue alone).
* Completion is polled with events; latency = completion time - arrival time.

Per-map arithmetic does not depend on the other maps of a batch (every
kernel indexes maps by grid.y and reduces each map in a fixed order), so a
result is bitwise the same alone and in any mix (with the same tail launch
shape; all slots of a size class share the one their first slot tuned).

The scheduling logic talks to a backend with five methods (``footprint``,
``make_slot``, ``launch``, ``ready``, ``collect``); ``GpuBackend`` drives the
HIP library through ``binding``.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np

from . import synth


@dataclasses.dataclass
class Request:
    rid: int
    n: int
    field: object                     # FP32 [N, N, N] host map: numpy array or pinned torch tensor
    arrival: float = 0.0
    done: float = 0.0
    result: Optional[dict] = None
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def standard_bins(n: int, n_bins: int = 12):
    """n_bins linear bins of width N/(2 n_bins) from 0, plus the one-pixel shell
    [1/2, 3/2) used as k_3 of the squeezed configurations."""
    lo, hi = synth.linear_bins(n, n_bins)
    return np.append(lo, 0.5), np.append(hi, 1.5)


def standard_triplets(n_bins: int = 12):
    """Equilateral (b, b, b) and squeezed (b, b, k_f shell) configurations."""
    sq = n_bins
    return np.array([(b, b, b) for b in range(n_bins)] + [(b, b, sq) for b in range(n_bins)], np.int32)


class GpuBackend:
    """Slots on one GPU through the C ABI (binding.Plan on its own stream)."""

    def __init__(self, device="cuda:0", precision="split_bf16", n_bins=12):
        import torch
        from . import binding
        self.torch = torch
        self.binding = binding
        self.device = torch.device(device)
        self.precision = precision
        self.n_bins = n_bins
        self.tuning = {}          # size class -> (tail blocks, tail shape)

    def _plan(self, n, max_batch, stream):
        lo, hi = standard_bins(n, self.n_bins)
        return self.binding.Plan(n, lo, hi, triplets=standard_triplets(self.n_bins), quads=np.zeros((1, 4), np.int32),
                                 precision=self.precision, max_batch=max_batch, stream=stream, device=self.device)

    def footprint(self, n, max_batch) -> int:
        """Workspace + input + output bytes of one slot."""
        plan = self._plan(n, max_batch, self.torch.cuda.current_stream(self.device))
        ws = plan.workspace_bytes
        out = 8 * max_batch * (plan.n_tri + plan.n_bins)
        plan.close()
        return ws + 4 * max_batch * n ** 3 + out

    def make_slot(self, n, max_batch):
        torch = self.torch
        stream = torch.cuda.Stream(self.device)
        plan = self._plan(n, max_batch, stream)
        # one tail launch shape per size class, so that a map's result does
        # not depend on the slot that serves it
        if n not in self.tuning:
            self.tuning[n] = plan.autotune()
        else:
            plan.set_tuning(*self.tuning[n])
        plan.graph(True)          # the slot's buffers are fixed: replay captured launches
        slot = {
            "n": n, "plan": plan, "stream": stream, "max_batch": max_batch,
            "inp": torch.empty(max_batch, n, n, n, dtype=torch.float32, device=self.device),
            "host": torch.empty(max_batch, n, n, n, dtype=torch.float32).pin_memory(),
            "B": torch.empty(max_batch, plan.n_tri, dtype=torch.float64, device=self.device),
            "P": torch.empty(max_batch, plan.n_bins, dtype=torch.float64, device=self.device),
            "Bh": torch.empty(max_batch, plan.n_tri, dtype=torch.float64).pin_memory(),
            "Ph": torch.empty(max_batch, plan.n_bins, dtype=torch.float64).pin_memory(),
            "event": None, "count": 0,
        }
        return slot

    def pinned(self, field) -> "object":
        """A page-locked host copy of a map, so its upload can be asynchronous."""
        t = self.torch.from_numpy(np.ascontiguousarray(field, dtype=np.float32))
        return t.pin_memory()

    def launch(self, slot, fields: List[object]):
        torch, b = self.torch, self.binding
        k = len(fields)
        with torch.cuda.stream(slot["stream"]):
            for i, f in enumerate(fields):
                if isinstance(f, np.ndarray):          # unpinned: stage through the slot's buffer
                    slot["host"][i].copy_(torch.from_numpy(f))
                    f = slot["host"][i]
                slot["inp"][i].copy_(f, non_blocking=True)
            plan = slot["plan"]
            b.check(b.polyspec_estimate(plan.handle, b._ptr(slot["inp"]), k, b._ptr(slot["P"]),
                                        b._ptr(slot["B"]), None), "polyspec_estimate")
            slot["Bh"][:k].copy_(slot["B"][:k], non_blocking=True)
            slot["Ph"][:k].copy_(slot["P"][:k], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(slot["stream"])
        slot["event"] = ev
        slot["count"] = k

    def ready(self, slot) -> bool:
        return slot["event"] is None or slot["event"].query()

    def collect(self, slot) -> List[dict]:
        k = slot["count"]
        return [{"B": slot["Bh"][i].numpy().copy(), "P": slot["Ph"][i].numpy().copy()} for i in range(k)]


class Server:
    """Continuous-batching request loop over a backend (see module docstring)."""

    def __init__(self, backend, sizes=(64, 128, 256), slots_per_size=2, max_batch=4,
                 hbm_budget: Optional[int] = None, clock: Callable[[], float] = time.perf_counter):
        self.backend = backend
        self.clock = clock
        self.max_batch = max_batch
        self.queues: Dict[int, collections.deque] = {n: collections.deque() for n in sizes}
        self.slots: Dict[int, list] = {n: [] for n in sizes}
        self.busy: Dict[int, list] = {n: [] for n in sizes}       # (slot, [requests])
        self.n_slots: Dict[int, int] = {n: 0 for n in sizes}      # slots of each class, free or busy
        self.committed = 0
        self.refused: List[Request] = []
        self.finished: List[Request] = []
        # smallest classes first, so a tight budget still serves them
        for n in sorted(sizes):
            fp = backend.footprint(n, max_batch)
            for _ in range(slots_per_size):
                if hbm_budget is not None and self.committed + fp > hbm_budget:
                    break
                self.slots[n].append(backend.make_slot(n, max_batch))
                self.n_slots[n] += 1
                self.committed += fp

    # -- request side -------------------------------------------------------
    def submit(self, req: Request):
        if req.n not in self.queues or self.n_slots[req.n] == 0:
            req.error = "no slot fits the HBM budget for N=%d" % req.n
            req.done = self.clock()
            self.refused.append(req)
            return False
        self.queues[req.n].append(req)
        return True

    # -- device side --------------------------------------------------------
    def poll(self):
        """Retire batches whose events completed; returns the number retired."""
        retired = 0
        for n, lst in self.busy.items():
            keep = []
            for slot, reqs in lst:
                if self.backend.ready(slot):
                    now = self.clock()
                    for r, res in zip(reqs, self.backend.collect(slot)):
                        r.result = res
                        r.done = now
                        self.finished.append(r)
                    self.slots[n].append(slot)
                    retired += 1
                else:
                    keep.append((slot, reqs))
            self.busy[n] = keep
        return retired

    def schedule(self):
        """Launch waiting requests on free slots; returns the number launched."""
        launched = 0
        for n, q in self.queues.items():
            while q and self.slots[n]:
                slot = self.slots[n].pop()
                reqs = [q.popleft() for _ in range(min(self.max_batch, len(q)))]
                self.backend.launch(slot, [r.field for r in reqs])
                self.busy[n].append((slot, reqs))
                launched += len(reqs)
        return launched

    def idle(self) -> bool:
        return not any(self.queues.values()) and not any(self.busy.values())

    def run(self, requests: List[Request], arrivals: List[float]):
        """Real-time loop: request i arrives at arrivals[i] seconds after start."""
        t0 = self.clock()
        i = 0
        while i < len(requests) or not self.idle():
            now = self.clock() - t0
            while i < len(requests) and arrivals[i] <= now:
                requests[i].arrival = t0 + arrivals[i]
                self.submit(requests[i])
                i += 1
            self.poll()
            self.schedule()
        return self.finished


def poisson_arrivals(rate: float, count: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def mixed_sizes(count: int, seed: int, sizes=(64, 128, 256), weights=(4, 2, 1)) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.asarray(weights, float) / np.sum(weights)
    return rng.choice(np.asarray(sizes), size=count, p=p)


def latency_summary(finished: List[Request]) -> dict:
    lat = np.array([r.latency for r in finished]) * 1e3
    if lat.size == 0:
        return {"p50_ms": None, "p99_ms": None, "count": 0}
    out = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "mean_ms": float(lat.mean()), "count": int(lat.size), "by_size": {}}
    for n in sorted({r.n for r in finished}):
        ln = np.array([r.latency for r in finished if r.n == n]) * 1e3
        out["by_size"][str(n)] = {"p50_ms": float(np.percentile(ln, 50)), "p99_ms": float(np.percentile(ln, 99)),
                                  "count": int(ln.size)}
    return out
