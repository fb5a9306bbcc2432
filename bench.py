#!/usr/bin/env python3
"""Benchmark of the FFT polyspectrum estimator hot path on one MI355X.

Workload (default): 256^3 toy-reionisation map (ionised spheres of radius 8
cells until half the volume is ionised, mean subtracted), 24 linear bins from
0 to k_Nyquist, every closed triplet (1528), the power spectrum (24 bins) and
every collapsed p = 4 configuration (a,a,b,b) (300).  One step is one map
through the whole path: FP64 mean, forward FFT, 24 shell-masked inverse FFTs,
split-BF16 MFMA product-Gram contraction, FP64 reduction and normalisation.
Inputs are resident in HBM before the timed region.

Prints one JSON line.  value = closed triplets estimated per second.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "bispectrum triangles/s at 256^3 vs plain FP32 path; p50/p99 map latency"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
F32_MFMA_PEAK_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3_256_bubbles")
    ap.add_argument("--batch", type=int, default=1, help="maps per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP32 comparison paths")
    ap.add_argument("--cpu-budget", type=float, default=2e9,
                    help="pair steps of the direct-sum oracle sample")
    ap.add_argument("--cpu-bins", type=int, default=8,
                    help="bins of the FP64 FFT-form sample of the CPU baseline")
    ap.add_argument("--inverse-batch", type=int, default=4,
                    help="maps per call of the inverse-stage measurement (0: skip)")
    ap.add_argument("--no-serving", action="store_true", help="skip the request-stream measurement")
    ap.add_argument("--no-toy600", action="store_true",
                    help="skip the 600^3 toy reionisation box (mixed-radix transforms, 61 shells)")
    ap.add_argument("--no-diag", action="store_true",
                    help="skip the diagonal-binned trispectrum on the 128^3 lognormal map")
    ap.add_argument("--no-onepixel", action="store_true",
                    help="skip the one-pixel-shell measurement with configuration binning")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shape")
    ap.add_argument("--all-tunings", action="store_true",
                    help="also run 3 steps with every tail launch shape the tuner may pick (for counter runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB (5 times), the reference kernel "
                         "for scaling the HBM byte counters of a profiler run")
    return ap.parse_args()


TAIL_SOURCES = ("paper_1705_06284_amd/csrc/mfma.hip", "paper_1705_06284_amd/csrc/fft_core.hpp",
                "paper_1705_06284_amd/csrc/launch.hpp")
FFT_SOURCES = ("paper_1705_06284_amd/csrc/kernels.hip", "paper_1705_06284_amd/csrc/fft_core.hpp",
               "paper_1705_06284_amd/csrc/launch.hpp", "paper_1705_06284_amd/csrc/api.cpp")


def tail_source_hash(sources=TAIL_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_values(name, sources):
    """key: value lines of a committed counter summary, if it was taken on the
    current sources; else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != tail_source_hash(sources):
        return None
    return kv


def measured_traffic(workload, nblk, shape):
    """HBM bytes per launch of the tail kernel from the committed counter
    summary, if it was taken on the current kernel source and holds this
    launch shape (block count, shape); else None."""
    path = os.path.join(ROOT, "profiles", "k_tail_%s_traffic.txt" % workload)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != tail_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch[%d,%d]" % (nblk, int(shape))])
    except (KeyError, ValueError):
        return None


def timed_steps(torch, step, steps, stream):
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        evs[0].record(stream)
        for i in range(steps):
            step()
            evs[i + 1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat = [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]
    return t1 - t0, lat


def onepixel_run(torch, binding, synth, np, dev, stream, steps, wl="onepix_128_lognormal"):
    """Narrow shells (one k_f: 63 bins at 128^3, 127 at 256^3; the bin fields
    go to HBM, the triplets run on the split-BF16 product-Gram over them in
    groups of 64 columns, P and the collapsed T on its pass over the
    squares), against the same plan on the FP32 vector-ALU terms, and the
    table B(theta) at k2 = 2 k1 for k1 = 2..21 (20 cos theta bins each) from
    bispec_rebin."""
    n = synth.WORKLOADS[wl]["n"]
    lo, hi = synth.workload_bins(wl)
    plan = binding.Plan(n, lo, hi, stream=stream, device=dev)
    d = torch.from_numpy(synth.workload_field(wl)).to(dev).unsqueeze(0)
    P = torch.empty(1, plan.n_bins, dtype=torch.float64, device=dev)
    B = torch.empty(1, plan.n_tri, dtype=torch.float64, device=dev)
    T = torch.empty(1, plan.n_quad, dtype=torch.float64, device=dev)
    groups = []
    for b1 in range(1, 21):
        g, _ = plan.theta_groups(b1, 2 * b1 + 1, 20)
        groups.append(torch.from_numpy(g).to(dev))
    tab = torch.empty(len(groups), 20, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def est():
        binding.check(binding.polyspec_estimate(plan.handle, binding._ptr(d), 1, binding._ptr(P), binding._ptr(B),
                                                binding._ptr(T)), "polyspec_estimate")

    def rebin():
        for i, g in enumerate(groups):
            binding.check(binding.bispec_rebin(plan.handle, binding._ptr(B), 1, binding._ptr(g), 20,
                                               binding._ptr(tab[i])), "bispec_rebin")

    for _ in range(2):
        est()
        rebin()
    k = max(3, steps // 2)
    plan.timing_read()
    plan.timing(True)
    we, _ = timed_steps(torch, est, k, stream)
    plan.timing(False)
    stages, calls = plan.timing_read()
    wr, _ = timed_steps(torch, rebin, k, stream)
    out = {"workload": wl, "n": n, "bins": plan.n_bins, "triplets": plan.n_tri, "quads": plan.n_quad,
           "outputs": "B, P, T",
           "contraction": "split-BF16 MFMA product-Gram over the bin fields in HBM (%d group(s) of 64 "
                          "columns), P and T from its pass over the squares" % ((plan.n_bins + 63) // 64),
           "ms_per_map": 1e3 * we / k, "triangles_per_s": plan.n_tri * k / we,
           "stages_ms": {key: v / max(calls, 1) for key, v in stages.items()},
           "theta_table": {"configs": "k2 = 2 k1, k1 = 2..21 k_f, 20 bins of cos theta",
                           "ms": 1e3 * wr / k, "groups": int(np.isfinite(tab.cpu().numpy()).sum())}}
    # the fields product-Gram against the peak, algorithmic flops as for the
    # headline kernel: one product per pair of bins and two flops per triplet
    npix = float(n) ** 3
    flops = (2.0 * plan.n_tri + plan.n_bins * (plan.n_bins + 1) / 2) * npix   # B; P and T not counted
    ach = flops / (out["stages_ms"]["contract"] * 1e-3) / 1e12
    out["roofline"] = {"bound": "mfma", "kernel": "k_pgram_fields (triplet pass) + k_reduce_dense", "achieved": ach,
                       "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / BF16_PEAK_TFLOPS,
                       "algorithmic_flop": flops}
    plan.set_precision("fp32")
    est()
    kv = max(2, k // 2)
    wv, _ = timed_steps(torch, est, kv, stream)
    out["fp32_valu"] = {"ms_per_map": 1e3 * wv / kv, "triangles_per_s": plan.n_tri * kv / wv,
                        "kind": "simple vector-ALU kernel, not tuned (a reference point, not a competitor)"}
    return out


def toy600_run(torch, binding, synth, dev, stream, steps, wl="toy600_xhi099"):
    """The 600^3 toy box of Section 3.3 (cells of 1 Mpc, 61 shells of 2 k_f,
    every closed triplet, P and the collapsed T) on the mixed-radix
    transforms and the fields product-Gram, split-BF16."""
    w = synth.WORKLOADS[wl]
    lo, hi = synth.workload_bins(wl)
    t0 = time.perf_counter()
    plan = binding.Plan((w["n"],) * 3, lo, hi, box_len=w["box_len"], stream=stream, device=dev)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    d = torch.from_numpy(synth.workload_field(wl)).to(dev).unsqueeze(0)
    P = torch.empty(1, plan.n_bins, dtype=torch.float64, device=dev)
    B = torch.empty(1, plan.n_tri, dtype=torch.float64, device=dev)
    T = torch.empty(1, plan.n_quad, dtype=torch.float64, device=dev)

    def est():
        binding.check(binding.polyspec_estimate(plan.handle, binding._ptr(d), 1, binding._ptr(P), binding._ptr(B),
                                                binding._ptr(T)), "polyspec_estimate")

    est()
    k = max(2, steps // 4)
    plan.timing_read()
    plan.timing(True)
    we, _ = timed_steps(torch, est, k, stream)
    plan.timing(False)
    stages, calls = plan.timing_read()
    return {"workload": wl, "shape": [w["n"]] * 3, "bins": plan.n_bins, "triplets": plan.n_tri,
            "quads": plan.n_quad, "outputs": "B, P, T", "plan_s": t_plan, "ms_per_map": 1e3 * we / k,
            "triangles_per_s": plan.n_tri * k / we,
            "stages_ms": {key: v / max(calls, 1) for key, v in stages.items()}}


def diag_run(torch, binding, synth, dev, stream, steps, wl="c2_128_lognormal"):
    """The diagonal-binned trispectrum T(a, b, c, d; e) on the 128^3 lognormal
    map with 16 linear bins: (a, b, a, b; e) and (a, a, b, b; e) for
    a <= b < 4 and diagonal shells e < 8, raw and with the Gaussian pairings
    removed (one map at a time: the fields of the shells used, the pair
    products and their transforms, the shell sums)."""
    n = synth.WORKLOADS[wl]["n"]
    lo, hi = synth.workload_bins(wl)
    dq = [(a, b, a, b, e) for a in range(4) for b in range(a, 4) for e in range(8)]
    dq += [(a, a, b, b, e) for a in range(4) for b in range(a, 4) for e in range(8)]
    plan = binding.Plan(n, lo, hi, dquads=dq, stream=stream, device=dev)
    d = torch.from_numpy(synth.workload_field(wl)).to(dev).unsqueeze(0)

    def step():
        plan.trispec_diag(d, connected=True)

    step()
    k = max(3, steps // 4)
    w, _ = timed_steps(torch, step, k, stream)
    return {"workload": wl, "n": n, "bins": plan.n_bins, "configs": len(dq),
            "kinds": "(a,b,a,b;e) and (a,a,b,b;e), a <= b < 4, e < 8; raw and connected",
            "ms_per_map": 1e3 * w / k, "configs_per_s": len(dq) * k / w}


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q))


def cpu_baseline(field, lo, hi, trip, n_bins_sample=8):
    """The FP64 FFT form of the estimator (oracle/fftref.py: the paper's own
    method, Section 2, on the CPU) on a bounded sample of the same map: the
    forward FFT, the bin fields of the first n_bins_sample bins and every
    closed triplet among them."""
    import numpy as np
    from oracle import fftref
    sel = trip[np.max(trip, axis=1) < n_bins_sample]
    t0 = time.perf_counter()
    R = fftref.FFTReference(field, lo, hi)
    R.bispectrum(sel)
    dt = time.perf_counter() - t0
    threads = fftref._workers()
    return {"value": len(sel) / dt, "unit": "triangles/s", "cores": threads, "kind": "oracle",
            "sample": "FP64 FFT form of the estimator (oracle/fftref.py, scipy.fft on %d threads) on the same "
                      "%d^3 map: forward FFT, bin and count fields of bins 0..%d and their %d closed triplets "
                      "(of %d), %.1f s" % (threads, field.shape[0], n_bins_sample - 1, len(sel), len(trip), dt)}


def cpu_direct_sum(field, lo, hi, trip, budget):
    """The FP64 direct-sum oracle on the triplets whose closed-pair loops are
    cheapest (up to `budget` pair steps in total)."""
    import numpy as np
    import oracle
    m = oracle.mode_counts(field.shape[0], lo, hi)
    pair = [tuple(sorted(t, key=lambda b: (m[b], b))[:2]) for t in trip]
    cost = {p: float(m[p[0]]) * float(m[p[1]]) for p in set(pair)}
    keep, used = set(), 0.0
    for p in sorted(cost, key=lambda p: cost[p]):
        if used + cost[p] > budget:
            break
        keep.add(p)
        used += cost[p]
    sel = trip[[p in keep for p in pair]]
    t0 = time.perf_counter()
    dk = oracle.dft3(oracle.prepare(field))
    oracle.bispectrum(field, lo, hi, sel, delta_k=dk)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": len(sel) / dt, "unit": "triangles/s", "cores": threads,
            "sample": "FP64 direct sums: separable DFT plus the %d of %d closed triplets with the cheapest "
                      "closed-pair loops (%.2e pair steps), %.1f s" % (len(sel), len(trip), used, dt)}


def serving_run(n_requests, warmup=200, load=0.7, seed=5):
    """Poisson stream of 64^3/128^3/256^3 lognormal maps (4:2:1) on one GPU:
    saturation throughput from a burst, then p50/p99 latency (overall and per
    size) at `load` times that rate.  Each request asks for 12 equilateral +
    12 squeezed triplets and P at 12 bins.  Request i carries its own map,
    drawn on the device before the run from seed 5000 + i."""
    import numpy as np
    import torch
    from paper_1705_06284_amd import serving, synth
    sizes = (64, 128, 256)
    be = serving.GpuBackend()
    total = n_requests + warmup
    ns = serving.mixed_sizes(total, seed)
    maps = [synth.lognormal_field_device(int(n), 1.5, 1.0, 5000 + i, device=be.device) for i, n in enumerate(ns)]
    torch.cuda.synchronize()

    def reqs():
        return [serving.Request(rid=i, n=int(n), field=maps[i]) for i, n in enumerate(ns)]

    srv = serving.Server(be, sizes=sizes, slots_per_size=2, max_batch=4)
    burst = reqs()
    t0 = time.perf_counter()
    srv.run(burst, [0.0] * len(burst))
    sat = len(burst) / (time.perf_counter() - t0)
    srv.finished.clear()
    rate = load * sat
    arr = serving.poisson_arrivals(rate, total, seed)
    t0 = time.perf_counter()
    done = srv.run(reqs(), list(arr))
    wall = time.perf_counter() - t0
    measured = [r for r in done if r.rid >= warmup]
    summ = serving.latency_summary(measured)
    ntri = 24
    summ.update({"rate_maps_per_s": rate, "saturation_maps_per_s": sat, "maps_per_s": len(done) / wall,
                 "triangles_per_s": len(done) * ntri / wall, "requests": len(measured), "warmup": warmup,
                 "mix": "64^3:128^3:256^3 = 4:2:1, one map per request (seed 5000 + id), 12 equilateral + "
                        "12 squeezed + P, slots 2/size, batch <= 4"})
    del maps
    return summ


def inverse_stage(torch, binding, plan_args, field, dev, stream, batch, steps):
    """The shell-masked inverse passes Z and Y of every bin pair on `batch`
    copies of the map (batch 4 at 256^3 puts 4 x 1.2 GB through HBM, far past
    the 256 MB Infinity Cache): stage time per call, and bytes per second
    from the committed counter summary when it was taken on these sources."""
    import numpy as np
    n, lo, hi = plan_args
    plan = binding.Plan(n, lo, hi, precision="split_bf16", max_batch=batch, stream=stream, device=dev)
    d = torch.from_numpy(np.broadcast_to(field, (batch,) + field.shape).copy()).to(dev)
    P = torch.empty(batch, plan.n_bins, dtype=torch.float64, device=dev)
    B = torch.empty(batch, plan.n_tri, dtype=torch.float64, device=dev)
    T = torch.empty(batch, plan.n_quad, dtype=torch.float64, device=dev)

    def step():
        binding.check(binding.polyspec_estimate(plan.handle, binding._ptr(d), batch, binding._ptr(P),
                                                binding._ptr(B), binding._ptr(T)), "polyspec_estimate")
    for _ in range(3):
        step()
    torch.cuda.synchronize()
    plan.timing_read()
    plan.timing(True)
    timed_steps(torch, step, steps, stream)
    plan.timing(False)
    st, calls = plan.timing_read()
    ms = st["inverse"] / max(calls, 1)
    npix = float(n) ** 3
    modes = plan.mode_counts.astype(np.float64)
    algo = float(np.sum(modes) * 8 + plan.n_bins * npix * 4) * batch
    out = {"batch": batch, "kernels": "k_inv_z_prune + k_inv_y_prune", "stage_ms": ms,
           "algorithmic_bytes": algo, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    kv = profile_values("fft_%dcube_traffic.txt" % n, FFT_SOURCES)
    if kv is not None and kv.get("batch") == str(batch):
        try:
            byts = float(kv["inverse_zy_bytes_per_call"])
            out["traffic"] = byts
            out["achieved"] = byts / (ms * 1e-3) / 1e9
            out["frac"] = out["achieved"] / HBM_PEAK_GBS
        except (KeyError, ValueError):
            pass
    plan.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the estimator runs every map on a single MI355X "
              "(maps shard across GPUs without communication); --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1705_06284_amd import binding, synth

    wl = args.workload
    n = synth.WORKLOADS[wl]["n"]
    lo, hi = synth.workload_bins(wl)
    field = synth.workload_field(wl)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    bsz = args.batch
    plan = binding.Plan(n, lo, hi, precision="split_bf16", max_batch=bsz, stream=stream, device=dev)
    ntri, nq, nb = plan.n_tri, plan.n_quad, plan.n_bins
    d = torch.from_numpy(np.broadcast_to(field, (bsz,) + field.shape).copy()).to(dev)
    tuned = plan.autotune(d[:1]) if not args.no_autotune else (None, None)
    P = torch.empty(bsz, nb, dtype=torch.float64, device=dev)
    B = torch.empty(bsz, ntri, dtype=torch.float64, device=dev)
    T = torch.empty(bsz, nq, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def step():
        binding.check(binding.polyspec_estimate(plan.handle, binding._ptr(d), bsz, binding._ptr(P),
                                                binding._ptr(B), binding._ptr(T)), "polyspec_estimate")

    def run(prec, steps, warmup, timing=False):
        plan.set_precision(prec)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        plan.timing_read()
        plan.timing(timing)
        wall, lat = timed_steps(torch, step, steps, stream)
        plan.timing(False)
        stages, calls = plan.timing_read()
        return wall, lat, {k: v / max(calls, 1) for k, v in stages.items()}

    wall, lat, stages = run("split_bf16", args.steps, args.warmup, timing=True)
    value = ntri * bsz * args.steps / wall
    out = {"metric": METRIC, "value": value, "unit": "triangles/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32 FFT + bf16x3 MFMA contraction",
           "data": "synthetic",
           "config": {"workload": wl, "n": n, "bins": nb, "triplets": ntri, "quads": nq, "batch": bsz,
                      "precision": "split_bf16", "outputs": "B, P, T"},
           "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)},
           "stages_ms": stages, "tuning": {"tail_blocks": tuned[0], "tail_shape": ["deep", "wide", "twin"][tuned[1]]
                                            if tuned[1] is not None else None}}

    # dominant kernel and its roofline
    npix = float(n) ** 3
    modes = plan.mode_counts.astype(np.float64)
    pairs = nb * (nb + 1) // 2
    con_ms = stages["contract"] / bsz
    inv_ms = stages["inverse"] / bsz
    if con_ms >= inv_ms:
        flops = (2.0 * ntri + pairs) * npix          # algorithmic: pair products + one FMA per triplet
        ach = flops / (con_ms * 1e-3) / 1e12
        traffic = measured_traffic(wl, tuned[0], tuned[1]) if bsz == 1 and tuned[0] else None
        out["roofline"] = {"bound": "mfma", "achieved": ach, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": ach / BF16_PEAK_TFLOPS, "traffic": traffic,
                           "kernel": "k_tail<split> (last inverse pass + split-BF16 product-Gram)",
                           "launch_ms": con_ms, "algorithmic_flop": flops}
    else:
        byts = float(np.sum(modes) * 8 + nb * npix * 4)   # shell modes read + bin fields written
        ach = byts / (inv_ms * 1e-3) / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS, "traffic": None, "kernel": "inverse FFT stage"}

    # tail kernel alone, in triangles/s (the contraction-only rate)
    out["tail_triangles_per_s"] = ntri * bsz / (stages["contract"] * 1e-3) if stages["contract"] > 0 else None

    # the same steps replayed from a captured HIP graph (no stage events)
    plan.set_precision("split_bf16")
    plan.graph(True)
    step()
    torch.cuda.synchronize()
    wg, latg = timed_steps(torch, step, args.steps, stream)
    plan.graph(False)
    out["graph_replay"] = {"value": ntri * bsz * args.steps / wg, "ms_per_step": 1e3 * wg / args.steps,
                           "latency_ms": {"p50": percentile(latg, 50), "p99": percentile(latg, 99)}}

    if not args.no_compare:
        # comparisons: the connected collapsed T (Gaussian pairings removed)
        # against the raw T alone, same plan and map; then the FP32 paths
        Tc = torch.empty_like(T)

        def t_only():
            binding.check(binding.polyspec_estimate(plan.handle, binding._ptr(d), bsz, None, None, binding._ptr(T)),
                          "polyspec_estimate")

        def t_conn():
            binding.check(binding.trispec_connected_estimate(plan.handle, binding._ptr(d), bsz, binding._ptr(T),
                                                             binding._ptr(Tc)), "trispec_connected_estimate")

        t_only()
        t_conn()
        w_t, _ = timed_steps(torch, t_only, args.steps, stream)
        w_c, _ = timed_steps(torch, t_conn, args.steps, stream)
        out["connected_T"] = {"quads": nq, "ms_per_map_raw_T": 1e3 * w_t / (args.steps * bsz),
                              "ms_per_map_connected": 1e3 * w_c / (args.steps * bsz)}
        w32, lat32, st32 = run("fp32", args.steps, 2, timing=True)
        wv, latv, stv = run("fp32_valu", max(3, args.steps // 4), 1, timing=True)
        kv = max(3, args.steps // 4)
        out["fp32_path"] = {"value": ntri * bsz * args.steps / w32, "ms_per_step": 1e3 * w32 / args.steps,
                            "contract_ms": st32["contract"], "kind": "same product-Gram on FP32 MFMA"}
        out["fp32_valu_path"] = {"value": ntri * bsz * kv / wv, "ms_per_step": 1e3 * wv / kv,
                                 "contract_ms": stv["contract"],
                                 "kind": "requested sums only, FP32 vector ALU (simple kernel, not tuned: "
                                         "a reference point, not a competitor)"}
        out["split_vs_fp32"] = {"end_to_end": out["fp32_path"]["ms_per_step"] / out["ms_per_step"],
                                "contraction": st32["contract"] / max(stages["contract"], 1e-9)}
        plan.set_precision("split_bf16")

    if args.inverse_batch > 0 and bsz == 1:
        out["roofline_inverse"] = inverse_stage(torch, binding, (n, lo, hi), field, dev, stream,
                                                args.inverse_batch, max(5, args.steps // 2))

    if not args.no_onepixel:
        out["onepixel_128"] = onepixel_run(torch, binding, synth, np, dev, stream, args.steps)
        out["onepixel_256"] = onepixel_run(torch, binding, synth, np, dev, stream, args.steps,
                                           wl="onepix_256_lognormal")

    if not args.no_toy600:
        out["toy600"] = toy600_run(torch, binding, synth, dev, stream, args.steps)

    if not args.no_diag:
        out["diag_T"] = diag_run(torch, binding, synth, dev, stream, args.steps)

    if not args.no_serving:
        out["serving"] = serving_run(args.serving_requests)

    if args.all_tunings:
        ran = []
        for shape in (binding.TAIL_DEEP, binding.TAIL_WIDE, binding.TAIL_TWIN):
            for nblk in (256, 512, 1024, 2048, 4096, 8192, 16384):
                try:
                    plan.set_tuning(nblk, shape)
                except binding.BispecError:
                    continue
                for _ in range(3):
                    step()
                ran.append([nblk, shape])
        torch.cuda.synchronize()
        if tuned[0]:
            plan.set_tuning(*tuned)
        out["all_tunings"] = ran

    if args.copy_calibration > 0:
        cnt = args.copy_calibration * (1 << 18)
        src = torch.ones(cnt, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"bytes_read": 4 * cnt, "bytes_written": 4 * cnt, "launches": 5}
        del src, dst

    # measured HBM copy rate on this machine (device-to-device copy of 512 MiB),
    # after the GPU measurements so that it does not disturb them (not in
    # counter runs, whose last copies are the calibration)
    if args.copy_calibration <= 0:
        src = torch.ones(1 << 27, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        out["hbm_copy_GBps"] = 5 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del src, dst
        # a library BF16 GEMM (8192^3, contiguous operands) as the practical
        # matrix-core ceiling on this machine, and the tail kernel against it
        a = torch.randn(8192, 8192, device=dev).to(torch.bfloat16)
        b = torch.randn(8192, 8192, device=dev).to(torch.bfloat16)
        torch.mm(a, b)
        e0.record()
        for _ in range(5):
            torch.mm(a, b)
        e1.record()
        torch.cuda.synchronize()
        gemm = 5 * 2 * 8192.0 ** 3 / (e0.elapsed_time(e1) * 1e-3) / 1e12
        out["gemm_bf16_TFLOPs"] = gemm
        if out["roofline"]["unit"] == "TFLOP/s":
            out["roofline"]["frac_of_measured_gemm"] = out["roofline"]["achieved"] / gemm
        del a, b

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(field, lo, hi, plan.triplets, args.cpu_bins)
        out["cpu_direct_sum"] = cpu_direct_sum(field, lo, hi, plan.triplets, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
