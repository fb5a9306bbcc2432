#!/usr/bin/env python3
"""Write the FP64 reference values of the large parity workloads.

Calls only ``oracle/`` (the FP64 FFT form of the estimator, pinned to the
direct sums in tests/test_oracle_fftref.py) and the seeded input generators
of ``paper_1705_06284_amd/synth.py``.  Nothing here touches the HIP path.
Each workload's values go to ``tests/golden/<workload>.fftref.npz`` together
with a digest of the input map (FP64 moments and a strided sample), which
the GPU tests compare with the map they generate before they use the values.

Configuration sets (Eq. Jeong_BI, Eq. Jeong_PS, Eq. Jeong_gen with p = 4):

* c2_128_lognormal, c3_256_bubbles: every closed triplet (the candidates of
  the triangle test whose FFT count is non-zero), every bin's P and every
  collapsed quad (a,a,b,b).
* onepix_128_lognormal (63 one-k_f shells): every closed triplet and P.
* toy600_xhi099, toy600_xhi088 (the ionised-sphere boxes of Section 3.3,
  600^3 cells of 1 Mpc, 61 shells of 2 k_f): every equilateral and the
  k_2 = 2 k_1 families of Fig. xH_bi (k_1 shells centred on 20, 30, 48 k_f,
  k_2 on 40, 60, 96 k_f, every closed third shell), P of every shell, and the
  Bharadwaj-Pandey theory averaged over the same configurations (the window
  moments of oracle/toymodel.py) with the sphere statistics of the map.
* onepix_256_lognormal (127 one-k_f shells): a stratified sample over all
  bins -- every equilateral, one seeded triplet per bin, the flattened
  triplets k = i + j + 1 (in k_f) with k >= 125, 32 more seeded triplets --
  and P of every shell.
* c4_512_lognormal (32 bins): a stratified sample that touches every bin --
  every equilateral (b,b,b), one seeded triplet per bin, the triangle-edge
  triplets k = i + j + 1 with k >= 29 (the worst-conditioned ones), 16 more
  seeded triplets -- and the quads (b,b,b,b) plus 32 seeded (a,a,b,b).

Usage: python tests/golden/make_fftref_goldens.py [workload ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import fftref, toymodel  # noqa: E402
from paper_1705_06284_amd import synth  # noqa: E402

WORKLOADS = ("c2_128_lognormal", "c3_256_bubbles", "onepix_128_lognormal", "c4_512_lognormal",
             "onepix_256_lognormal", "toy600_xhi099", "toy600_xhi088")


def onepix_sample(nb, cand, seed=8):
    """Unit shells centred on k = b + 1: equilaterals, one seeded triplet per
    bin, the flattened triplets k3 = k1 + k2 + 1 with k3 >= 125, 32 more."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cs = {tuple(int(x) for x in t) for t in cand}
    pick = [(b, b, b) for b in range(nb) if (b, b, b) in cs]
    by_bin = {b: [] for b in range(nb)}
    for t in sorted(cs):
        for b in set(t):
            by_bin[b].append(t)
    for b in range(nb):
        pick.append(by_bin[b][int(rng.integers(len(by_bin[b])))])
    for k in (124, 125, 126):               # bin k is k_f = k + 1
        for i in range(k):
            j = k - 2 - i                   # (i + 1) + (j + 1) + 1 = k + 1
            if i <= j and (i, j, k) in cs:
                pick.append((i, j, k))
    allc = sorted(cs)
    for _ in range(32):
        pick.append(allc[int(rng.integers(len(allc)))])
    out = []
    seen = set()
    for t in pick:
        if t not in seen:
            seen.add(t)
            out.append(t)
    return np.array(out, np.int32)


def toy_configurations(nb):
    """Equilaterals, then (b1, b2, b3) for b1, b2 = (9, 19), (14, 29), (23, 47)
    and every third shell b3 in [b2 - b1 - 1, b2 + b1 + 1] inside the bins,
    each tuple sorted (the triangle test drops the open ones)."""
    out = [(b, b, b) for b in range(nb)]
    for b1, b2 in ((9, 19), (14, 29), (23, 47)):
        for b3 in range(max(0, b2 - b1 - 1), min(nb, b2 + b1 + 2)):
            t = tuple(sorted((b1, b2, b3)))
            if t not in out:
                out.append(t)
    return np.array(out, np.int32)


def make_toy(wl, cache_bytes):
    w = synth.WORKLOADS[wl]
    n, L, rad = w["n"], w["box_len"], w["radius"]
    lo, hi = synth.workload_bins(wl)
    nb = len(lo)
    t0 = time.time()
    d, st = synth.toy_bubbles(n, rad, w["target"], w["seed"], max_tries=w["max_tries"], return_stats=True)
    assert np.array_equal(d, synth.workload_field(wl))
    dig = fftref.field_digest(d)
    cand = {tuple(int(x) for x in t) for t in oracle.candidate_triplets(lo, hi)}
    trip = np.array([t for t in toy_configurations(nb) if tuple(int(x) for x in t) in cand], np.int32)
    print("%s: %d triplets, %d spheres, x_ion %.6f" % (wl, len(trip), st["spheres"], st["ionized_fraction"]),
          flush=True)
    R = fftref.FFTReference(d, lo, hi, box_len=L, cache_bytes=cache_bytes)
    fb = R.bispectrum(trip)
    keep = fb.count > 0
    print("  B done (%.0f s), %d closed" % (time.time() - t0, int(keep.sum())), flush=True)
    assert R.max_imag < 1e-10, R.max_imag
    trip = trip[keep]
    kappa = R.condition(trip, fb.count[keep])
    del R
    p, m = oracle.power_spectrum(d, lo, hi, box_len=L)
    print("  P done (%.0f s)" % (time.time() - t0), flush=True)
    # the bin-averaged window moments depend on the grid, bins, radius and
    # triplets only: taken from another toy box with the same ones if stored
    w2 = www = None
    for other in WORKLOADS:
        path_o = os.path.join(HERE, "%s.fftref.npz" % other)
        if other == wl or not other.startswith("toy") or not os.path.exists(path_o):
            continue
        zo = np.load(path_o)
        if (int(zo["n"]) == n and float(zo["box_len"]) == L and float(zo["radius"]) == rad
                and np.array_equal(zo["k_lo"], lo) and np.array_equal(zo["k_hi"], hi)
                and np.array_equal(zo["triplets"], trip) and np.array_equal(zo["B_count"], fb.count[keep])):
            w2, www = zo["W2_bin"], zo["WWW_bin"]
            print("  window moments from %s" % other, flush=True)
            break
    if w2 is None:
        w2, www, _ = toymodel.binned_window_moments((n, n, n), lo, hi, L, rad, trip, cache_bytes=cache_bytes,
                                                    counts=fb.count[keep])
    out = dict(triplets=trip, B=fb.value[keep], B_noise=fb.noise[keep], B_count=fb.count[keep].astype(np.int64),
               B_count_frac=fb.count_frac[keep], kappa=kappa, P=p, M=m, k_lo=lo, k_hi=hi, n=np.int64(n),
               box_len=np.float64(L), radius=np.float64(rad), spheres=np.int64(st["spheres"]),
               ionized_fraction=np.float64(st["ionized_fraction"]), W2_bin=w2, WWW_bin=www,
               quads=np.zeros((0, 4), np.int32), T=np.zeros(0), T_noise=np.zeros(0),
               T_count=np.zeros(0, np.int64), T_count_frac=np.zeros(0),
               digest_moments=np.array([dig["size"], dig["sum"], dig["sum2"], dig["sum3"]], np.float64),
               digest_sample=np.array(dig["sample"], np.float64))
    fr, ct = out["B_count_frac"], np.maximum(out["B_count"], 1)
    assert np.all((fr < 0.01) | (fr < 1e-13 * ct)), np.max(fr)
    path = os.path.join(HERE, "%s.fftref.npz" % wl)
    np.savez_compressed(path, **out)
    print("  wrote %s (%.0f s; max count distance %.1e, max kappa %.2f)"
          % (path, time.time() - t0, out["B_count_frac"].max(), out["kappa"].max()), flush=True)


def c4_sample(nb, cand, seed=4):
    rng = np.random.Generator(np.random.PCG64(seed))
    cs = {tuple(int(x) for x in t) for t in cand}
    pick = []
    for b in range(nb):
        if (b, b, b) in cs:
            pick.append((b, b, b))
    for b in range(nb):
        mem = sorted(t for t in cs if b in t)
        pick.append(mem[int(rng.integers(len(mem)))])
    for k in (29, 30, 31):
        for i in range(0, k):
            j = k - 1 - i
            if i <= j and (i, j, k) in cs:
                pick.append((i, j, k))
    allc = sorted(cs)
    for _ in range(16):
        pick.append(allc[int(rng.integers(len(allc)))])
    out = []
    for t in pick:
        if t not in out:
            out.append(t)
    quads = [(b, b, b, b) for b in range(nb)]
    while len(quads) < nb + 32:
        a, b = sorted(int(x) for x in rng.integers(nb, size=2))
        if a != b and (a, a, b, b) not in quads:
            quads.append((a, a, b, b))
    return np.array(out, np.int32), np.array(quads, np.int32)


def make(wl, cache_bytes):
    n = synth.WORKLOADS[wl]["n"]
    lo, hi = synth.workload_bins(wl)
    nb = len(lo)
    t0 = time.time()
    d = synth.workload_field(wl)
    dig = fftref.field_digest(d)
    R = fftref.FFTReference(d, lo, hi, cache_bytes=cache_bytes)
    cand = oracle.candidate_triplets(lo, hi)
    if wl == "c4_512_lognormal":
        trip, quads = c4_sample(nb, cand)
    elif wl == "onepix_256_lognormal":
        trip, quads = onepix_sample(nb, cand), np.zeros((0, 4), np.int32)
    else:
        trip = cand
        quads = oracle.collapsed_quads(nb) if not wl.startswith("onepix") else np.zeros((0, 4), np.int32)
    print("%s: %d triplets, %d quads" % (wl, len(trip), len(quads)), flush=True)
    fb = R.bispectrum(trip)
    keep = fb.count > 0
    print("  B done (%.0f s), %d closed" % (time.time() - t0, int(keep.sum())), flush=True)
    p, m = R.power_spectrum()
    out = dict(triplets=trip[keep], B=fb.value[keep], B_noise=fb.noise[keep], B_count=fb.count[keep].astype(np.int64),
               B_count_frac=fb.count_frac[keep], kappa=R.condition(trip[keep], fb.count[keep]),
               P=p, M=m, k_lo=lo, k_hi=hi, n=np.int64(n),
               digest_moments=np.array([dig["size"], dig["sum"], dig["sum2"], dig["sum3"]], np.float64),
               digest_sample=np.array(dig["sample"], np.float64))
    if len(quads):
        ft = R.trispectrum(quads)
        out.update(quads=quads, T=ft.value, T_noise=ft.noise, T_count=ft.count, T_count_frac=ft.count_frac)
    else:
        out.update(quads=quads, T=np.zeros(0), T_noise=np.zeros(0), T_count=np.zeros(0, np.int64),
                   T_count_frac=np.zeros(0))
    assert R.max_imag < 1e-10, R.max_imag
    # triangle counts resolve to single units up to 256^3; at 512^3 the FP64
    # rounding of the count fields moves sum I I I / N_pix by a few 1e-2 for
    # counts near 1e12 (2e-14 relative), so they are held to a relative 1e-13
    # there; p = 4 counts outgrow the unit resolution of N_pix N_q and are held
    # to a relative 1e-9
    fr, ct = out["B_count_frac"], np.maximum(out["B_count"], 1)
    assert np.all((fr < 0.01) | (fr < 1e-13 * ct)), np.max(fr)
    assert not len(quads) or np.max(out["T_count_frac"] / np.maximum(out["T_count"], 1)) < 1e-9
    path = os.path.join(HERE, "%s.fftref.npz" % wl)
    np.savez_compressed(path, **out)
    print("  wrote %s (%.0f s; max count distance %.1e, max kappa %.2f)"
          % (path, time.time() - t0, out["B_count_frac"].max(), out["kappa"].max()), flush=True)


def remake_quads(wl, cache_bytes):
    """Recompute the p = 4 part of a stored workload (FP64 counts) in place."""
    z = dict(np.load(os.path.join(HERE, "%s.fftref.npz" % wl)))
    lo, hi = synth.workload_bins(wl)
    d = synth.workload_field(wl)
    R = fftref.FFTReference(d, lo, hi, cache_bytes=cache_bytes)
    ft = R.trispectrum(z["quads"])
    z.update(T=ft.value, T_noise=ft.noise, T_count=ft.count, T_count_frac=ft.count_frac)
    assert np.max(z["T_count_frac"] / np.maximum(z["T_count"], 1)) < 1e-9
    np.savez_compressed(os.path.join(HERE, "%s.fftref.npz" % wl), **z)
    print("  rewrote the quads of", wl, flush=True)


def load(wl):
    """The stored values of a workload and a check of the map they belong to."""
    z = np.load(os.path.join(HERE, "%s.fftref.npz" % wl))
    dm = z["digest_moments"]
    dig = {"size": int(dm[0]), "sum": dm[1], "sum2": dm[2], "sum3": dm[3], "sample": list(z["digest_sample"])}
    return z, dig


if __name__ == "__main__":
    if sys.argv[1:2] == ["--quads"]:
        for wl in sys.argv[2:]:
            remake_quads(wl, cache_bytes=(34 << 30) if wl.startswith("c4") else (16 << 30))
        sys.exit(0)
    todo = sys.argv[1:] or list(WORKLOADS)
    for wl in todo:
        if wl.startswith("toy"):
            make_toy(wl, cache_bytes=16 << 30)
        else:
            make(wl, cache_bytes=(34 << 30) if wl.startswith("c4") else (8 << 30))
