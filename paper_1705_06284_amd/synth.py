"""Seeded synthetic input fields (numpy, FP64 generation, FP32 output).

This module holds none of the estimator's arithmetic: it only draws the
fields that both the GPU path and the CPU oracle are fed.  The recipes follow
the workloads the paper measures on (Watkinson et al. 2017, Sections 3.2 and
3.3) with synthetic stand-ins:

* ``gaussian_field``   -- Gaussian random field with power P(m) = |m|^-n on
  every non-DC mode, rescaled to an exact sample variance sigma^2.
* ``lognormal_field``  -- delta = exp(g - sigma^2/2) - 1 (stand-in for the
  weakly non-Gaussian evolved density field of Section 3.2).
* ``local_quadratic_field`` -- delta = g + f (g^2 - <g^2>), whose tree-level
  bispectrum has a closed form.
* ``toy_bubbles``      -- the randomly placed ionised-sphere toy model of
  Section 3.3 (x_HI = 1 outside spheres, 0 inside), mean subtracted.
"""
from __future__ import annotations

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _kgrid2(n):
    f = np.fft.fftfreq(n, d=1.0 / n)
    fr = np.fft.rfftfreq(n, d=1.0 / n)
    return (f[:, None, None] ** 2 + f[None, :, None] ** 2 + fr[None, None, :] ** 2)


def gaussian_field(n: int, spectral_index: float, sigma: float, seed: int) -> np.ndarray:
    """FP64 Gaussian field with P(m) proportional to |m|^-spectral_index, variance sigma^2."""
    rng = _rng(seed)
    white = rng.standard_normal((n, n, n))
    wk = np.fft.rfftn(white)
    k2 = _kgrid2(n)
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = k2[nz] ** (-spectral_index / 4.0)   # sqrt(|m|^-n)
    g = np.fft.irfftn(wk * amp, s=(n, n, n), axes=(0, 1, 2))
    g -= g.mean()
    g *= sigma / np.sqrt(np.mean(g * g))
    return g


def lognormal_field(n: int, spectral_index: float, sigma: float, seed: int) -> np.ndarray:
    """FP32 lognormal field delta = exp(g - sigma^2/2) - 1."""
    g = gaussian_field(n, spectral_index, sigma, seed)
    return (np.exp(g - 0.5 * sigma * sigma) - 1.0).astype(np.float32)


def lognormal_field_device(n: int, spectral_index: float, sigma: float, seed: int, device="cuda"):
    """The lognormal recipe of ``lognormal_field`` drawn on a GPU with torch
    (its own seeded generator and FFTs, FP64), for request streams that need
    a fresh map per request: an FP32 [N, N, N] device tensor.  Not bit-equal
    to ``lognormal_field`` for the same seed."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    white = torch.randn((n, n, n), generator=g, dtype=torch.float64, device=device)
    wk = torch.fft.rfftn(white)
    f = torch.fft.fftfreq(n, d=1.0 / n, device=device, dtype=torch.float64)
    fr = torch.fft.rfftfreq(n, d=1.0 / n, device=device, dtype=torch.float64)
    k2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + fr[None, None, :] ** 2
    amp = torch.where(k2 > 0, k2.clamp_min(1.0) ** (-spectral_index / 4.0), torch.zeros_like(k2))
    gf = torch.fft.irfftn(wk * amp, s=(n, n, n))
    gf = gf - gf.mean()
    gf = gf * (sigma / torch.sqrt(torch.mean(gf * gf)))
    return (torch.exp(gf - 0.5 * sigma * sigma) - 1.0).to(torch.float32)


def local_quadratic_field(n: int, spectral_index: float, sigma_g: float, f_nl: float,
                          seed: int, dtype=np.float32) -> np.ndarray:
    """delta = g + f (g^2 - <g^2>) with <g^2> the realisation mean."""
    g = gaussian_field(n, spectral_index, sigma_g, seed)
    g2 = g * g
    return (g + f_nl * (g2 - g2.mean())).astype(dtype)


def _ball_offsets(radius: float) -> np.ndarray:
    r = int(np.floor(radius))
    a = np.arange(-r, r + 1)
    dz, dy, dx = np.meshgrid(a, a, a, indexing="ij")
    sel = dz * dz + dy * dy + dx * dx <= radius * radius
    return np.stack([dz[sel], dy[sel], dx[sel]], axis=1)


def toy_bubbles(n: int, radius: float, ionized_target: float, seed: int,
                max_tries: int = 1000, return_stats: bool = False):
    """Randomly placed ionised spheres of one radius (Section 3.3 toy model).

    Each sphere first tries up to ``max_tries`` uniform lattice centres for a
    spot whose periodic distance to every earlier centre is >= 2 R (no
    overlap); if none is free it takes an overlapping one (``max_tries = 0``:
    every centre uniform, overlap allowed).  Spheres are the
    lattice cells within periodic distance R of the centre.  Placement stops
    once the ionised cell fraction reaches ``ionized_target``.  Returns the
    mean-subtracted FP32 x_HI field (and placement statistics on request).
    """
    rng = _rng(seed)
    ion = np.zeros((n, n, n), dtype=bool)
    blocked = np.zeros((n, n, n), dtype=bool)      # centres closer than 2R to a sphere
    sphere = _ball_offsets(radius)
    excl = _ball_offsets(np.nextafter(2.0 * radius, 0.0))  # distance < 2R
    target = int(np.ceil(ionized_target * n ** 3))
    n_ion = 0
    placed = overlapping = 0
    batch = 64
    while n_ion < target:
        centre = None
        tries = 0
        while tries < max_tries:
            c = rng.integers(0, n, size=(batch, 3))
            ok = ~blocked[c[:, 0], c[:, 1], c[:, 2]]
            take = min(batch, max_tries - tries)
            hit = np.flatnonzero(ok[:take])
            if hit.size:
                centre = c[hit[0]]
                tries += hit[0] + 1
                break
            tries += take
        if centre is None:
            centre = rng.integers(0, n, size=3)
            overlapping += 1
        cells = (centre[None, :] + sphere) % n
        newly = ~ion[cells[:, 0], cells[:, 1], cells[:, 2]]
        n_ion += int(newly.sum())
        ion[cells[:, 0], cells[:, 1], cells[:, 2]] = True
        ex = (centre[None, :] + excl) % n
        blocked[ex[:, 0], ex[:, 1], ex[:, 2]] = True
        placed += 1
    x_hi = (~ion).astype(np.float64)
    out = (x_hi - x_hi.mean()).astype(np.float32)
    if return_stats:
        return out, {"spheres": placed, "overlapping": overlapping,
                     "ionized_fraction": n_ion / n ** 3}
    return out


# ----------------------------------------------------------------------------
# Bin layouts of the standard workloads
# ----------------------------------------------------------------------------

def linear_bins(n: int, n_bins: int):
    """n_bins linear bins from 0 to the Nyquist mode: edges b (N/2) / n_bins."""
    e = np.arange(n_bins + 1, dtype=np.float64) * (n / 2.0) / n_bins
    return e[:-1].copy(), e[1:].copy()


def unit_bins(first: int, last: int):
    """Bins of width k_f centred on the integers first..last: [b - 1/2, b + 1/2)."""
    c = np.arange(first, last + 1, dtype=np.float64)
    return c - 0.5, c + 0.5


WORKLOADS = {
    # name: (N, field recipe, bins)
    "c1_32_localquad": dict(n=32, kind="local_quadratic", spectral_index=2.0, sigma=0.1,
                            f_nl=0.5, seed=1, bins=("unit", 1, 8)),
    "c2_128_lognormal": dict(n=128, kind="lognormal", spectral_index=1.5, sigma=1.0,
                             seed=2, bins=("linear", 16)),
    "c3_256_bubbles": dict(n=256, kind="bubbles", radius=8.0, target=0.5, seed=3,
                           bins=("linear", 24)),
    "c4_512_lognormal": dict(n=512, kind="lognormal", spectral_index=1.0, sigma=1.5,
                             seed=4, bins=("linear", 32)),
    # one-pixel shells for configuration binning: every shell below the
    # Nyquist mode at 128^3 (63) and at 256^3 (127)
    "onepix_128_lognormal": dict(n=128, kind="lognormal", spectral_index=1.5, sigma=1.0,
                                 seed=2, bins=("unit", 1, 63)),
    "onepix_256_lognormal": dict(n=256, kind="lognormal", spectral_index=1.5, sigma=1.0,
                                 seed=8, bins=("unit", 1, 127)),
    # the toy reionisation boxes of Section 3.3: 600^3 cells of 1 Mpc, spheres
    # of radius 10 Mpc at uniform random centres (overlap allowed, as in the
    # paper's boxes), neutral fractions 0.99 and 0.88; 61 shells of 2 k_f
    "toy600_xhi099": dict(n=600, kind="bubbles", radius=10.0, target=0.01, seed=6, bins=("width", 1.0, 2.0, 61),
                          box_len=600.0, max_tries=0),
    "toy600_xhi088": dict(n=600, kind="bubbles", radius=10.0, target=0.12, seed=7, bins=("width", 1.0, 2.0, 61),
                          box_len=600.0, max_tries=0),
}


def workload_bins(name: str):
    w = WORKLOADS[name]
    b = w["bins"]
    if b[0] == "unit":
        return unit_bins(b[1], b[2])
    if b[0] == "width":               # nb bins of width w from lo: [lo + i w, lo + (i + 1) w)
        e = b[1] + b[2] * np.arange(b[3] + 1, dtype=np.float64)
        return e[:-1].copy(), e[1:].copy()
    return linear_bins(w["n"], b[1])


def workload_field(name: str, seed=None) -> np.ndarray:
    w = WORKLOADS[name]
    s = w["seed"] if seed is None else seed
    if w["kind"] == "local_quadratic":
        return local_quadratic_field(w["n"], w["spectral_index"], w["sigma"], w["f_nl"], s)
    if w["kind"] == "lognormal":
        return lognormal_field(w["n"], w["spectral_index"], w["sigma"], s)
    if w["kind"] == "bubbles":
        return toy_bubbles(w["n"], w["radius"], w["target"], s, max_tries=w.get("max_tries", 1000))
    raise KeyError(name)
