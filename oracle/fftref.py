"""FP64 FFT form of the polyspectrum estimator (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the HIP path.

This is the paper's own method (Watkinson et al. 2017, arXiv:1705.06284,
Section 2) written out plainly in FP64 with a library FFT, in the paper's
order of steps:

1. Promote the FP32 input exactly to FP64 and subtract the FP64 mean; take
   the unnormalised forward transform Delta(m) = sum_n delta(n)
   exp(-2 pi i m.n / N) (Eq. DeltaFFTtoDelta).
2. For each bin b, fill a fresh box with Delta on the shell S_b and zero
   elsewhere, and take its unnormalised inverse transform: the bin field
   F_b(n) (Eq. delta_nr, first line).  The same box filled with ones gives
   the count field I_b(n) (Eq. delta_nr, second line).
3. For a configuration of p bins, sum_n prod F over the grid divided by
   sum_n prod I, times H^p / V with H = V / N_pix (Eq. Jeong_gen; p = 2 is
   Eq. Jeong_PS, p = 3 is Eq. Jeong_BI).

The shells are the same as the direct-sum oracle's (``polyspec``): mode m
(signed integer components in [-N/2, N/2)) is in bin b iff
lo_b^2 <= |m|^2 < hi_b^2 and m != 0, with the squared edges formed in FP64;
on a non-cubic grid of cubic cells |m|^2 is the integer q of ``polyspec``.

For the parity bar the module also forms the random-phase noise level of
each estimate, norm * sqrt(sum over closed tuples of prod |Delta|^2) / count.
By the phase-sum identity before Eq. gen_Nspec4 that closed-tuple sum is
sum_n prod Q_b / N_pix, where Q_b is the inverse transform of the shell box
filled with |Delta|^2 (a real, even spectrum, so Q_b is real).

Every grid sum is numpy's pairwise FP64 summation of the pointwise product.
There is no pruning, no pairing of bins into one transform, no reuse of one
configuration's sums for another and no matrix reformulation: each
configuration's sums are formed from its own fields.
"""
from __future__ import annotations

import os
from collections import OrderedDict
from dataclasses import dataclass

import numpy as np

try:
    import scipy.fft as _fft
    _HAS_SCIPY = True
except ImportError:                         # pragma: no cover - scipy is in the image
    _fft = np.fft
    _HAS_SCIPY = False

from . import polyspec


def _workers():
    w = os.environ.get("OMP_NUM_THREADS")
    return int(w) if w else (os.cpu_count() or 1)


def _fftn(a):
    return _fft.fftn(a, workers=_workers()) if _HAS_SCIPY else _fft.fftn(a)


def _ifftn(a):
    return _fft.ifftn(a, workers=_workers()) if _HAS_SCIPY else _fft.ifftn(a)


@dataclass
class FFTSpectrum:
    """Estimates of one configuration list from the FFT form."""
    value: np.ndarray        # B, T or P in the paper's normalisation
    s: np.ndarray            # closed-tuple sum of prod Delta: sum_n prod F / N_pix
    count: np.ndarray        # closed tuples (ordered, closure modulo N), rounded, FP64
                             # (p = 4 counts pass 2^63 on large grids)
    count_frac: np.ndarray   # |sum_n prod I / N_pix - count|: distance to an integer
    noise: np.ndarray        # norm * sqrt(sum_closed prod |Delta|^2) / count


class FFTReference:
    """Bin fields of one map in FP64 and the sums of Eq. (Jeong_gen).

    Fields are computed on demand and kept in a least-recently-used cache of
    at most ``cache_bytes`` bytes (at 512^3 one FP64 field is 1 GiB).
    """

    def __init__(self, delta, k_lo, k_hi, box_len=None, cache_bytes=16 << 30):
        d = polyspec.prepare(delta)
        self._setup(d.shape, k_lo, k_hi, box_len, cache_bytes, _fftn(d))     # step 1

    @classmethod
    def from_spectrum(cls, delta_k, k_lo, k_hi, box_len=None, cache_bytes=16 << 30):
        """The same sums for a given full complex spectrum on the grid
        (Hermitian: real fields), e.g. a model spectrum whose averages over
        the closed tuples of each configuration are wanted."""
        self = cls.__new__(cls)
        self._setup(delta_k.shape, k_lo, k_hi, box_len, cache_bytes, np.asarray(delta_k, np.complex128))
        return self

    def _setup(self, shape, k_lo, k_hi, box_len, cache_bytes, delta_k):
        self.shape = shape
        self.npix = float(np.prod(shape))
        self.volume = polyspec._volume(shape, box_len)
        self.lo2, self.hi2 = polyspec.squared_edges(k_lo, k_hi, shape)
        self.n_bins = len(self.lo2)
        self.delta_k = delta_k
        sc = polyspec.q_scales(shape)
        fz, fy, fx = (sc[a] * polyspec.freq(shape[a]).astype(np.int64) for a in range(3))
        self.r2 = fz[:, None, None] ** 2 + fy[None, :, None] ** 2 + fx[None, None, :] ** 2
        self._cache = OrderedDict()
        self._cache_bytes = int(cache_bytes)
        self.max_imag = 0.0                                  # largest |Im| / max |Re| seen

    # -- step 2 ---------------------------------------------------------------
    def shell(self, b):
        """Boolean mask of S_b on the full grid (m != 0)."""
        r2 = self.r2.astype(np.float64)
        return (self.r2 > 0) & (r2 >= self.lo2[b]) & (r2 < self.hi2[b])

    def _make(self, kind, b):
        m = self.shell(b)
        if kind == "F":
            box = np.where(m, self.delta_k, 0.0)
        elif kind == "I":
            box = m.astype(np.complex128)
        elif kind == "Q":
            box = np.where(m, np.abs(self.delta_k) ** 2, 0.0).astype(np.complex128)
        else:
            raise KeyError(kind)
        full = _ifftn(box) * self.npix                       # unnormalised inverse
        re = np.ascontiguousarray(full.real)
        scale = float(np.max(np.abs(re))) or 1.0
        self.max_imag = max(self.max_imag, float(np.max(np.abs(full.imag))) / scale)
        return re

    def field(self, kind, b):
        key = (kind, int(b))
        if key in self._cache:
            self._cache.move_to_end(key)
            return self._cache[key]
        v = self._make(kind, b)
        self._cache[key] = v
        while len(self._cache) > 1 and sum(a.nbytes for a in self._cache.values()) > self._cache_bytes:
            self._cache.popitem(last=False)
        return v

    # -- step 3 ---------------------------------------------------------------
    def grid_sum(self, kind, bins):
        """sum_n prod_{b in bins} field(kind, b)(n), pairwise FP64 summation."""
        bins = [int(b) for b in bins]
        prod = self.field(kind, bins[0]) * self.field(kind, bins[1])
        for b in bins[2:]:
            prod *= self.field(kind, b)
        return float(np.sum(prod))

    def _spectrum(self, tuples, order, norm):
        tuples = np.asarray(tuples, dtype=np.int64).reshape(-1, order)
        out = {}
        # one kind of field at a time, the tuples in bin order, so that the
        # field cache holds the few fields the next tuples reuse
        order_t = sorted(range(len(tuples)), key=lambda t: tuple(sorted(tuples[t])))
        for key, kind in (("S", "F"), ("C", "I"), ("Q", "Q")):
            out[key] = np.zeros(len(tuples))
            for t in order_t:
                out[key][t] = self.grid_sum(kind, tuples[t]) / self.npix
        cnt = np.rint(out["C"])
        with np.errstate(invalid="ignore", divide="ignore"):
            val = norm * out["S"] / cnt
            noise = norm * np.sqrt(np.maximum(out["Q"], 0.0)) / cnt
        return FFTSpectrum(value=val, s=out["S"], count=cnt, count_frac=np.abs(out["C"] - cnt), noise=noise)

    def bispectrum(self, triplets):
        """Eq. (Jeong_BI): B = V^2 / N_pix^3 sum F F F / sum I I I."""
        return self._spectrum(triplets, 3, self.volume ** 2 / self.npix ** 3)

    def trispectrum(self, quads):
        """Eq. (Jeong_gen) with p = 4: T = V^3 / N_pix^4 sum F F F F / sum I I I I."""
        return self._spectrum(quads, 4, self.volume ** 3 / self.npix ** 4)

    def power_spectrum(self):
        """Eq. (Jeong_PS): P_b = V / N_pix^2 sum F_b^2 / sum I_b^2, and M_b."""
        p = np.zeros(self.n_bins)
        m = np.zeros(self.n_bins, dtype=np.int64)
        for b in range(self.n_bins):
            c = self.grid_sum("I", (b, b)) / self.npix
            m[b] = int(np.rint(c))
            p[b] = self.volume / self.npix ** 2 * self.grid_sum("F", (b, b)) / self.grid_sum("I", (b, b))
        return p, m

    def condition(self, triplets, counts):
        """kappa_t = sqrt(M_i M_j M_k / (N_pix N_t)) from the shell sizes and counts."""
        t = np.asarray(triplets, dtype=np.int64).reshape(-1, 3)
        m = np.array([int(self.shell(b).sum()) for b in range(self.n_bins)], dtype=np.float64)
        with np.errstate(divide="ignore"):
            return np.sqrt(m[t[:, 0]] * m[t[:, 1]] * m[t[:, 2]] / (self.npix * np.asarray(counts, float)))


def field_digest(delta, n_sample=4096):
    """A digest of an FP32 map that does not change when a few entries move by
    one unit in the last place (generators that call exp may round
    differently on different CPUs): FP64 moments and a strided sample."""
    d = np.asarray(delta, dtype=np.float64).ravel()
    step = max(1, d.size // n_sample)
    return {"size": int(d.size), "sum": float(np.sum(d)), "sum2": float(np.sum(d * d)),
            "sum3": float(np.sum(d * d * d)), "sample": [float(x) for x in d[::step][:n_sample]]}


def digest_matches(a, b, rtol=1e-9):
    """Two digests agree up to single-ulp differences of a few entries."""
    if a["size"] != b["size"] or len(a["sample"]) != len(b["sample"]):
        return False
    sa, sb = np.asarray(a["sample"]), np.asarray(b["sample"])
    amax = float(np.max(np.abs(sa))) or 1.0
    if np.mean(sa != sb) > 0.01 or np.max(np.abs(sa - sb)) > 1e-6 * amax:
        return False
    l2 = float(np.sqrt(a["sum2"] * a["size"]))        # scale of a sum of `size` terms
    return bool(abs(a["sum"] - b["sum"]) <= rtol * l2
                and abs(a["sum2"] - b["sum2"]) <= rtol * a["sum2"]
                and abs(a["sum3"] - b["sum3"]) <= rtol * (abs(a["sum3"]) + amax * a["sum2"]))
