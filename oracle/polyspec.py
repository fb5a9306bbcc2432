"""FP64 direct-sum oracle of the FFT polyspectrum estimator (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the HIP path.

What it computes (Watkinson et al. 2017, arXiv:1705.06284, Section 2):

* Delta_fft(m) = sum_n delta(n) exp(-2 pi i m.n / N), the unnormalised forward
  DFT of Eq. (DeltaFFTtoDelta), evaluated as three matrix products with the
  DFT matrix (twiddle angle from the exactly reduced integer (m n) mod N).
* Shells: bin b holds the modes with lo_b^2 <= |m|^2 < hi_b^2, m != 0, every
  component in [-N/2, N/2) (the spherical-shell reading of the bin rule of
  Eq. gen_Nspec3; Nyquist modes never qualify because hi_b <= N/2,
  Eq. nyqvist).  Non-cubic grids N_z x N_y x N_x (footnote to the pixel
  coordinates, Section 2: one fundamental per axis) have cubic cells, so
  L_i = L_x N_i / N_x; with P the lcm of the sides and s_i = P / N_i,
  q = sum_i (s_i m_i)^2 is |k|^2 in units of (2 pi / (P cells))^2 and the
  shells, with edges in units of the x-axis fundamental 2 pi / L_x, are
  (lo_b s_x)^2 <= q < (hi_b s_x)^2.  On a cubic grid q = |m|^2.
* The bispectrum of Eq. (Jeong_BI) equals the direct sum over ordered closed
  triples (Kronecker delta taken modulo N, the phase-sum identity before
  Eq. gen_Nspec4):

      S_t = sum_{m1 in S_i, m2 in S_j, m3 in S_k, m1+m2+m3 = 0 mod N} D1 D2 D3
      N_t = the same sum with every amplitude set to 1
      B_t = (V^2 / N_pix^3) Re S_t / N_t

* Power spectrum (Eq. Jeong_PS; by Parseval the shell average of |Delta|^2):
      P_b = (V / N_pix^2) sum_{m in S_b} |Delta(m)|^2 / M_b
* p = 4 (Eq. Jeong_gen with four fields):
      T_q = (V^3 / N_pix^4) Re S_q / N_q

The closed-triplet loops run in ``direct.c``; everything else is numpy.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct.c")
_LIB = os.path.join(_HERE, "_direct.so")
_NACC = 7
_lib = None


def build(force: bool = True) -> str:
    """Compile ``direct.c`` into ``_direct.so`` with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        up = ctypes.POINTER(ctypes.c_uint64)
        six = [ctypes.c_int] * 6
        lib.orc_pair_sums.argtypes = six + [dp, dp, ctypes.c_int, ip, ctypes.c_int, ip,
                                            up, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, dp]
        lib.orc_pair_sums.restype = ctypes.c_int
        lib.orc_triple_sums.argtypes = six + [dp, dp, ctypes.c_int, ip, ctypes.c_int, ip,
                                              ctypes.c_int, ip, up, ctypes.c_int64, ctypes.c_uint64,
                                              ctypes.c_int, dp]
        lib.orc_triple_sums.restype = ctypes.c_int
        lib.orc_triple_sums_diag.argtypes = six + [dp, dp, ctypes.c_int, ip, ctypes.c_int, ip,
                                                   ctypes.c_int, ip, up, ctypes.c_int64, ctypes.c_uint64,
                                                   ctypes.c_double, ctypes.c_double, ctypes.c_int, dp]
        lib.orc_triple_sums_diag.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a, ctype):
    if a is None:
        return ctypes.POINTER(ctype)()
    return a.ctypes.data_as(ctypes.POINTER(ctype))


# ----------------------------------------------------------------------------
# Bins and shells (Eq. gen_Nspec3 with the spherical-shell reading)
# ----------------------------------------------------------------------------

def grid_shape(n):
    """(N_z, N_y, N_x) of a grid given by its side N (cubic) or its shape."""
    if np.ndim(n) == 0:
        return (int(n),) * 3
    t = tuple(int(x) for x in n)
    assert len(t) == 3
    return t


def q_scales(n):
    """(s_z, s_y, s_x) = P / N_i with P the lcm of the sides (1, 1, 1 on a cube)."""
    nz, ny, nx = grid_shape(n)
    P = int(np.lcm.reduce([nz, ny, nx]))
    return P // nz, P // ny, P // nx


def squared_edges(k_lo, k_hi, n=None):
    """FP64 squared bin edges in q units: (lo s_x)^2 and (hi s_x)^2, formed as
    (lo * lo) * (s_x * s_x); on a cubic grid lo^2 and hi^2, in units of k_f."""
    lo = np.asarray(k_lo, dtype=np.float64)
    hi = np.asarray(k_hi, dtype=np.float64)
    sx2 = float(q_scales(n)[2] ** 2) if n is not None else 1.0
    return (lo * lo) * sx2, (hi * hi) * sx2


def freq(n: int) -> np.ndarray:
    """Signed integer frequency of each DFT index: 0..ceil(N/2)-1, then
    -floor(N/2)..-1 (for even N: -N/2..N/2-1)."""
    i = np.arange(n)
    return np.where(i < n - n // 2, i, i - n)


def _q_of(mz, my, mx, s):
    return ((s[0] * np.asarray(mz, np.int64)) ** 2 + (s[1] * np.asarray(my, np.int64)) ** 2
            + (s[2] * np.asarray(mx, np.int64)) ** 2)


def bin_mask_table(n, k_lo, k_hi, bins=None) -> np.ndarray:
    """uint64 bit mask per integer q: bit i set iff the modes with that q are
    in bin bins[i] (q = |m|^2 on a cubic grid; bins: at most 64 bin indices,
    default all bins).  q = 0 (the mean) is in no bin."""
    shape, s = grid_shape(n), q_scales(n)
    lo2, hi2 = squared_edges(k_lo, k_hi, n)
    bins = list(range(len(lo2))) if bins is None else list(bins)
    assert len(bins) <= 64
    qmax = int(_q_of(shape[0] // 2, shape[1] // 2, shape[2] // 2, s))
    q = np.arange(qmax + 1, dtype=np.float64)
    mask = np.zeros(qmax + 1, dtype=np.uint64)
    for i, b in enumerate(bins):
        sel = (q >= lo2[b]) & (q < hi2[b])
        sel[0] = False
        mask[sel] |= np.uint64(1) << np.uint64(i)
    return mask


def shell_modes(n, k_lo, k_hi, b: int) -> np.ndarray:
    """All mode vectors (mz, my, mx) of bin b as an int32 array [M_b, 3]."""
    shape, s = grid_shape(n), q_scales(n)
    lo2, hi2 = squared_edges(k_lo, k_hi, n)
    axes = []
    for ax in range(3):
        f = freq(shape[ax])
        h = int(np.ceil(np.sqrt(hi2[b]) / s[ax])) + 1
        axes.append(np.sort(f[np.abs(f) <= h]))
    mz, my, mx = np.meshgrid(*axes, indexing="ij")
    q = _q_of(mz, my, mx, s)
    qf = q.astype(np.float64)
    sel = (q > 0) & (qf >= lo2[b]) & (qf < hi2[b])
    return np.ascontiguousarray(np.stack([mz[sel], my[sel], mx[sel]], axis=1).astype(np.int32))


def mode_counts(n, k_lo, k_hi) -> np.ndarray:
    """M_b: number of modes in each shell."""
    return np.array([len(shell_modes(n, k_lo, k_hi, b)) for b in range(len(k_lo))], dtype=np.int64)


# ----------------------------------------------------------------------------
# Forward DFT (Eq. DeltaFFTtoDelta)
# ----------------------------------------------------------------------------

def dft_matrix(n: int) -> np.ndarray:
    """W[m, j] = exp(-2 pi i ((m j) mod N) / N), the argument reduced exactly."""
    j = np.arange(n, dtype=np.int64)
    red = np.outer(j, j) % n
    ang = (-2.0 * np.pi / n) * red.astype(np.float64)
    return np.cos(ang) + 1j * np.sin(ang)


def dft3(delta: np.ndarray) -> np.ndarray:
    """Unnormalised 3D DFT of a real [z][y][x] grid, as three matrix products."""
    d = np.asarray(delta, dtype=np.float64)
    nz, ny, nx = d.shape
    a = d @ dft_matrix(nx).T                                    # x axis
    a = np.matmul(dft_matrix(ny), a)                            # y axis (batched over z)
    a = (dft_matrix(nz) @ a.reshape(nz, ny * nx)).reshape(nz, ny, nx)  # z axis
    return a


def prepare(delta32) -> np.ndarray:
    """Promote the FP32 input exactly to FP64 and subtract the FP64 mean."""
    d = np.asarray(delta32).astype(np.float64)
    return d - d.mean()


# ----------------------------------------------------------------------------
# Direct sums
# ----------------------------------------------------------------------------

@dataclass
class Spectrum:
    """Per-configuration direct sums and the normalised estimate."""
    value: np.ndarray        # B, T or P in the paper's normalisation
    s: np.ndarray            # complex numerator sum S
    count: np.ndarray        # N_t (or N_q, M_b): ordered closed tuples, mod N
    s_strict: np.ndarray     # numerator restricted to tuples closed in Z^3
    count_strict: np.ndarray
    noise: np.ndarray        # norm * sqrt(sum |product|^2) / count


def _volume(n, box_len):
    """V = L_x L_y L_z with cubic cells: L_i = L_x N_i / N_x (L_x = N_x cells
    when box_len is not given)."""
    nz, ny, nx = grid_shape(n)
    L = float(nx) if (box_len is None or box_len <= 0) else float(box_len)
    return L ** 3 * (nz / nx) * (ny / nx)


def _grid_parts(delta_k):
    if delta_k is None:
        return None, None
    re = np.ascontiguousarray(delta_k.real, dtype=np.float64)
    im = np.ascontiguousarray(delta_k.imag, dtype=np.float64)
    return re, im


def _pair_sums(n, re, im, ma, mb, mask, want_bits, n_bins):
    lib = _load()
    out = np.zeros((n_bins, _NACC), dtype=np.float64)
    rc = lib.orc_pair_sums(*grid_shape(n), *q_scales(n), _ptr(re, ctypes.c_double), _ptr(im, ctypes.c_double),
                           len(ma), _ptr(ma, ctypes.c_int32), len(mb), _ptr(mb, ctypes.c_int32),
                           _ptr(mask, ctypes.c_uint64), len(mask), ctypes.c_uint64(want_bits),
                           n_bins, _ptr(out, ctypes.c_double))
    assert rc == 0, rc
    return out


def _triple_sums(n, re, im, ma, mb, mc, mask, want_bits, n_bins):
    lib = _load()
    out = np.zeros((n_bins, _NACC), dtype=np.float64)
    rc = lib.orc_triple_sums(*grid_shape(n), *q_scales(n), _ptr(re, ctypes.c_double), _ptr(im, ctypes.c_double),
                             len(ma), _ptr(ma, ctypes.c_int32), len(mb), _ptr(mb, ctypes.c_int32),
                             len(mc), _ptr(mc, ctypes.c_int32),
                             _ptr(mask, ctypes.c_uint64), len(mask), ctypes.c_uint64(want_bits),
                             n_bins, _ptr(out, ctypes.c_double))
    assert rc == 0, rc
    return out


def _tuple_sums(n, delta_k, k_lo, k_hi, tuples, order):
    """Direct sums for each tuple of bins (length ``order`` = 3 or 4).

    The sum over ordered slot assignments is symmetric in the slots, so the
    loops run over the (order-1) shells with the fewest modes and the last
    slot is closed by the modulo-N reduction.
    """
    tuples = np.asarray(tuples, dtype=np.int64).reshape(-1, order)
    n_bins = len(k_lo)
    # the bit masks hold 64 bins: beyond that, each group of tuples gets a
    # table of its own closing bins
    full = bin_mask_table(n, k_lo, k_hi) if n_bins <= 64 else None
    modes = {}

    def sh(b):
        if b not in modes:
            modes[b] = shell_modes(n, k_lo, k_hi, b)
        return modes[b]

    counts = np.array([len(sh(b)) for b in range(n_bins)])
    re, im = _grid_parts(delta_k)
    groups = {}
    for t, tup in enumerate(tuples):
        srt = sorted(int(b) for b in tup)
        srt.sort(key=lambda b: (counts[b], b))
        key = tuple(srt[:-1])
        groups.setdefault(key, []).append((t, srt[-1]))
    acc = np.zeros((len(tuples), _NACC))
    for key, items in groups.items():
        lasts = sorted({last for _, last in items})
        for c0 in range(0, len(lasts), 64):
            part = lasts[c0:c0 + 64]
            if full is not None:
                mask, slot, nslot = full, {b: b for b in part}, n_bins
            else:
                mask, slot, nslot = bin_mask_table(n, k_lo, k_hi, part), {b: i for i, b in enumerate(part)}, len(part)
            want = 0
            for b in part:
                want |= 1 << slot[b]
            if order == 3:
                out = _pair_sums(n, re, im, sh(key[0]), sh(key[1]), mask, want, nslot)
            else:
                out = _triple_sums(n, re, im, sh(key[0]), sh(key[1]), sh(key[2]), mask, want, nslot)
            for t, last in items:
                if last in slot:
                    acc[t] = out[slot[last]]
    return acc


def _finish(acc, norm):
    s = acc[:, 0] + 1j * acc[:, 1]
    cnt = acc[:, 2]
    ss = acc[:, 3] + 1j * acc[:, 4]
    cs = acc[:, 5]
    with np.errstate(invalid="ignore", divide="ignore"):
        val = norm * s.real / cnt
        noise = norm * np.sqrt(acc[:, 6]) / cnt
    return Spectrum(value=val, s=s, count=cnt.astype(np.int64), s_strict=ss,
                    count_strict=cs.astype(np.int64), noise=noise)


def bispectrum(delta, k_lo, k_hi, triplets, box_len=None, delta_k=None) -> Spectrum:
    """Direct-sum bispectrum of Eq. (Jeong_BI) for each triplet of bin indices."""
    d = prepare(delta)
    n = d.shape
    if delta_k is None:
        delta_k = dft3(d)
    acc = _tuple_sums(n, delta_k, k_lo, k_hi, triplets, 3)
    vol = _volume(n, box_len)
    npix = float(np.prod(n))
    return _finish(acc, vol ** 2 / npix ** 3)


def trispectrum(delta, k_lo, k_hi, quads, box_len=None, delta_k=None) -> Spectrum:
    """Direct-sum p = 4 polyspectrum of Eq. (Jeong_gen) for each quad of bins."""
    d = prepare(delta)
    n = d.shape
    if delta_k is None:
        delta_k = dft3(d)
    acc = _tuple_sums(n, delta_k, k_lo, k_hi, quads, 4)
    vol = _volume(n, box_len)
    npix = float(np.prod(n))
    return _finish(acc, vol ** 3 / npix ** 4)


def triangle_counts(n, k_lo, k_hi, triplets):
    """N_t: ordered closed triples (mod N) of each triplet, and the strict count."""
    acc = _tuple_sums(n, None, k_lo, k_hi, triplets, 3)
    return acc[:, 2].astype(np.int64), acc[:, 5].astype(np.int64)


def quad_counts(n, k_lo, k_hi, quads):
    acc = _tuple_sums(n, None, k_lo, k_hi, quads, 4)
    return acc[:, 2].astype(np.int64), acc[:, 5].astype(np.int64)


def power_spectrum(delta, k_lo, k_hi, box_len=None, delta_k=None):
    """P_b of Eq. (Jeong_PS) as the shell average of |Delta|^2 (Parseval)."""
    d = prepare(delta)
    n = d.shape
    if delta_k is None:
        delta_k = dft3(d)
    vol = _volume(n, box_len)
    npix = float(np.prod(n))
    out = np.zeros(len(k_lo))
    m = np.zeros(len(k_lo), dtype=np.int64)
    for b in range(len(k_lo)):
        md = shell_modes(n, k_lo, k_hi, b)
        v = delta_k[md[:, 0] % n[0], md[:, 1] % n[1], md[:, 2] % n[2]]
        m[b] = len(md)
        out[b] = vol / npix ** 2 * np.sum(np.abs(v) ** 2) / len(md) if len(md) else np.nan
    return out, m


# ----------------------------------------------------------------------------
# Configuration sets (readings of the paper's silent points)
# ----------------------------------------------------------------------------

def candidate_triplets(k_lo, k_hi):
    """i <= j <= k whose shells admit a strict triangle: each lower edge is
    below the sum of the other two upper edges (necessary for closure in Z^3)."""
    lo = np.asarray(k_lo, dtype=np.float64)
    hi = np.asarray(k_hi, dtype=np.float64)
    nb = len(lo)
    out = []
    for i in range(nb):
        for j in range(i, nb):
            for k in range(j, nb):
                if lo[k] < hi[i] + hi[j] and lo[j] < hi[i] + hi[k] and lo[i] < hi[j] + hi[k]:
                    out.append((i, j, k))
    return np.array(out, dtype=np.int32).reshape(-1, 3)


def closed_triplets(n, k_lo, k_hi):
    """Candidate triplets with a non-zero count N_t (modulo-N closure)."""
    cand = candidate_triplets(k_lo, k_hi)
    cnt, _ = triangle_counts(n, k_lo, k_hi, cand)
    return cand[cnt > 0], cnt[cnt > 0]


def collapsed_quads(n_bins):
    """(a, a, b, b) for a <= b: the collapsed p = 4 configurations."""
    return np.array([(a, a, b, b) for a in range(n_bins) for b in range(a, n_bins)],
                    dtype=np.int32).reshape(-1, 4)


def disconnected_sums(delta, k_lo, k_hi, quads, delta_k=None):
    """S_D per collapsed quad (a, a, b, b): the sum of D(k1) D(k2) D(k3) D(k4)
    over the closed quadruples (k1, k2 in S_a; k3, k4 in S_b) that split into
    two pairs k_i = -k_j (the Gaussian pairings of Wick's theorem), each
    quadruple counted once.  Written out as the union of the three pairing
    sets, enumerated mode by mode and de-duplicated."""
    d = prepare(delta)
    n = d.shape[0]
    if delta_k is None:
        delta_k = dft3(d)
    out = np.zeros(len(quads), dtype=np.complex128)
    for q, quad in enumerate(np.asarray(quads).reshape(-1, 4)):
        a, a2, b, b2 = sorted(int(x) for x in quad)
        if a != a2 or b != b2:
            raise ValueError("only collapsed quads (a, a, b, b)")
        sa = [tuple(int(c) for c in m) for m in shell_modes(n, k_lo, k_hi, a)]
        sb = [tuple(int(c) for c in m) for m in shell_modes(n, k_lo, k_hi, b)]
        in_a, in_b = set(sa), set(sb)
        neg = lambda m: (-m[0], -m[1], -m[2])
        quadset = set()
        for k1 in sa:
            for k3 in sb:
                quadset.add((k1, neg(k1), k3, neg(k3)))           # k2 = -k1, k4 = -k3
        for k1 in sa:
            if neg(k1) not in in_b:
                continue
            for k2 in sa:
                if neg(k2) in in_b:
                    quadset.add((k1, k2, neg(k1), neg(k2)))       # k3 = -k1, k4 = -k2
                    quadset.add((k1, k2, neg(k2), neg(k1)))       # k4 = -k1, k3 = -k2
        amp = lambda m: delta_k[m[0] % n, m[1] % n, m[2] % n]
        out[q] = sum(amp(t[0]) * amp(t[1]) * amp(t[2]) * amp(t[3]) for t in quadset)
    return out


def trispectrum_connected(delta, k_lo, k_hi, quads, box_len=None, delta_k=None):
    """Collapsed T with the Gaussian pairings removed: (V^3 / N_pix^4)
    Re(S_q - S_D) / N_q, S_q the closed-quadruple sum of Eq. Jeong_gen and
    S_D the part of it over paired quadruples (disconnected_sums)."""
    d = prepare(delta)
    n = d.shape[0]
    if delta_k is None:
        delta_k = dft3(d)
    full = trispectrum(d, k_lo, k_hi, quads, box_len=box_len, delta_k=delta_k)
    sd = disconnected_sums(d, k_lo, k_hi, quads, delta_k=delta_k)
    vol = _volume(n, box_len)
    npix = float(n) ** 3
    with np.errstate(invalid="ignore", divide="ignore"):
        val = vol ** 3 / npix ** 4 * (full.s - sd).real / full.count
    return val, full, sd


# ----------------------------------------------------------------------------
# Diagonal-binned trispectrum
# ----------------------------------------------------------------------------
#
# Four shells leave the quadrilateral k1 + k2 + k3 + k4 = 0 free to fold
# along its diagonal q = k1 + k2 = -(k3 + k4); binning |q| as well fixes the
# shape (Section 2, Eq. Jeong_gen with p = 4).  For a diagonal quad
# (a, b, c, d, e) the sum runs over closed quadruples (modulo N) with k1 in
# S_a, k2 in S_b, k3 in S_c, k4 in S_d and the reduced q in shell e (q = 0,
# the pairing k2 = -k1, is in no shell).

def _diag_order(counts, a, b, c, d):
    """A slot order with the same sum: the pair (k1, k2) may swap with
    (k3, k4) and each pair within itself; loop over the pair with fewer mode
    combinations, then the smaller shell of the other, and close the last."""
    if counts[c] * counts[d] < counts[a] * counts[b]:
        a, b, c, d = c, d, a, b
    if counts[d] < counts[c]:
        c, d = d, c
    return a, b, c, d


def trispectrum_diag(delta, k_lo, k_hi, dquads, box_len=None, delta_k=None) -> Spectrum:
    """Direct-sum diagonal-binned p = 4 polyspectrum for each (a, b, c, d, e):
    (V^3 / N_pix^4) S / N_q over the closed quadruples whose diagonal
    k1 + k2 lies in shell e."""
    d = prepare(delta)
    n = d.shape
    if delta_k is None:
        delta_k = dft3(d)
    dq = np.asarray(dquads, dtype=np.int64).reshape(-1, 5)
    lo2, hi2 = squared_edges(k_lo, k_hi, n)
    counts = mode_counts(n, k_lo, k_hi)
    modes = {}

    def sh(b):
        if b not in modes:
            modes[b] = shell_modes(n, k_lo, k_hi, b)
        return modes[b]

    re, im = _grid_parts(delta_k)
    acc = np.zeros((len(dq), _NACC))
    lib = _load()
    for t, (a, b, c, dd, e) in enumerate(dq):
        a, b, c, dd = _diag_order(counts, int(a), int(b), int(c), int(dd))
        mask = bin_mask_table(n, k_lo, k_hi, [dd])
        out = np.zeros((1, _NACC), dtype=np.float64)
        ma, mb, mc = sh(a), sh(b), sh(c)
        rc = lib.orc_triple_sums_diag(*grid_shape(n), *q_scales(n), _ptr(re, ctypes.c_double),
                                      _ptr(im, ctypes.c_double), len(ma), _ptr(ma, ctypes.c_int32),
                                      len(mb), _ptr(mb, ctypes.c_int32), len(mc), _ptr(mc, ctypes.c_int32),
                                      _ptr(mask, ctypes.c_uint64), len(mask), ctypes.c_uint64(1),
                                      float(lo2[e]), float(hi2[e]), 1, _ptr(out, ctypes.c_double))
        assert rc == 0, rc
        acc[t] = out[0]
    vol = _volume(n, box_len)
    npix = float(np.prod(n))
    return _finish(acc, vol ** 3 / npix ** 4)


def diag_disconnected_sums(delta, k_lo, k_hi, dquads, delta_k=None):
    """S_D per diagonal quad (a, b, c, d, e): the sum of D(k1) D(k2) D(k3) D(k4)
    over the closed quadruples of the diagonal sum that split into two pairs
    k_i = -k_j (Wick's pairings; k2 = -k1 has q = 0 and never enters), each
    quadruple counted once: the pairings k3 = -k1, k4 = -k2 and k4 = -k1,
    k3 = -k2 written out mode by mode as a set of quadruples."""
    d = prepare(delta)
    n = d.shape
    if delta_k is None:
        delta_k = dft3(d)
    lo2, hi2 = squared_edges(k_lo, k_hi, n)
    sc = q_scales(n)

    def wrap(m):
        return tuple(int(((m[i] + n[i] // 2) % n[i]) - n[i] // 2) if n[i] % 2 == 0
                     else int(((m[i] + (n[i] - 1) // 2) % n[i]) - (n[i] - 1) // 2) for i in range(3))

    def neg(m):
        return wrap((-m[0], -m[1], -m[2]))

    out = np.zeros(len(np.asarray(dquads).reshape(-1, 5)), dtype=np.complex128)
    for t, (a, b, c, dd, e) in enumerate(np.asarray(dquads, dtype=np.int64).reshape(-1, 5)):
        sets = [{tuple(int(x) for x in m) for m in shell_modes(n, k_lo, k_hi, int(x))} for x in (a, b, c, dd)]
        sa, sb, scs, sd = sets
        quadset = set()
        for k1 in sa:
            for k2 in sb:
                q = wrap((k1[0] + k2[0], k1[1] + k2[1], k1[2] + k2[2]))
                qq = float(_q_of(q[0], q[1], q[2], sc))
                if qq <= 0 or qq < lo2[e] or qq >= hi2[e]:
                    continue
                if neg(k1) in scs and neg(k2) in sd:
                    quadset.add((k1, k2, neg(k1), neg(k2)))       # k3 = -k1, k4 = -k2
                if neg(k2) in scs and neg(k1) in sd:
                    quadset.add((k1, k2, neg(k2), neg(k1)))       # k3 = -k2, k4 = -k1
        amp = lambda m: delta_k[m[0] % n[0], m[1] % n[1], m[2] % n[2]]
        out[t] = sum(amp(x[0]) * amp(x[1]) * amp(x[2]) * amp(x[3]) for x in quadset)
    return out


def trispectrum_diag_connected(delta, k_lo, k_hi, dquads, box_len=None, delta_k=None):
    """Diagonal-binned T with the Gaussian pairings removed: (V^3 / N_pix^4)
    Re(S - S_D) / N_q (diag_disconnected_sums).  Returns (value, raw
    Spectrum, S_D)."""
    d = prepare(delta)
    if delta_k is None:
        delta_k = dft3(d)
    full = trispectrum_diag(d, k_lo, k_hi, dquads, box_len=box_len, delta_k=delta_k)
    sd = diag_disconnected_sums(d, k_lo, k_hi, dquads, delta_k=delta_k)
    vol = _volume(d.shape, box_len)
    npix = float(np.prod(d.shape))
    with np.errstate(invalid="ignore", divide="ignore"):
        val = vol ** 3 / npix ** 4 * (full.s - sd).real / full.count
    return val, full, sd
