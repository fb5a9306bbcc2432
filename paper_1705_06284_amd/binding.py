"""ctypes binding of libbispec (the C ABI declared in include/bispec.h).

Argument marshalling only: every step of the estimator runs in the HIP
library.  PyTorch provides device memory (inputs, outputs, the workspace) and
the stream.  Importing this module loads ``libbispec.so`` and raises if it is
missing; there is no CPU fallback.

The module exposes the C entry points under their own names and a ``Plan``
class that owns a plan handle and a torch-allocated workspace.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbispec.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libbispec.so is not built (run __graft_entry__.build()); "
                      "there is no CPU fallback for the estimator")

_lib = ctypes.CDLL(LIB_PATH)

BISPEC_OK = 0
BISPEC_FP32 = 0
BISPEC_SPLIT_BF16 = 1
BISPEC_FP32_VALU = 2
TAIL_DEEP, TAIL_WIDE, TAIL_TWIN = 0, 1, 2        # block shapes of the fused tail kernel
STATUS = {0: "BISPEC_OK", -1: "BISPEC_E_INVALID", -2: "BISPEC_E_UNSUPPORTED_N", -3: "BISPEC_E_BIN_RANGE",
          -4: "BISPEC_E_EMPTY_BIN", -5: "BISPEC_E_NO_WORKSPACE", -6: "BISPEC_E_OOM", -7: "BISPEC_E_HIP",
          -8: "BISPEC_E_NUMERIC"}


class PlanDesc(ctypes.Structure):
    _fields_ = [("n_side", ctypes.c_int32), ("box_len", ctypes.c_double), ("n_bins", ctypes.c_int32),
                ("k_lo", ctypes.POINTER(ctypes.c_double)), ("k_hi", ctypes.POINTER(ctypes.c_double)),
                ("n_tri", ctypes.c_int32), ("tri", ctypes.POINTER(ctypes.c_int32)),
                ("n_quad", ctypes.c_int32), ("quad", ctypes.POINTER(ctypes.c_int32)),
                ("precision", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("n_y", ctypes.c_int32), ("n_x", ctypes.c_int32),
                ("n_dquad", ctypes.c_int32), ("dquad", ctypes.POINTER(ctypes.c_int32))]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_SIGS = {
    "bispec_plan": [ctypes.POINTER(PlanDesc), ctypes.POINTER(_vp)],
    "bispec_plan_footprint": [_vp, _i32, ctypes.POINTER(ctypes.c_size_t)],
    "bispec_set_workspace": [_vp, _vp, ctypes.c_size_t],
    "bispec_set_precision": [_vp, _i32],
    "bispec_set_stream": [_vp, _vp],
    "bispec_plan_query": [_vp, _ip, _ip, _dp, _dp],
    "bispec_plan_query_quads": [_vp, _ip, _ip],
    "bispec_plan_mode_counts": [_vp, ctypes.POINTER(ctypes.c_int64)],
    "bispec_bin_fields": [_vp, _vp, _i32, _vp],
    "bispec_estimate": [_vp, _vp, _i32, _vp, _vp],
    "trispec_estimate": [_vp, _vp, _i32, _vp],
    "trispec_connected_estimate": [_vp, _vp, _i32, _vp, _vp],
    "trispec_diag_estimate": [_vp, _vp, _i32, _vp, _vp],
    "bispec_plan_query_dquads": [_vp, _ip, _dp],
    "bispec_set_count_memory": [ctypes.c_size_t],
    "polyspec_estimate": [_vp, _vp, _i32, _vp, _vp, _vp],
    "polyspec_estimate_noalloc": [_vp, _vp, _i32, _vp, _vp, _vp],
    "bispec_timing_enable": [_vp, _i32],
    "bispec_graph_enable": [_vp, _i32],
    "bispec_autotune": [_vp, _vp, _ip, _ip],
    "bispec_set_tuning": [_vp, _i32, _i32],
    "bispec_plan_condition": [_vp, _dp],
    "bispec_theta_groups": [_vp, _i32, _i32, _i32, _ip, _dp],
    "bispec_rebin": [_vp, _vp, _i32, _vp, _i32, _vp],
    "bispec_timing_read": [_vp, _dp, _ip],
    "bispec_destroy": [_vp],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.bispec_status_string.argtypes = [ctypes.c_int]
_lib.bispec_status_string.restype = ctypes.c_char_p
_lib.bispec_last_error.argtypes = []
_lib.bispec_last_error.restype = ctypes.c_char_p

# The C entry points under their own names.
bispec_plan = _lib.bispec_plan
bispec_plan_footprint = _lib.bispec_plan_footprint
bispec_set_workspace = _lib.bispec_set_workspace
bispec_set_precision = _lib.bispec_set_precision
bispec_set_stream = _lib.bispec_set_stream
bispec_plan_query = _lib.bispec_plan_query
bispec_plan_query_quads = _lib.bispec_plan_query_quads
bispec_plan_mode_counts = _lib.bispec_plan_mode_counts
bispec_bin_fields = _lib.bispec_bin_fields
bispec_estimate = _lib.bispec_estimate
trispec_estimate = _lib.trispec_estimate
trispec_connected_estimate = _lib.trispec_connected_estimate
trispec_diag_estimate = _lib.trispec_diag_estimate
bispec_plan_query_dquads = _lib.bispec_plan_query_dquads
bispec_set_count_memory = _lib.bispec_set_count_memory
polyspec_estimate = _lib.polyspec_estimate
polyspec_estimate_noalloc = _lib.polyspec_estimate_noalloc
bispec_timing_enable = _lib.bispec_timing_enable
bispec_graph_enable = _lib.bispec_graph_enable
bispec_autotune = _lib.bispec_autotune
bispec_set_tuning = _lib.bispec_set_tuning
bispec_plan_condition = _lib.bispec_plan_condition
bispec_theta_groups = _lib.bispec_theta_groups
bispec_rebin = _lib.bispec_rebin
bispec_timing_read = _lib.bispec_timing_read
bispec_destroy = _lib.bispec_destroy
N_STAGES = 4
STAGES = ("forward", "inverse", "contract", "finalize")
bispec_status_string = _lib.bispec_status_string
bispec_last_error = _lib.bispec_last_error


class BispecError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        detail = bispec_last_error().decode()
        super().__init__("%s: %s (%s)%s" % (where, STATUS.get(code, code), bispec_status_string(code).decode(),
                                           (" [" + detail + "]") if detail else ""))


def check(code, where):
    if code != BISPEC_OK:
        raise BispecError(code, where)


def _precision(p):
    if isinstance(p, str):
        return {"fp32": BISPEC_FP32, "split_bf16": BISPEC_SPLIT_BF16, "fp32_valu": BISPEC_FP32_VALU}[p]
    return int(p)


def _arr(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Plan:
    """One estimator plan with a workspace allocated from torch on ``device``.

    n: the side N of a cubic grid, or its shape (N_z, N_y, N_x); k_lo, k_hi:
    shell edges in units of k_f (of the x axis); triplets: [n, 3] bin indices
    or None for every closed triplet; quads: [n, 4] or None for every
    (a,a,b,b); dquads: [n, 5] diagonal-binned configurations (a, b, c, d, e)
    or None.
    """

    def __init__(self, n, k_lo, k_hi, triplets=None, quads=None, box_len=None,
                 precision="split_bf16", max_batch=1, stream=None, device="cuda", dquads=None):
        import torch
        self._torch = torch
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the estimator runs on a GPU device only")
        torch.cuda.init()
        torch.empty(1, device=self.device)        # HIP context current before the library's first call
        shape = (int(n),) * 3 if np.ndim(n) == 0 else tuple(int(x) for x in n)
        if len(shape) != 3:
            raise ValueError("n: a side or a shape (N_z, N_y, N_x)")
        self.shape = shape
        self.n = shape[0]
        self.k_lo = _arr(k_lo, np.float64)
        self.k_hi = _arr(k_hi, np.float64)
        self.n_bins = len(self.k_lo)
        if len(self.k_hi) != self.n_bins:
            raise ValueError("k_lo and k_hi differ in length")
        tri = None if triplets is None else _arr(triplets, np.int32).reshape(-1, 3)
        qd = None if quads is None else _arr(quads, np.int32).reshape(-1, 4)
        dq = None if dquads is None else _arr(dquads, np.int32).reshape(-1, 5)
        self.max_batch = int(max_batch)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        d = PlanDesc()
        d.n_side = shape[0]
        d.n_y = shape[1]
        d.n_x = shape[2]
        d.n_dquad = 0 if dq is None else len(dq)
        d.dquad = dq.ctypes.data_as(_ip) if dq is not None else ctypes.cast(None, _ip)
        d.box_len = -1.0 if box_len is None else float(box_len)
        d.n_bins = self.n_bins
        d.k_lo = self.k_lo.ctypes.data_as(_dp)
        d.k_hi = self.k_hi.ctypes.data_as(_dp)
        d.n_tri = 0 if tri is None else len(tri)
        d.tri = tri.ctypes.data_as(_ip) if tri is not None else ctypes.cast(None, _ip)
        d.n_quad = 0 if qd is None else len(qd)
        d.quad = qd.ctypes.data_as(_ip) if qd is not None else ctypes.cast(None, _ip)
        d.precision = _precision(precision)
        d.max_batch = self.max_batch
        d.stream = ctypes.c_void_p(stream.cuda_stream)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(bispec_plan(ctypes.byref(d), ctypes.byref(h)), "bispec_plan")
        self.handle = h
        nt = ctypes.c_int32()
        check(bispec_plan_query(h, ctypes.byref(nt), None, None, None), "bispec_plan_query")
        self.n_tri = nt.value
        nq = ctypes.c_int32()
        check(bispec_plan_query_quads(h, ctypes.byref(nq), None), "bispec_plan_query_quads")
        self.n_quad = nq.value
        ndq = ctypes.c_int32()
        check(bispec_plan_query_dquads(h, ctypes.byref(ndq), None), "bispec_plan_query_dquads")
        self.n_dquad = ndq.value
        sz = ctypes.c_size_t()
        check(bispec_plan_footprint(h, self.max_batch, ctypes.byref(sz)), "bispec_plan_footprint")
        self.workspace_bytes = sz.value
        self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        check(bispec_set_workspace(h, _ptr(self.workspace), self.workspace_bytes), "bispec_set_workspace")

    # -- queries ------------------------------------------------------------
    @property
    def dquad_counts(self):
        """N_q(e) of every diagonal-binned configuration (exact integers)."""
        out = np.zeros(self.n_dquad, np.float64)
        check(bispec_plan_query_dquads(self.handle, None, out.ctypes.data_as(_dp)), "bispec_plan_query_dquads")
        return out

    @property
    def triplets(self):
        out = np.zeros((self.n_tri, 3), np.int32)
        check(bispec_plan_query(self.handle, None, out.ctypes.data_as(_ip), None, None), "query")
        return out

    @property
    def counts(self):
        out = np.zeros(self.n_tri, np.float64)
        check(bispec_plan_query(self.handle, None, None, out.ctypes.data_as(_dp), None), "query")
        return out

    @property
    def quads(self):
        out = np.zeros((self.n_quad, 4), np.int32)
        check(bispec_plan_query_quads(self.handle, None, out.ctypes.data_as(_ip)), "query_quads")
        return out

    @property
    def quad_counts(self):
        out = np.zeros(self.n_quad, np.float64)
        check(bispec_plan_query(self.handle, None, None, None, out.ctypes.data_as(_dp)), "query")
        return out

    @property
    def mode_counts(self):
        out = np.zeros(self.n_bins, np.int64)
        check(bispec_plan_mode_counts(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
              "mode_counts")
        return out

    def set_precision(self, precision):
        check(bispec_set_precision(self.handle, _precision(precision)), "bispec_set_precision")
        sz = ctypes.c_size_t()
        check(bispec_plan_footprint(self.handle, self.max_batch, ctypes.byref(sz)), "bispec_plan_footprint")
        if sz.value != self.workspace_bytes:          # the mode needs a different workspace
            self.workspace = None
            self.workspace_bytes = sz.value
            self.workspace = self._torch.empty(sz.value, dtype=self._torch.uint8, device=self.device)
            check(bispec_set_workspace(self.handle, _ptr(self.workspace), sz.value), "bispec_set_workspace")

    def autotune(self, delta=None):
        """Time the contraction kernel's launch shapes on the map delta (its
        compact rows; None: zeros); returns (blocks, shape), shape one of
        TAIL_DEEP, TAIL_WIDE, TAIL_TWIN."""
        nb, sh = ctypes.c_int32(), ctypes.c_int32()
        ptr = None
        if delta is not None:
            d = self._input(delta)
            ptr = _ptr(d[0])
            self._torch.cuda.synchronize(self.device)     # the map is ready before the plan's stream reads it
        check(bispec_autotune(self.handle, ptr, ctypes.byref(nb), ctypes.byref(sh)), "bispec_autotune")
        return nb.value, sh.value

    def set_tuning(self, nblk, shape):
        check(bispec_set_tuning(self.handle, int(nblk), int(shape)), "bispec_set_tuning")

    @property
    def condition(self):
        out = np.zeros(self.n_tri, np.float64)
        check(bispec_plan_condition(self.handle, out.ctypes.data_as(_dp)), "bispec_plan_condition")
        return out

    def theta_groups(self, b1, b2, n_cos=20):
        """(group [n_tri] int32, cos theta [n_tri]) for B(theta) at k1 in bin
        b1 and k2 in bin b2, as in bispec_theta_groups."""
        group = np.zeros(self.n_tri, np.int32)
        cos = np.zeros(self.n_tri, np.float64)
        check(bispec_theta_groups(self.handle, int(b1), int(b2), int(n_cos), group.ctypes.data_as(_ip),
                                  cos.ctypes.data_as(_dp)), "bispec_theta_groups")
        return group, cos

    def rebin(self, B, group, n_group):
        """Count-weighted averages of B ([batch, n_tri] device FP64) over the
        groups of triplets (host or device [n_tri] int32): [batch, n_group]."""
        torch = self._torch
        if B.dim() == 1:
            B = B.unsqueeze(0)
        if B.dtype != torch.float64 or not B.is_cuda or tuple(B.shape[1:]) != (self.n_tri,):
            raise ValueError("expected B as a [batch, %d] float64 tensor on %s" % (self.n_tri, self.device))
        B = B.contiguous()
        g = torch.as_tensor(np.asarray(group, dtype=np.int32) if not isinstance(group, torch.Tensor) else group)
        g = g.to(device=self.device, dtype=torch.int32).contiguous()
        if g.numel() != self.n_tri:
            raise ValueError("expected %d group entries" % self.n_tri)
        out = self._empty(B.shape[0], int(n_group))
        torch.cuda.synchronize(self.device)      # B and the group table are ready before the plan's stream reads them
        check(bispec_rebin(self.handle, _ptr(B), B.shape[0], _ptr(g), int(n_group), _ptr(out)), "bispec_rebin")
        return out

    def graph(self, on=True):
        check(bispec_graph_enable(self.handle, 1 if on else 0), "bispec_graph_enable")

    def timing(self, on=True):
        check(bispec_timing_enable(self.handle, 1 if on else 0), "bispec_timing_enable")

    def timing_read(self):
        """(per-stage milliseconds summed over calls, number of calls)."""
        ms = np.zeros(N_STAGES, np.float64)
        calls = ctypes.c_int32()
        check(bispec_timing_read(self.handle, ms.ctypes.data_as(_dp), ctypes.byref(calls)), "bispec_timing_read")
        return dict(zip(STAGES, ms.tolist())), calls.value

    def set_stream(self, stream):
        self.stream = stream
        check(bispec_set_stream(self.handle, ctypes.c_void_p(stream.cuda_stream)), "bispec_set_stream")

    # -- compute ------------------------------------------------------------
    def _input(self, delta):
        torch = self._torch
        if not isinstance(delta, torch.Tensor):
            delta = torch.from_numpy(np.ascontiguousarray(delta, dtype=np.float32))
        delta = delta.to(device=self.device, dtype=torch.float32).contiguous()
        if delta.dim() == 3:
            delta = delta.unsqueeze(0)
        if tuple(delta.shape[1:]) != self.shape:
            raise ValueError("expected [batch, %d, %d, %d]" % self.shape)
        return delta

    def _empty(self, *shape):
        return self._torch.empty(*shape, dtype=self._torch.float64, device=self.device)

    def _enter(self):
        """The plan's stream waits for the work queued so far on the current
        stream (the staging of the input, the allocation of the outputs)."""
        torch = self._torch
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)

    def _leave(self, *tensors):
        """Tensors the library reads or writes on the plan's stream stay
        allocated until that stream's work is done, even if the caller drops
        them (the caching allocator otherwise reuses their blocks on the
        current stream)."""
        torch = self._torch
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream == self.stream.cuda_stream:
            return
        for t in tensors:
            if t is not None:
                t.record_stream(self.stream)

    def polyspec(self, delta, want_p=True, want_b=True, want_t=True, out=None, batch=None):
        """(P, B, T) device tensors [batch, ...]; entries not wanted are None.
        delta None: the bin fields resident in the workspace (of ``batch``
        maps; see bin_fields(keep=True))."""
        if delta is None:
            d, bsz = None, int(batch or 1)
        else:
            d = self._input(delta)
            bsz = d.shape[0]
        if out is None:
            P = self._empty(bsz, self.n_bins) if want_p else None
            B = self._empty(bsz, self.n_tri) if want_b else None
            T = self._empty(bsz, self.n_quad) if want_t else None
        else:
            P, B, T = out
        self._enter()
        check(polyspec_estimate(self.handle, _ptr(d), bsz, _ptr(P), _ptr(B), _ptr(T)), "polyspec_estimate")
        self._leave(*[x for x in (d, P, B, T) if x is not None])
        return P, B, T

    def estimate(self, delta, want_p=True):
        """(B, P) as in bispec_estimate."""
        d = self._input(delta)
        bsz = d.shape[0]
        B = self._empty(bsz, self.n_tri)
        P = self._empty(bsz, self.n_bins) if want_p else None
        self._enter()
        check(bispec_estimate(self.handle, _ptr(d), bsz, _ptr(B), _ptr(P)), "bispec_estimate")
        self._leave(d, B, P)
        return B, P

    def trispec(self, delta):
        d = self._input(delta)
        bsz = d.shape[0]
        T = self._empty(bsz, self.n_quad)
        self._enter()
        check(trispec_estimate(self.handle, _ptr(d), bsz, _ptr(T)), "trispec_estimate")
        self._leave(d, T)
        return T

    def trispec_connected(self, delta):
        """(T, Tc) as in trispec_connected_estimate: the raw and the connected
        collapsed trispectrum, device tensors [batch, n_quad]."""
        d = self._input(delta)
        bsz = d.shape[0]
        T = self._empty(bsz, self.n_quad)
        Tc = self._empty(bsz, self.n_quad)
        self._enter()
        check(trispec_connected_estimate(self.handle, _ptr(d), bsz, _ptr(T), _ptr(Tc)), "trispec_connected_estimate")
        self._leave(d, T, Tc)
        return T, Tc

    def trispec_diag(self, delta, connected=True):
        """(Td, Tdc) as in trispec_diag_estimate: the diagonal-binned
        trispectrum of every planned (a, b, c, d, e) and, with connected, the
        same with the Gaussian pairings removed (else None); device tensors
        [batch, n_dquad]."""
        d = self._input(delta)
        bsz = d.shape[0]
        Td = self._empty(bsz, self.n_dquad)
        Tdc = self._empty(bsz, self.n_dquad) if connected else None
        self._enter()
        check(trispec_diag_estimate(self.handle, _ptr(d), bsz, _ptr(Td), _ptr(Tdc) if connected else None),
              "trispec_diag_estimate")
        self._leave(d, Td, *([Tdc] if connected else []))
        return Td, Tdc

    def bin_fields(self, delta, keep=False):
        """Device tensor [batch, n_bins, *shape] of the bin fields; keep=True
        leaves them in the workspace instead (returns None)."""
        d = self._input(delta)
        bsz = d.shape[0]
        if keep:
            self._enter()
            check(bispec_bin_fields(self.handle, _ptr(d), bsz, None), "bispec_bin_fields")
            self._leave(d)
            return None
        f = self._torch.empty((bsz, self.n_bins) + self.shape, dtype=self._torch.float32, device=self.device)
        self._enter()
        check(bispec_bin_fields(self.handle, _ptr(d), bsz, _ptr(f)), "bispec_bin_fields")
        self._leave(d, f)
        return f

    def close(self):
        if getattr(self, "handle", None):
            bispec_destroy(self.handle)
            self.handle = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
