"""The C-ABI library loads and exports every entry point include/bispec.h
declares; descriptor validation errors come back without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bispec.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:bispec_status|const char \*)\s*([a-z_]+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def b():
    from paper_1705_06284_amd import binding
    return binding


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("bispec_plan", "bispec_bin_fields", "bispec_estimate", "trispec_estimate",
                 "bispec_destroy", "bispec_plan_footprint", "bispec_set_workspace"):
        assert want in names


def test_library_exports_every_declared_symbol(b):
    lib = ctypes.CDLL(b.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings(b):
    for code, name in b.STATUS.items():
        assert b.bispec_status_string(code)
    assert b.bispec_status_string(-3).decode().startswith("bin edges")


def _desc(b, n=32, lo=(1.0,), hi=(4.0,), prec=0, batch=1, tri=None):
    d = b.PlanDesc()
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    d._keep = (lo, hi)
    d.n_side = n
    d.box_len = -1.0
    d.n_bins = len(lo)
    d.k_lo = lo.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.k_hi = hi.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if tri is not None:
        t = np.asarray(tri, np.int32)
        d._keep = (lo, hi, t)
        d.n_tri = len(t)
        d.tri = t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.precision = prec
    d.max_batch = batch
    return d


@pytest.mark.parametrize("kw,code", [
    (dict(n=1), -2), (dict(n=2048), -2), (dict(n=49), -2), (dict(n=131), -2), (dict(n=143), -2),
    (dict(lo=(1.0,), hi=(17.0,)), -3), (dict(lo=(5.0,), hi=(5.0,)), -3), (dict(lo=(-1.0,), hi=(2.0,)), -3),
    (dict(lo=(float("nan"),), hi=(2.0,)), -3),
    (dict(prec=7), -1), (dict(batch=0), -1), (dict(tri=[(0, 0, 3)]), -1),
])
def test_plan_rejects_bad_descriptors(b, kw, code):
    d = _desc(b, **kw)
    h = ctypes.c_void_p()
    assert b.bispec_plan(ctypes.byref(d), ctypes.byref(h)) == code
    assert not h.value


def test_null_arguments(b):
    h = ctypes.c_void_p()
    assert b.bispec_plan(None, ctypes.byref(h)) == -1
    assert b.bispec_estimate(None, None, 1, None, None) == -1
    assert b.trispec_estimate(None, None, 1, None) == -1
    assert b.bispec_bin_fields(None, None, 1, None) == -1
    assert b.bispec_theta_groups(None, 0, 0, 20, None, None) == -1
    assert b.bispec_rebin(None, None, 1, None, 1, None) == -1
    assert b.trispec_connected_estimate(None, None, 1, None, None) == -1
    sz = ctypes.c_size_t()
    assert b.bispec_plan_footprint(None, 1, ctypes.byref(sz)) == -1
