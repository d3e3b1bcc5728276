"""Host-side checks of the C ABI that need no GPU: the shared library loads,
exports every function declared in include/nyspcg.h, and rejects invalid
arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    import paper_2110_02820_amd as nys
    if not os.path.exists(nys.LIB_PATH):
        from paper_2110_02820_amd import _build
        _build.build()
    return nys.lib()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "nyspcg.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\*|size_t|nys_status)\s+(nys_\w+)\s*\(", src, re.M)))


def test_header_declares_the_four_entry_points():
    names = declared_functions()
    for f in ("nys_sketch", "nys_factor", "nys_pcg_solve", "nys_pcg_backward"):
        assert f in names


def test_library_exports_every_declared_symbol(L):
    import paper_2110_02820_amd as nys
    names = declared_functions()
    assert len(names) >= 12
    for f in names:
        assert hasattr(L, f), f
    assert set(names) == set(nys.EXPORTED)


def test_struct_layouts_match_header(L):
    import paper_2110_02820_amd as nys
    assert ctypes.sizeof(nys._Operator) == 64
    assert ctypes.sizeof(nys._Precond) == 56
    assert ctypes.sizeof(nys._Opts) == 32


def _op(nys, kind=0, n=100, rows=100, cols=100, sigma=1.0):
    return nys._Operator(kind, nys.NYS_F64, n, 1, rows, cols, cols, sigma, 1.0)


def test_argument_errors_before_device_use(L):
    import paper_2110_02820_amd as nys
    op = _op(nys)
    # sketch size larger than n
    st = L.nys_sketch(ctypes.byref(op), 101, 0, None, 1, 1, 0, 1, 1 << 20, None)
    assert st == nys.NYS_ERR_ARG and b"ell" in L.nys_last_error()
    # bad operator: RBF with sigma <= 0
    bad = _op(nys, kind=nys.NYS_OP_RBF, cols=3, sigma=0.0)
    assert L.nys_workspace_size(ctypes.byref(bad), 10, 1, 0) == 0
    st = L.nys_sketch(ctypes.byref(bad), 10, 0, None, 1, 1, 0, 1, 1 << 20, None)
    assert st == nys.NYS_ERR_ARG and b"sigma" in L.nys_last_error()
    # X^T X shape mismatch
    bad = _op(nys, kind=nys.NYS_OP_XTX, n=50, rows=80, cols=60)
    assert L.nys_workspace_size(ctypes.byref(bad), 10, 1, 0) == 0
    # gaussian with empty shape
    assert L.nys_gaussian(1, 0, 5, 1, 5, None) == nys.NYS_ERR_ARG
    # preconditioner with ell > n
    P = nys._Precond(10, 11, 1, 11, 0, 0, 1, 0.0)
    assert L.nys_factor(1, 1, ctypes.byref(P), 0, 1, 1 << 20, None) == nys.NYS_ERR_ARG
    # more than 256 simultaneous columns
    P = nys._Precond(100, 10, 1, 10, 0, 0, 1, 0.0)
    mu = (ctypes.c_double * 300)(*([1.0] * 300))
    o = nys._Opts(1e-10, 100, 0, 0, 0, 0.0)
    st = L.nys_pcg_solve(ctypes.byref(op), ctypes.byref(P), mu, 300, 1, 1, 1, 1, 300, ctypes.byref(o), None,
                         1, 1 << 20, None)
    assert st == nys.NYS_ERR_ARG


def test_workspace_size_grows_with_problem(L):
    import paper_2110_02820_amd as nys
    a = L.nys_workspace_size(ctypes.byref(_op(nys, n=1000, rows=1000, cols=1000)), 50, 1, 0)
    b = L.nys_workspace_size(ctypes.byref(_op(nys, n=2000, rows=2000, cols=2000)), 100, 1, 0)
    assert 0 < a < b
