"""Host-side checks of the C ABI that need no GPU: the shared library loads,
exports every function declared in include/nyspcg.h, and rejects invalid
arguments before touching the device."""
import ctypes
import os
import re
import subprocess

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
    return sorted(set(re.findall(r"^\s*(?:const\s+char\*|size_t|int64_t|nys_status)\s+(nys_\w+)\s*\(", src, re.M)))


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


def _c_layout(tmp_path, structs):
    """sizeof and every field offset of the header's structs, as the C compiler
    lays them out."""
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "nyspcg.h"', 'int main(void) {']
    for cname, fields in structs:
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in fields:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {tuple(line.split()[:2]): int(line.split()[2]) for line in out.splitlines()}


def test_struct_layouts_match_header(L, tmp_path):
    import paper_2110_02820_amd as nys
    pairs = [("nys_operator", nys._Operator), ("nys_precond", nys._Precond), ("nys_solve_opts", nys._Opts),
             ("nys_solve_info", nys._Info)]
    lay = _c_layout(tmp_path, [(c, [f[0] for f in py._fields_]) for c, py in pairs])
    for cname, py in pairs:
        assert lay[(cname, "size")] == ctypes.sizeof(py), cname
        for f in py._fields_:
            assert lay[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])


def _op(nys, kind=0, n=100, rows=100, cols=100, sigma=1.0):
    return nys._Operator(kind, nys.NYS_F64, n, 1, rows, cols, cols, sigma, 1.0)


def test_callback_operator_checked_on_host(L):
    import paper_2110_02820_amd as nys
    # a callback operator without a routine is refused before any device work
    op = nys._Operator(nys.NYS_OP_CALLBACK, nys.NYS_F64, 100, None, 0, 0, 0, 0.0, 1.0)
    assert L.nys_workspace_size(ctypes.byref(op), 10, 1, 0) == 0
    st = L.nys_sketch(ctypes.byref(op), 10, 0, None, 1, 1, 0, 1, 1 << 20, None)
    assert st == nys.NYS_ERR_ARG and b"apply" in L.nys_last_error()
    # with a routine, data / rows / cols / ld are not looked at
    fn = nys.APPLY_FN(lambda *a: 0)
    op = nys._Operator(nys.NYS_OP_CALLBACK, nys.NYS_F64, 100, None, 0, 0, 0, 0.0, 1.0, fn, None)
    assert L.nys_workspace_size(ctypes.byref(op), 10, 1, 0) > 0
    # the column-sampling sketch has no callback form
    assert L.nys_workspace_size_columns(ctypes.byref(op), 10) == 0
    st = L.nys_sketch_columns(ctypes.byref(op), 10, 1, 1, 1, 1, 1 << 20, None)
    assert st == nys.NYS_ERR_ARG and b"callback" in L.nys_last_error()


def test_device_info_form_argument_checks(L):
    import paper_2110_02820_amd as nys
    op = _op(nys)
    P = nys._Precond(100, 10, 1, 10, 0, 0, 1, 0.0)
    mu = (ctypes.c_double * 2)(1e-3, 0.0)
    o = nys._Opts(1e-10, 100, 0, 0, 0, 0.0, 1, 0)
    # mu = 0 is refused in the device-info form (nothing is read back to check lam_l + mu)
    st = L.nys_pcg_solve(ctypes.byref(op), ctypes.byref(P), mu, 2, 1, 1, 1, 1, 2, ctypes.byref(o), None,
                         1, 1 << 20, None)
    assert st == nys.NYS_ERR_ARG and b"mu" in L.nys_last_error()
    o = nys._Opts(1e-10, 100, 0, 0, 0, 0.0, 2, 0)
    st = L.nys_pcg_solve(ctypes.byref(op), ctypes.byref(P), mu, 1, 1, 1, 1, 1, 1, ctypes.byref(o), None,
                         1, 1 << 20, None)
    assert st == nys.NYS_ERR_ARG and b"device_info" in L.nys_last_error()
    # the adjoint and the ragged batch synchronise: no device-info form
    o = nys._Opts(1e-10, 100, 0, 0, 0, 0.0, 1, 0)
    g = ctypes.c_double(0.0)
    st = L.nys_pcg_backward(ctypes.byref(op), ctypes.byref(P), 1e-3, 1, 1, 1, ctypes.byref(g), None, None,
                            ctypes.byref(o), None, 1, 1 << 20, None)
    assert st == nys.NYS_ERR_ARG and b"device-info" in L.nys_last_error()


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
    o = nys._Opts(1e-10, 100, 0, 0, 0, 0.0, 0, 0)
    st = L.nys_pcg_solve(ctypes.byref(op), ctypes.byref(P), mu, 300, 1, 1, 1, 1, 300, ctypes.byref(o), None,
                         1, 1 << 20, None)
    assert st == nys.NYS_ERR_ARG


def test_workspace_size_grows_with_problem(L):
    import paper_2110_02820_amd as nys
    a = L.nys_workspace_size(ctypes.byref(_op(nys, n=1000, rows=1000, cols=1000)), 50, 1, 0)
    b = L.nys_workspace_size(ctypes.byref(_op(nys, n=2000, rows=2000, cols=2000)), 100, 1, 0)
    assert 0 < a < b


def test_autotune_table_load_save_query(L, tmp_path):
    """The tile-shape table of the RBF block products: a cache file is merged
    into the table, a lookup takes the entry with the smallest tuned column
    count >= k for the same (n, d, Gram precision) and falls back to the
    built-in rule otherwise, save writes what was loaded, and a malformed
    file is rejected as a whole.  Host only: the operator's data pointer is
    never dereferenced by these calls."""
    import paper_2110_02820_amd as nys
    L.nys_autotune_clear()
    assert L.nys_autotune_entries() == 0
    # RBF operator, n = 5000 points in d = 16 (pointer not used by the lookup)
    op = nys._Operator(nys.NYS_OP_RBF, nys.NYS_F32, 5000, ctypes.c_void_p(1), 5000, 16, 16, 4.0, 1.0)
    ch = (ctypes.c_int32 * 4)()
    tuned = ctypes.c_int32(7)
    f32 = nys.NYS_PREC_FP32_REFINE64
    bf = nys.NYS_PREC_BF16X3_REFINE64
    # built-in rule: register kernel with 1 / 2 / 4 tiles up to 64 columns, past that the LDS
    # kernel with 128 columns and two row fragments per wave
    for k, want in ((8, (1, 1, 8, 1)), (32, (1, 2, 8, 1)), (64, (1, 4, 8, 1)), (100, (0, 8, 8, 2)),
                    (256, (0, 8, 8, 2))):
        assert L.nys_autotune_query(ctypes.byref(op), f32, k, ch, ctypes.byref(tuned)) == 0
        assert tuple(ch) == want and tuned.value == 0
    cache = tmp_path / "tune.txt"
    cache.write_text("# comment\n"
                     "rbf_kv 5000 16 1 16 1 4 16 10.5\n"
                     "rbf_kv 5000 16 1 128 0 16 4 99.0 2\n"
                     "rbf_kv 5000 16 0 128 1 2 8 77.0\n"
                     "rbf_kv 6000 16 1 512 1 1 4 1.0\n")
    assert L.nys_autotune_load(str(cache).encode()) == 0
    assert L.nys_autotune_entries() == 4
    cases = [(f32, 10, (1, 4, 16, 1), 1), (f32, 16, (1, 4, 16, 1), 1), (f32, 17, (0, 16, 4, 2), 1),
             (f32, 128, (0, 16, 4, 2), 1), (f32, 129, (0, 8, 8, 2), 0), (bf, 100, (1, 2, 8, 1), 1),
             (bf, 8, (1, 2, 8, 1), 1)]
    for prec, k, want, t in cases:
        assert L.nys_autotune_query(ctypes.byref(op), prec, k, ch, ctypes.byref(tuned)) == 0
        assert (tuple(ch), tuned.value) == (want, t), (prec, k)
    # another d: no entry applies
    op_d8 = nys._Operator(nys.NYS_OP_RBF, nys.NYS_F32, 5000, ctypes.c_void_p(1), 5000, 8, 8, 4.0, 1.0)
    assert L.nys_autotune_query(ctypes.byref(op_d8), f32, 16, ch, ctypes.byref(tuned)) == 0
    assert tuned.value == 0
    out = tmp_path / "saved.txt"
    assert L.nys_autotune_save(str(out).encode()) == 0
    rows = sorted(l.split()[:8] + l.split()[9:10] for l in out.read_text().splitlines() if not l.startswith("#"))
    src = sorted(l.split()[:8] + (l.split()[9:10] or ["1"]) for l in cache.read_text().splitlines()
                 if not l.startswith("#"))
    assert rows == src
    # a malformed file (cf 3 is no shape) changes nothing
    bad = tmp_path / "bad.txt"
    bad.write_text("rbf_kv 5000 16 1 32 1 3 8 1.0\n")
    assert L.nys_autotune_load(str(bad).encode()) == nys.NYS_ERR_ARG
    bad.write_text("rbf_kv 5000 16 1 32 1 4 8 1.0 2\n")  # the register kernel has one fragment
    assert L.nys_autotune_load(str(bad).encode()) == nys.NYS_ERR_ARG
    assert L.nys_autotune_entries() == 4
    assert L.nys_autotune_load(str(tmp_path / "missing.txt").encode()) == nys.NYS_ERR_ARG
    # loading again replaces entries with the same key instead of adding them
    assert L.nys_autotune_load(str(cache).encode()) == 0
    assert L.nys_autotune_entries() == 4
    # only reduced-precision RBF products are tuned
    assert L.nys_autotune_query(ctypes.byref(op), nys.NYS_PREC_FP64, 16, ch, None) == nys.NYS_ERR_ARG
    L.nys_autotune_clear()
    assert L.nys_autotune_entries() == 0
