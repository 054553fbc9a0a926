"""The C-ABI library loads, exports every entry point include/mm.h declares, and its
host-only logic (FFT-length rule, descriptor validation) behaves; no GPU needed."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[A-Za-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_0906_1775_amd import _lib
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "mm_solve" in names and "mm_plan_create" in names and "mm_apply_A" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_declares_every_header_function():
    from paper_0906_1775_amd import _lib
    assert sorted(_lib.EXPORTED) == declared_functions()


def test_fft_length_rule_matches_the_oracle(lib):
    from oracle import fftlen
    rows = [tuple(int(v) for v in l.split()) for l in open(os.path.join(ROOT, "tests", "golden",
            "fft_length_rule.txt")) if l.strip() and not l.startswith("#")]
    for nc, longest, nf in rows:
        assert lib.mm_fft_length_rule(nc, longest) == nf
    rng = np.random.default_rng(0)
    for _ in range(2000):
        nc = int(rng.integers(1, 20000))
        longest = int(rng.integers(1, 1 << 23))
        assert lib.mm_fft_length_rule(nc, longest) == fftlen.paper_fft_length(nc, longest), (nc, longest)


def test_version_and_defaults(lib):
    from paper_0906_1775_amd import _lib
    assert lib.mm_version().decode().startswith("mm ")
    o = _lib.MMSolveOpts()
    lib.mm_solve_opts_default(ctypes.byref(o))
    assert o.tol == 1e-6 and o.max_iter == 50      # the paper's defaults
    assert lib.mm_last_error() is not None


def _desc(**kw):
    from paper_0906_1775_amd import _lib
    d = _lib.MMDesc()
    iv = np.array([0, 100], np.int64)
    fl = np.array([0], np.int32)
    fp = np.array([1.0, 0.1, 1.5])
    d.n_stokes, d.n_pix, d.n_samples, d.n_intervals = 1, 10, 100, 1
    d.iv_start = iv.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    d.iv_filter = fl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.n_filters = 1
    d.filter_params = fp.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.f_samp, d.n_c, d.n_rhs = 100.0, 8, 1
    for k, v in kw.items():
        setattr(d, k, v)
    return d, (iv, fl, fp)


@pytest.mark.parametrize("field,value,msg", [
    ("n_stokes", 2, "n_stokes"), ("n_rhs", 0, "n_rhs"), ("n_c", 0, "n_c"),
    ("n_f", 24, "n_f"), ("n_f", 16, "n_f"), ("precision", 7, "precision"),
    ("n_samples", -1, "n_samples"), ("f_samp", 0.0, "f_samp"),
])
def test_descriptor_validation_fails_before_touching_the_device(lib, field, value, msg):
    from paper_0906_1775_amd import _lib
    d, keep = _desc(**{field: value})
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    st = lib.mm_plan_create(ctypes.byref(d), fake, None, None, ctypes.byref(h))
    assert st == _lib.MM_EINVAL
    assert msg in lib.mm_last_error().decode()
    assert not h.value


def test_null_descriptor(lib):
    from paper_0906_1775_amd import _lib
    h = ctypes.c_void_p()
    assert lib.mm_plan_create(None, None, None, None, ctypes.byref(h)) == _lib.MM_EINVAL
    assert lib.mm_plan_create(None, None, None, None, None) == _lib.MM_EINVAL


def _template_desc(tmpl):
    from paper_0906_1775_amd import _lib
    d, keep = _desc()
    arr = (_lib.MMTemplate * 1)(tmpl)
    d.n_templates = 1
    d.templates = ctypes.cast(arr, ctypes.POINTER(_lib.MMTemplate))
    return d, (keep, arr)


@pytest.mark.parametrize("case,msg", [
    ("kind", "unknown template kind"), ("n_amp", "n_amp"), ("idx", "d_idx"),
    ("n_seg", "n_seg"), ("seg_end", "end at n_samples"), ("seg_order", "non-decreasing"),
    ("omega", "d_omega"),
])
def test_template_validation_fails_before_touching_the_device(lib, case, msg):
    from paper_0906_1775_amd import _lib
    fake = 0x1000                     # never dereferenced: validation fails first
    seg_ok = np.array([0, 40, 100], np.int64)
    seg_end = np.array([0, 40, 99], np.int64)
    seg_order = np.array([0, 60, 40, 100], np.int64)
    t = _lib.MMTemplate()
    if case in ("kind", "n_amp", "idx"):
        t.kind, t.n_amp, t.d_idx = _lib.MM_TMPL_ONEHOT, 5, fake
        if case == "kind":
            t.kind = 9
        if case == "n_amp":
            t.n_amp = 0
        if case == "idx":
            t.d_idx = None
    else:
        seg = {"seg_end": seg_end, "seg_order": seg_order}.get(case, seg_ok)
        t.kind, t.n_seg, t.d_omega = _lib.MM_TMPL_HWP, seg.shape[0] - 1, fake
        t.seg_start = seg.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        if case == "n_seg":
            t.n_seg = 0
        if case == "omega":
            t.d_omega = None
    d, keep = _template_desc(t)
    h = ctypes.c_void_p()
    st = lib.mm_plan_create(ctypes.byref(d), ctypes.c_void_p(fake), None, None, ctypes.byref(h))
    assert st == _lib.MM_EINVAL
    assert msg in lib.mm_last_error().decode()
    assert not h.value


def test_ctypes_layouts_match_the_header(tmp_path):
    """sizeof / offsetof of every ABI struct, from a C program built with gcc, equal the binding's."""
    import shutil
    import subprocess
    from paper_0906_1775_amd import _lib
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"mm_desc_t": _lib.MMDesc, "mm_template_t": _lib.MMTemplate, "mm_plan_info_t": _lib.MMPlanInfo,
               "mm_solve_opts_t": _lib.MMSolveOpts, "mm_solve_info_t": _lib.MMSolveInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mm.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def _ws_size(lib, d):
    n = ctypes.c_size_t(0)
    st = lib.mm_plan_workspace_size(ctypes.byref(d), ctypes.byref(n))
    return st, int(n.value)


def _big_desc(n_t, n_pix, R, precision, ns=3, n_c=8192, iv_len=1 << 20, n_f=0):
    from paper_0906_1775_amd import _lib
    iv = np.arange(0, n_t + 1, iv_len, dtype=np.int64)
    if iv[-1] != n_t:
        iv = np.append(iv, n_t)
    fl = np.zeros(iv.shape[0] - 1, np.int32)
    fp = np.array([1.0, 0.2, 1.7])
    d = _lib.MMDesc()
    d.n_stokes, d.n_pix, d.n_samples, d.n_intervals = ns, n_pix, n_t, fl.shape[0]
    d.iv_start = iv.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    d.iv_filter = fl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.n_filters = 1
    d.filter_params = fp.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.f_samp, d.n_c, d.n_rhs, d.precision, d.n_f = 200.0, n_c, R, precision, n_f
    return d, (iv, fl, fp)


def test_workspace_bound_is_host_only_and_grows_with_the_problem(lib):
    from paper_0906_1775_amd import _lib
    sizes = {}
    for R in (1, 4):
        for prec in (_lib.MM_FP64, _lib.MM_MIXED):
            d, keep = _big_desc(1 << 24, 1 << 16, R, prec)
            st, n = _ws_size(lib, d)
            assert st == _lib.MM_OK, lib.mm_last_error()
            sizes[(R, prec)] = n
    # every bound holds at least the two TOD work buffers and the pointing index
    assert sizes[(1, _lib.MM_MIXED)] >= 2 * 8 * (1 << 24) + 4 * (1 << 24)
    assert sizes[(4, _lib.MM_FP64)] > sizes[(1, _lib.MM_FP64)]
    assert sizes[(4, _lib.MM_MIXED)] > sizes[(1, _lib.MM_MIXED)]
    assert sizes[(4, _lib.MM_FP64)] > sizes[(4, _lib.MM_MIXED)]   # float64 TOD work buffers


def test_workspace_bound_of_the_largest_workload_fits_one_device(lib):
    """2^30 samples, 12 x 2048^2 pixels x TQU, 8 RHS, mixed precision: the plan's bound plus its
    inputs (index, polarisation pair, 8 float32 TOD rows) stays within one MI355X's 288 GB."""
    from paper_0906_1775_amd import _lib
    n_t = 1 << 30
    d, keep = _big_desc(n_t, 12 * 2048 * 2048, 8, _lib.MM_MIXED, iv_len=1 << 20)
    st, n = _ws_size(lib, d)
    assert st == _lib.MM_OK, lib.mm_last_error()
    inputs = n_t * (4 + 8 + 8 * 4)
    assert n + inputs < 270e9, (n, inputs)


@pytest.mark.parametrize("field,value,msg", [
    ("n_stokes", 2, "n_stokes"), ("n_rhs", 65, "n_rhs"), ("n_f", 24, "n_f"), ("f_samp", 0.0, "f_samp"),
])
def test_workspace_size_validates_the_descriptor(lib, field, value, msg):
    from paper_0906_1775_amd import _lib
    d, keep = _desc(**{field: value})
    st, n = _ws_size(lib, d)
    assert st == _lib.MM_EINVAL and msg in lib.mm_last_error().decode()
    assert lib.mm_plan_workspace_size(None, None) == _lib.MM_EINVAL


def test_forced_transform_beyond_the_chip_is_unsupported_in_the_bound(lib):
    from paper_0906_1775_amd import _lib
    d, keep = _big_desc(1 << 20, 1024, 1, _lib.MM_MIXED, n_f=1 << 20)
    st, _ = _ws_size(lib, d)
    assert st == _lib.MM_EUNSUPPORTED


def test_workspace_checks_fail_before_touching_the_device(lib):
    from paper_0906_1775_amd import _lib
    d, keep = _desc()
    st, need = _ws_size(lib, d)
    assert st == _lib.MM_OK and need > 0
    fake = ctypes.c_void_p(0x1000)          # never dereferenced: the checks fail first
    h = ctypes.c_void_p()
    assert lib.mm_plan(ctypes.byref(d), fake, None, None, need, None, ctypes.byref(h)) == _lib.MM_EINVAL
    assert "d_ws" in lib.mm_last_error().decode() and not h.value
    assert lib.mm_plan(ctypes.byref(d), fake, None, ctypes.c_void_p(0x100000), need - 1, None,
                       ctypes.byref(h)) == _lib.MM_EINVAL
    assert "below" in lib.mm_last_error().decode() and not h.value
    assert lib.mm_plan(ctypes.byref(d), fake, None, ctypes.c_void_p(0x100001), need, None,
                       ctypes.byref(h)) == _lib.MM_EINVAL
    assert "aligned" in lib.mm_last_error().decode() and not h.value
    assert lib.mm_destroy(None) == _lib.MM_OK


def test_lag_construction_arguments_fail_before_touching_the_device(lib):
    from paper_0906_1775_amd import _lib
    n = ctypes.c_size_t(0)
    assert lib.mm_noise_lags_workspace_size(8192, 1 << 20, ctypes.byref(n)) == _lib.MM_OK
    assert n.value >= 128 * 8192 * 16          # one filter's 2^20 / 2^13 partial transforms of 8192 points
    assert lib.mm_noise_lags_workspace_size(8192, 1 << 14, ctypes.byref(n)) == _lib.MM_EINVAL   # < 4 n_c
    assert lib.mm_noise_lags_workspace_size(1 << 15, 1 << 20, ctypes.byref(n)) == _lib.MM_EUNSUPPORTED
    fake = ctypes.c_void_p(0x1000)              # never dereferenced: the checks fail first
    cases = [dict(n_filters=0), dict(n_c=0), dict(f_samp=0.0), dict(deriv=4), dict(lag=3 << 18),
             dict(ws=None), dict(ws_bytes=16), dict(ws=ctypes.c_void_p(0x1001))]
    for c in cases:
        st = lib.mm_noise_lags(fake, c.get("n_filters", 2), c.get("f_samp", 200.0), c.get("n_c", 64),
                               c.get("lag", 1 << 14), c.get("deriv", 0), fake, c.get("ws", fake),
                               c.get("ws_bytes", 1 << 30), None)
        assert st == _lib.MM_EINVAL, (c, lib.mm_last_error())
