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
