"""ctypes declarations of the C ABI in include/mm.h (argument marshalling only)."""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmm.so")

MM_OK, MM_EINVAL, MM_ENOMEM, MM_EDEVICE, MM_ENOTCONV, MM_ESINGULAR, MM_EUNSUPPORTED = range(7)
STATUS_NAMES = {0: "MM_OK", 1: "MM_EINVAL", 2: "MM_ENOMEM", 3: "MM_EDEVICE", 4: "MM_ENOTCONV",
                5: "MM_ESINGULAR", 6: "MM_EUNSUPPORTED"}
MM_FP64, MM_MIXED = 0, 1
MM_PRECOND_BLOCK, MM_PRECOND_JACOBI, MM_PRECOND_NONE = 0, 1, 2
MM_F32, MM_F64 = 0, 1
MM_TMPL_ONEHOT, MM_TMPL_HWP = 1, 2

EXPORTED = ["mm_plan_workspace_size", "mm_plan", "mm_plan_create", "mm_destroy", "mm_plan_destroy",
            "mm_plan_get_info", "mm_hits", "mm_filter_lags", "mm_unpoint", "mm_point", "mm_weight", "mm_apply_A",
            "mm_rhs", "mm_solve_opts_default", "mm_solve", "mm_solve_rhs", "mm_noise_gradient",
            "mm_noise_lags_workspace_size", "mm_noise_lags", "mm_noise_lags_noalloc", "mm_fft_length_rule",
            "mm_last_error",
            "mm_version"]


class MMTemplate(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("n_seg", c_int32), ("n_amp", c_int64), ("d_idx", c_void_p),
                ("d_omega", c_void_p), ("seg_start", POINTER(c_int64))]


class MMDesc(ctypes.Structure):
    _fields_ = [
        ("n_stokes", c_int32), ("n_pix", c_int64), ("n_samples", c_int64), ("n_intervals", c_int32),
        ("iv_start", POINTER(c_int64)), ("iv_filter", POINTER(c_int32)), ("n_filters", c_int32),
        ("filter_params", POINTER(c_double)), ("filter_lags", POINTER(c_double)), ("f_samp", c_double),
        ("n_c", c_int32), ("n_f", c_int32), ("lag_dft_len", c_int32), ("precision", c_int32),
        ("precond", c_int32), ("n_rhs", c_int32), ("n_templates", c_int32),
        ("templates", POINTER(MMTemplate)), ("fft_shape", c_int32),
    ]


class MMPlanInfo(ctypes.Structure):
    _fields_ = [("n_obs", c_int64), ("n_valid", c_int64), ("n_f", c_int32), ("n_chunks", c_int32),
                ("n_singular", c_int32), ("device_bytes", c_int64), ("n_sliced", c_int64),
                ("n_tmpl", c_int64), ("fft_shape", c_int32)]


class MMSolveOpts(ctypes.Structure):
    _fields_ = [("tol", c_double), ("max_iter", c_int32), ("fixed_iters", c_int32),
                ("check_every", c_int32), ("use_graph", c_int32), ("true_residual", c_int32),
                ("d_x0", c_void_p), ("refine", c_int32), ("map_error", c_int32)]


class MMSolveInfo(ctypes.Structure):
    _fields_ = [("iters", POINTER(c_int32)), ("best_iter", POINTER(c_int32)),
                ("best_rel_res", POINTER(c_double)), ("true_rel_res", POINTER(c_double)),
                ("history", POINTER(c_double)), ("map_error", POINTER(c_double))]


class MMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_LIB = None


def load(path: str = LIB_PATH):
    """Load libmm.so; raises if it has not been built (there is no fallback)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_0906_1775_amd.build_lib`")
    lib = ctypes.CDLL(path)
    P = c_void_p
    lib.mm_plan_workspace_size.argtypes = [POINTER(MMDesc), POINTER(ctypes.c_size_t)]
    lib.mm_plan.argtypes = [POINTER(MMDesc), P, P, P, ctypes.c_size_t, P, POINTER(c_void_p)]
    lib.mm_plan_create.argtypes = [POINTER(MMDesc), P, P, P, POINTER(c_void_p)]
    lib.mm_destroy.argtypes = [P]
    lib.mm_plan_destroy.argtypes = [P]
    lib.mm_plan_get_info.argtypes = [P, POINTER(MMPlanInfo)]
    lib.mm_hits.argtypes = [P, P, P]
    lib.mm_filter_lags.argtypes = [P, P, P]
    lib.mm_unpoint.argtypes = [P, P, P, c_int32, P]
    lib.mm_point.argtypes = [P, P, c_int32, P, P]
    lib.mm_weight.argtypes = [P, P, P, c_int32, P]
    lib.mm_apply_A.argtypes = [P, P, P, P]
    lib.mm_rhs.argtypes = [P, P, c_int32, P, P]
    lib.mm_solve_opts_default.argtypes = [POINTER(MMSolveOpts)]
    lib.mm_solve_opts_default.restype = None
    lib.mm_solve.argtypes = [P, P, c_int32, P, POINTER(MMSolveOpts), POINTER(MMSolveInfo), P]
    lib.mm_solve_rhs.argtypes = [P, P, P, POINTER(MMSolveOpts), POINTER(MMSolveInfo), P]
    lib.mm_noise_gradient.argtypes = [P, P, c_int32, P, P, P, P]
    lib.mm_noise_lags_workspace_size.argtypes = [c_int32, c_int64, POINTER(ctypes.c_size_t)]
    lib.mm_noise_lags.argtypes = [P, c_int32, c_double, c_int32, c_int64, c_int32, P, P, ctypes.c_size_t, P]
    lib.mm_noise_lags_noalloc.argtypes = [P, c_int32, c_double, c_int32, c_int64, c_int32, P, P]
    lib.mm_fft_length_rule.argtypes = [c_int32, c_int64]
    lib.mm_fft_length_rule.restype = c_int32
    lib.mm_last_error.restype = c_char_p
    lib.mm_version.restype = c_char_p
    for name in ("mm_plan_workspace_size", "mm_plan", "mm_plan_create", "mm_destroy", "mm_plan_destroy",
                 "mm_plan_get_info", "mm_hits", "mm_filter_lags",
                 "mm_unpoint", "mm_point", "mm_weight", "mm_apply_A", "mm_rhs", "mm_solve",
                 "mm_solve_rhs", "mm_noise_gradient", "mm_noise_lags_workspace_size", "mm_noise_lags",
                 "mm_noise_lags_noalloc"):
        getattr(lib, name).restype = c_int32
    _LIB = lib
    return lib


def check(status: int, lib=None, allow=()):
    if status == MM_OK or status in allow:
        return status
    lib = lib or load()
    raise MMError(status, lib.mm_last_error().decode())
