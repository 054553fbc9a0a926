"""Torch-facing wrapper of libmm: device tensors in, device tensors out.

Every computation runs in the HIP library; this module only checks tensor
shapes and dtypes, passes pointers and the current stream, and converts
results.  Maps are float64 tensors [n_rhs, n_pix, n_stokes]; TOD tensors are
float32 or float64 [n_rhs, n_samples].  A plan with templates (the extended
pointing [P B]) uses flat map-shaped tensors [n_rhs, n_pix * n_stokes + n_tmpl]
instead: the map values, then the template amplitudes (``split`` separates them).
"""

from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib as L

_PREC = {"fp64": L.MM_FP64, "mixed": L.MM_MIXED}
_PRECOND = {"block": L.MM_PRECOND_BLOCK, "jacobi": L.MM_PRECOND_JACOBI, "none": L.MM_PRECOND_NONE}


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _tod_dtype(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return L.MM_F32
    if t.dtype == torch.float64:
        return L.MM_F64
    raise TypeError("TOD must be float32 or float64")


def fft_length_rule(n_c: int, longest: int) -> int:
    return int(L.load().mm_fft_length_rule(int(n_c), int(longest)))


def noise_lags(params: torch.Tensor, f_samp: float, n_c: int, lag_dft_len: int = 1 << 20,
               deriv: int = 0) -> torch.Tensor:
    """Lags f(tau) [n_filters, n_c] (or their derivative, deriv = 1 .. 3 for sigma, f_knee,
    alpha) of the inverse-noise filter for the parameters ``params`` (float64 CUDA tensor
    [n_filters, 3] = sigma, f_knee, alpha), computed by mm_noise_lags in a torch workspace."""
    lib = L.load()
    if not params.is_cuda or params.dtype != torch.float64 or not params.is_contiguous() \
            or params.dim() != 2 or params.shape[1] != 3:
        raise ValueError("params must be a contiguous float64 CUDA tensor [n_filters, 3]")
    n = ctypes.c_size_t(0)
    L.check(lib.mm_noise_lags_workspace_size(int(n_c), int(lag_dft_len), ctypes.byref(n)), lib)
    ws = torch.empty(int(n.value), dtype=torch.uint8, device=params.device)
    out = torch.empty((params.shape[0], int(n_c)), dtype=torch.float64, device=params.device)
    L.check(lib.mm_noise_lags(_ptr(params), int(params.shape[0]), float(f_samp), int(n_c), int(lag_dft_len),
                              int(deriv), _ptr(out), _ptr(ws), ctypes.c_size_t(ws.numel()), _stream()), lib)
    return out


class MapMaker:
    """A plan of the map-making operators for one pointing and noise model."""

    def __init__(self, pix: torch.Tensor, w: Optional[torch.Tensor], n_pix: int, n_stokes: int,
                 iv_start, iv_filter, filter_params=None, filter_lags=None, f_samp: float = 0.0,
                 n_c: int = 1, n_f: int = 0, lag_dft_len: int = 0, precision: str = "fp64",
                 precond: str = "block", n_rhs: int = 1, templates=None, fft_shape: int = 0):
        """``templates``: optional list of dicts, each
        ``{"kind": "onehot", "idx": int32 CUDA tensor [n_samples], "n_amp": int}`` or
        ``{"kind": "hwp", "omega": float32 CUDA tensor [n_samples], "seg_start": int sequence}``;
        the plan reads the tensors until it is destroyed."""
        self._lib = L.load()
        if not pix.is_cuda or pix.dtype != torch.int32 or not pix.is_contiguous():
            raise ValueError("pix must be a contiguous int32 CUDA tensor")
        if n_stokes == 3:
            if w is None or not w.is_cuda or w.dtype != torch.float32 or not w.is_contiguous() \
                    or tuple(w.shape) != (pix.shape[0], 2):
                raise ValueError("w must be a contiguous float32 CUDA tensor [n_samples, 2]")
        self.pix, self.w = pix, w            # the plan reads w until it is destroyed
        self.n_pix, self.n_stokes, self.n_rhs = int(n_pix), int(n_stokes), int(n_rhs)
        self.n_samples = int(pix.shape[0])
        self.n_c = int(n_c)
        self._iv_start = np.ascontiguousarray(iv_start, dtype=np.int64)
        self._iv_filter = np.ascontiguousarray(iv_filter, dtype=np.int32)
        self._params = None if filter_params is None else np.ascontiguousarray(filter_params, np.float64)
        self._lags = None if filter_lags is None else np.ascontiguousarray(filter_lags, np.float64)
        n_filters = (self._params if self._params is not None else self._lags).shape[0]
        self.n_filters = int(n_filters)
        d = L.MMDesc()
        d.n_stokes = self.n_stokes
        d.n_pix = self.n_pix
        d.n_samples = self.n_samples
        d.n_intervals = int(self._iv_filter.shape[0])
        d.iv_start = self._iv_start.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        d.iv_filter = self._iv_filter.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.n_filters = self.n_filters
        d.filter_params = None if self._params is None else \
            self._params.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.filter_lags = None if self._lags is None else \
            self._lags.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.f_samp = float(f_samp)
        d.n_c = self.n_c
        d.n_f = int(n_f)
        d.lag_dft_len = int(lag_dft_len)
        d.precision = _PREC[precision]
        d.precond = _PRECOND[precond]
        d.n_rhs = self.n_rhs
        d.fft_shape = int(fft_shape)
        self._tmpl_keep = []
        self.templates = list(templates or [])
        if self.templates:
            arr = (L.MMTemplate * len(self.templates))()
            for k, t in enumerate(self.templates):
                if t["kind"] == "onehot":
                    idx = t["idx"]
                    if not idx.is_cuda or idx.dtype != torch.int32 or not idx.is_contiguous() \
                            or tuple(idx.shape) != (self.n_samples,):
                        raise ValueError("one-hot idx must be a contiguous int32 CUDA tensor [n_samples]")
                    arr[k].kind, arr[k].n_amp, arr[k].d_idx = L.MM_TMPL_ONEHOT, int(t["n_amp"]), idx.data_ptr()
                    self._tmpl_keep.append(idx)
                elif t["kind"] == "hwp":
                    om = t["omega"]
                    if not om.is_cuda or om.dtype != torch.float32 or not om.is_contiguous() \
                            or tuple(om.shape) != (self.n_samples,):
                        raise ValueError("HWP omega must be a contiguous float32 CUDA tensor [n_samples]")
                    seg = np.ascontiguousarray(t["seg_start"], dtype=np.int64)
                    arr[k].kind, arr[k].n_seg, arr[k].d_omega = L.MM_TMPL_HWP, int(seg.shape[0] - 1), om.data_ptr()
                    arr[k].seg_start = seg.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
                    self._tmpl_keep += [om, seg]
                else:
                    raise ValueError(f"unknown template kind {t['kind']!r}")
            d.n_templates = len(self.templates)
            d.templates = ctypes.cast(arr, ctypes.POINTER(L.MMTemplate))
            self._tmpl_keep.append(arr)
        self.precision = precision
        # the plan's device memory: one workspace from torch's allocator, sized by the library
        nbytes = ctypes.c_size_t(0)
        L.check(self._lib.mm_plan_workspace_size(ctypes.byref(d), ctypes.byref(nbytes)), self._lib)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=pix.device)
        h = ctypes.c_void_p()
        L.check(self._lib.mm_plan(ctypes.byref(d), _ptr(pix), _ptr(w), _ptr(self.workspace),
                                  ctypes.c_size_t(self.workspace.numel()), _stream(), ctypes.byref(h)), self._lib)
        self._h = h
        # (plan info waits for the plan's last counts: asked only when templates add amplitudes,
        # so that the caller can queue work behind an unfinished plan)
        self.n_tmpl = int(self.info()["n_tmpl"]) if self.templates else 0
        self._map_shape = (self.n_rhs, self.n_pix, self.n_stokes) if self.n_tmpl == 0 else \
            (self.n_rhs, self.n_pix * self.n_stokes + self.n_tmpl)

    # ------------------------------------------------------------------ lifecycle
    def close(self):
        """Destroy the plan (the library waits for the device) and release its workspace."""
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.mm_destroy(self._h)
            self._h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        i = L.MMPlanInfo()
        L.check(self._lib.mm_plan_get_info(self._h, ctypes.byref(i)), self._lib)
        return dict(n_obs=i.n_obs, n_valid=i.n_valid, n_f=i.n_f, n_chunks=i.n_chunks,
                    n_singular=i.n_singular, device_bytes=i.device_bytes, n_sliced=i.n_sliced,
                    n_tmpl=i.n_tmpl, fft_shape=i.fft_shape)

    def split(self, x: torch.Tensor):
        """(map view [n_rhs, n_pix, n_stokes], [amplitude views, one per template]) of a
        map-shaped tensor of this plan."""
        if self.n_tmpl == 0:
            return x, []
        n_map = self.n_pix * self.n_stokes
        out, pos = [], n_map
        for t in self.templates:
            n = int(t["n_amp"]) if t["kind"] == "onehot" else 32 * (len(t["seg_start"]) - 1)
            out.append(x[:, pos:pos + n])
            pos += n
        return x[:, :n_map].view(self.n_rhs, self.n_pix, self.n_stokes), out

    # ------------------------------------------------------------------ helpers
    def _map_like(self) -> torch.Tensor:
        return torch.empty(self._map_shape, dtype=torch.float64, device=self.pix.device)

    def _check_map(self, x: torch.Tensor):
        if not x.is_cuda or x.dtype != torch.float64 or not x.is_contiguous() or tuple(x.shape) != self._map_shape:
            raise ValueError(f"map must be a contiguous float64 CUDA tensor of shape {list(self._map_shape)}")

    def _check_tod(self, y: torch.Tensor):
        if not y.is_cuda or not y.is_contiguous() or tuple(y.shape) != (self.n_rhs, self.n_samples):
            raise ValueError(f"TOD must be contiguous CUDA [{self.n_rhs}, {self.n_samples}]")
        return _tod_dtype(y)

    # ------------------------------------------------------------------ operators
    def hits(self) -> torch.Tensor:
        h = torch.empty(self.n_pix, dtype=torch.int32, device=self.pix.device)
        L.check(self._lib.mm_hits(self._h, _ptr(h), _stream()), self._lib)
        return h

    def lags(self) -> np.ndarray:
        out = np.zeros((self.n_filters, self.n_c))
        L.check(self._lib.mm_filter_lags(self._h, out.ctypes.data_as(ctypes.c_void_p), _stream()), self._lib)
        return out

    def unpoint(self, x: torch.Tensor, dtype=torch.float64) -> torch.Tensor:
        self._check_map(x)
        y = torch.empty((self.n_rhs, self.n_samples), dtype=dtype, device=x.device)
        L.check(self._lib.mm_unpoint(self._h, _ptr(x), _ptr(y), _tod_dtype(y), _stream()), self._lib)
        return y

    def point(self, y: torch.Tensor) -> torch.Tensor:
        dt = self._check_tod(y)
        x = self._map_like()
        L.check(self._lib.mm_point(self._h, _ptr(y), dt, _ptr(x), _stream()), self._lib)
        return x

    def weight(self, y: torch.Tensor) -> torch.Tensor:
        dt = self._check_tod(y)
        out = torch.empty_like(y)
        L.check(self._lib.mm_weight(self._h, _ptr(y), _ptr(out), dt, _stream()), self._lib)
        return out

    def apply_A(self, x: torch.Tensor) -> torch.Tensor:
        self._check_map(x)
        y = self._map_like()
        L.check(self._lib.mm_apply_A(self._h, _ptr(x), _ptr(y), _stream()), self._lib)
        return y

    def rhs(self, tod: torch.Tensor) -> torch.Tensor:
        dt = self._check_tod(tod)
        b = self._map_like()
        L.check(self._lib.mm_rhs(self._h, _ptr(tod), dt, _ptr(b), _stream()), self._lib)
        return b

    def _solve_call(self, fn, rhs_args, tol, max_iter, fixed_iters, check_every, use_graph, true_residual,
                    x0, out, raise_on_notconv, refine, map_error=False):
        if x0 is not None:
            self._check_map(x0)
        x = out if out is not None else self._map_like()
        self._check_map(x)
        o = L.MMSolveOpts()
        self._lib.mm_solve_opts_default(ctypes.byref(o))
        o.tol, o.max_iter, o.fixed_iters = float(tol), int(max_iter), int(fixed_iters)
        o.check_every, o.use_graph, o.true_residual = int(check_every), int(bool(use_graph)), int(bool(true_residual))
        o.d_x0 = None if x0 is None else x0.data_ptr()
        o.refine = int(bool(refine))
        o.map_error = int(bool(map_error))
        R = self.n_rhs
        n_hist = (fixed_iters if fixed_iters > 0 else max_iter) + 1
        iters = (ctypes.c_int32 * R)()
        best = (ctypes.c_int32 * R)()
        best_rel = (ctypes.c_double * R)()
        true_rel = (ctypes.c_double * R)()
        merr = (ctypes.c_double * R)()
        hist = np.zeros((R, n_hist))
        inf = L.MMSolveInfo()
        inf.iters = ctypes.cast(iters, ctypes.POINTER(ctypes.c_int32))
        inf.best_iter = ctypes.cast(best, ctypes.POINTER(ctypes.c_int32))
        inf.best_rel_res = ctypes.cast(best_rel, ctypes.POINTER(ctypes.c_double))
        inf.true_rel_res = ctypes.cast(true_rel, ctypes.POINTER(ctypes.c_double))
        inf.history = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        inf.map_error = ctypes.cast(merr, ctypes.POINTER(ctypes.c_double))
        st = fn(self._h, *rhs_args, _ptr(x), ctypes.byref(o), ctypes.byref(inf), _stream())
        allow = () if raise_on_notconv else (L.MM_ENOTCONV,)
        L.check(st, self._lib, allow=allow)
        info = dict(status=L.STATUS_NAMES[st], iters=list(iters), best_iter=list(best),
                    best_rel_res=list(best_rel), true_rel_res=list(true_rel), history=hist,
                    map_error=list(merr))
        return x, info

    def solve(self, tod: torch.Tensor, tol: float = 1e-6, max_iter: int = 50, fixed_iters: int = 0,
              check_every: int = 8, use_graph: bool = True, true_residual: bool = False,
              x0: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
              raise_on_notconv: bool = False, refine: bool = True, map_error: bool = False):
        """PCG solve of H m = P^T N^-1 d; returns (map [n_rhs, n_pix, n_stokes], info dict).
        map_error: also estimate each map's distance to the exact float64 solution
        (info["map_error"])."""
        dt = self._check_tod(tod)
        return self._solve_call(self._lib.mm_solve, (_ptr(tod), dt), tol, max_iter, fixed_iters, check_every,
                                use_graph, true_residual, x0, out, raise_on_notconv, refine, map_error)

    def solve_rhs(self, b: torch.Tensor, tol: float = 1e-6, max_iter: int = 50, fixed_iters: int = 0,
                  check_every: int = 8, use_graph: bool = True, true_residual: bool = False,
                  x0: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                  raise_on_notconv: bool = False, refine: bool = True):
        """PCG solve of H x = b for a map right-hand side b [n_rhs, n_pix, n_stokes]."""
        self._check_map(b)
        return self._solve_call(self._lib.mm_solve_rhs, (_ptr(b),), tol, max_iter, fixed_iters, check_every,
                                use_graph, true_residual, x0, out, raise_on_notconv, refine)

    def noise_gradient(self, tod: torch.Tensor, m: torch.Tensor, lam: torch.Tensor) -> np.ndarray:
        """dL/d(sigma, f_knee, alpha) per filter, float64 array [n_filters, 3]: the sum over
        RHS of (P lam)^T (dN^-1/dtheta) (tod - P m), for the map m and the adjoint lam of a loss."""
        dt = self._check_tod(tod)
        self._check_map(m)
        self._check_map(lam)
        out = np.zeros((self.n_filters, 3))
        L.check(self._lib.mm_noise_gradient(self._h, _ptr(tod), dt, _ptr(m), _ptr(lam),
                                            out.ctypes.data_as(ctypes.c_void_p), _stream()), self._lib)
        return out
