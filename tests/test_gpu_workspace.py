"""Plans in a caller's workspace (mm_plan_workspace_size + mm_plan), through the C ABI.

* a plan built in a torch-allocated workspace gives bit-identical hits, operators and
  maps to one built in a workspace the library allocates (mm_plan_create);
* the bound from the descriptor holds for every kind of plan (precisions, Stokes,
  right-hand sides, templates, white noise, the autotuner, the four-step transform), and the workspace's
  contents on entry do not matter;
* the plan orders every call after its build, whatever the stream: a plan built on one
  side stream and used at once on another gives the same lags and maps.
"""

import ctypes

import numpy as np
import pytest
import torch

import synth
from gpu_helpers import oracle_for, rel_err, tod_tensor

pytestmark = pytest.mark.gpu

L_K = 1 << 14


def _lib():
    from paper_0906_1775_amd import _lib as L
    return L, L.load()


def _problem(n_stokes=3, **kw):
    args = dict(grid=(10, 10), det_lens=(3000, 2600), interval_lens=[[1800, 1200], [2600]],
                filters=((1.0, 0.4, 1.5), (0.8, 0.2, 1.8)), n_c=48, f_samp=20.0, seed=21)
    args.update(kw)
    return synth.make_custom(n_stokes, **args)


class _Desc:
    """An mm_desc_t of a synthetic problem (host arrays kept alive with it)."""

    def __init__(self, p, precision=0, n_rhs=None, n_f=0, templates=None):
        L, _ = _lib()
        self.iv = np.ascontiguousarray(p.iv_start, np.int64)
        self.fl = np.ascontiguousarray(p.iv_filter, np.int32)
        self.fp = np.ascontiguousarray(p.filter_params, np.float64)
        d = L.MMDesc()
        d.n_stokes, d.n_pix, d.n_samples, d.n_intervals = p.n_stokes, p.n_pix, p.n_samples, self.fl.shape[0]
        d.iv_start = self.iv.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        d.iv_filter = self.fl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.n_filters = self.fp.shape[0]
        d.filter_params = self.fp.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.f_samp, d.n_c, d.n_f, d.lag_dft_len = p.f_samp, p.n_c, n_f, L_K
        d.precision, d.n_rhs = precision, p.n_rhs if n_rhs is None else n_rhs
        self.arr = None
        if templates:
            self.arr = (L.MMTemplate * len(templates))(*templates)
            d.n_templates = len(templates)
            d.templates = ctypes.cast(self.arr, ctypes.POINTER(L.MMTemplate))
        self.d = d


def _ws_bytes(desc):
    L, lib = _lib()
    n = ctypes.c_size_t(0)
    L.check(lib.mm_plan_workspace_size(ctypes.byref(desc.d), ctypes.byref(n)), lib)
    return int(n.value)


def _plan(desc, pix, w, ws=None, stream=None):
    L, lib = _lib()
    h = ctypes.c_void_p()
    s = ctypes.c_void_p(0 if stream is None else stream.cuda_stream)
    wp = ctypes.c_void_p(0 if w is None else w.data_ptr())
    if ws is None:
        L.check(lib.mm_plan_create(ctypes.byref(desc.d), ctypes.c_void_p(pix.data_ptr()), wp, s, ctypes.byref(h)), lib)
    else:
        L.check(lib.mm_plan(ctypes.byref(desc.d), ctypes.c_void_p(pix.data_ptr()), wp, ctypes.c_void_p(ws.data_ptr()),
                            ctypes.c_size_t(ws.numel()), s, ctypes.byref(h)), lib)
    return h


def _info(h):
    L, lib = _lib()
    i = L.MMPlanInfo()
    L.check(lib.mm_plan_get_info(h, ctypes.byref(i)), lib)
    return i


def _solve(h, tod, R, n_map, fixed=6, stream=None, tol=1e-10):
    L, lib = _lib()
    x = torch.empty((R, n_map), dtype=torch.float64, device="cuda:0")
    o = L.MMSolveOpts()
    lib.mm_solve_opts_default(ctypes.byref(o))
    o.fixed_iters, o.tol, o.max_iter = fixed, tol, 200
    s = ctypes.c_void_p(0 if stream is None else stream.cuda_stream)
    dt = L.MM_F32 if tod.dtype == torch.float32 else L.MM_F64
    st = lib.mm_solve(h, ctypes.c_void_p(tod.data_ptr()), dt, ctypes.c_void_p(x.data_ptr()), ctypes.byref(o), None, s)
    L.check(st, lib, allow=(L.MM_ENOTCONV,))
    return x


def _hits(h, n_pix):
    L, lib = _lib()
    out = torch.empty(n_pix, dtype=torch.int32, device="cuda:0")
    L.check(lib.mm_hits(h, ctypes.c_void_p(out.data_ptr()), None), lib)
    return out


def _apply(h, x):
    L, lib = _lib()
    y = torch.empty_like(x)
    L.check(lib.mm_apply_A(h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), None), lib)
    return y


@pytest.mark.parametrize("precision", [0, 1])
def test_torch_workspace_plan_is_bit_identical_to_the_library_allocated_plan(precision):
    L, lib = _lib()
    p = _problem()
    desc = _Desc(p, precision=precision)
    pix = torch.from_numpy(p.pix).cuda()
    w = torch.from_numpy(p.w).cuda()
    tod = tod_tensor(p)
    n_map = p.n_pix * p.n_stokes
    a = _plan(desc, pix, w)
    ws = torch.empty(_ws_bytes(desc), dtype=torch.uint8, device="cuda:0")
    b = _plan(desc, pix, w, ws)
    try:
        assert torch.equal(_hits(a, p.n_pix), _hits(b, p.n_pix))
        x = torch.from_numpy(np.random.default_rng(3).standard_normal((p.n_rhs, n_map))).cuda()
        assert torch.equal(_apply(a, x), _apply(b, x))
        ma, mb = _solve(a, tod, p.n_rhs, n_map), _solve(b, tod, p.n_rhs, n_map)
        assert torch.equal(ma, mb)
        ma, mb = _solve(a, tod, p.n_rhs, n_map, fixed=0), _solve(b, tod, p.n_rhs, n_map, fixed=0)
        assert torch.equal(ma, mb)
        # and the map is the oracle's
        o = oracle_for(p, L_K)
        xo, _ = o.pcg(o.rhs(p.tod[0]), fixed_iters=6)
        mf = _solve(b, tod, p.n_rhs, n_map)
        tolr = 1e-10 if precision == 0 else 1e-5
        assert rel_err(mf.cpu().numpy()[0], o.to_global(xo).ravel()) <= tolr
        assert _info(b).device_bytes <= ws.numel()
    finally:
        lib.mm_destroy(a)
        lib.mm_destroy(b)


def _template_list(p):
    L, _ = _lib()
    rng = np.random.default_rng(5)
    idx = torch.from_numpy(rng.integers(-1, 7, p.n_samples).astype(np.int32)).cuda()
    om = torch.from_numpy(rng.uniform(0, 6.28, p.n_samples).astype(np.float32)).cuda()
    seg = np.array([0, 2000, p.n_samples], np.int64)
    t1 = L.MMTemplate()
    t1.kind, t1.n_amp, t1.d_idx = L.MM_TMPL_ONEHOT, 7, idx.data_ptr()
    t2 = L.MMTemplate()
    t2.kind, t2.n_seg, t2.d_omega = L.MM_TMPL_HWP, 2, om.data_ptr()
    t2.seg_start = seg.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    return [t1, t2], (idx, om, seg)


@pytest.mark.parametrize("case", ["t_fp64", "tqu_mixed_3rhs", "templates_mixed", "white", "autotune_fp64",
                                  "all_excised", "four_step_mixed", "four_step_fp64"])
def test_the_bound_holds_in_a_workspace_of_exactly_its_size(case):
    """Every plan kind builds and solves in a workspace of exactly mm_plan_workspace_size
    bytes, pre-filled with NaN bytes, and uses no more of it than the bound."""
    L, lib = _lib()
    keep = None
    kw = {}
    if case == "t_fp64":
        p, kw = _problem(1), dict(precision=0)
    elif case == "tqu_mixed_3rhs":
        p, kw = _problem(3, n_rhs=3), dict(precision=1)
    elif case == "templates_mixed":
        p = _problem(3)
        tl, keep = _template_list(p)
        kw = dict(precision=1, templates=tl)
    elif case == "white":
        p, kw = _problem(3, n_c=1), dict(precision=0)
    elif case == "autotune_fp64":
        p, kw = _problem(3, n_c=16), dict(precision=0, n_f=-1)
    elif case == "four_step_mixed":      # the batched four-step transform (2^16 complex points)
        p, kw = _problem(3, n_rhs=2), dict(precision=1, n_f=1 << 17)
    elif case == "four_step_fp64":       # 2^17 complex points in float64
        p, kw = _problem(3), dict(precision=0, n_f=1 << 18)
    else:
        p, kw = _problem(3), dict(precision=1)
        p.pix[:] = -1
    desc = _Desc(p, **kw)
    n = _ws_bytes(desc)
    ws = torch.full((n,), 0xFF, dtype=torch.uint8, device="cuda:0")
    pix = torch.from_numpy(p.pix).cuda()
    w = torch.from_numpy(p.w).cuda() if p.n_stokes == 3 else None
    h = _plan(desc, pix, w, ws)
    try:
        inf = _info(h)
        assert 0 < inf.device_bytes <= n
        n_map = p.n_pix * p.n_stokes + inf.n_tmpl
        x = _solve(h, tod_tensor(p), desc.d.n_rhs, n_map, fixed=4)
        assert torch.isfinite(x).all()
        # a second plan in a fresh workspace of the same bound gives the same map
        ws2 = torch.zeros((n,), dtype=torch.uint8, device="cuda:0")
        h2 = _plan(desc, pix, w, ws2)
        try:
            if case != "autotune_fp64":      # the tuner may time two shapes differently
                assert torch.equal(x, _solve(h2, tod_tensor(p), desc.d.n_rhs, n_map, fixed=4))
        finally:
            lib.mm_destroy(h2)
    finally:
        lib.mm_destroy(h)
    del keep


def test_calls_on_another_stream_wait_for_the_build():
    """Build on one side stream and, without any synchronisation, read the lags and solve
    on a second one: both see the finished build."""
    L, lib = _lib()
    p = _problem(3)
    desc = _Desc(p, precision=1)
    pix = torch.from_numpy(p.pix).cuda()
    w = torch.from_numpy(p.w).cuda()
    tod = tod_tensor(p)
    n_map = p.n_pix * p.n_stokes
    ref = _plan(desc, pix, w)
    torch.cuda.synchronize()
    want = _solve(ref, tod, p.n_rhs, n_map)
    lags_want = np.zeros((p.filter_params.shape[0], p.n_c))
    L.check(lib.mm_filter_lags(ref, lags_want.ctypes.data_as(ctypes.c_void_p), None), lib)
    lib.mm_destroy(ref)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ws = torch.empty(_ws_bytes(desc), dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    h = _plan(desc, pix, w, ws, stream=s1)
    try:
        lags = np.zeros_like(lags_want)
        L.check(lib.mm_filter_lags(h, lags.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(s2.cuda_stream)), lib)
        assert np.array_equal(lags, lags_want)
        got = _solve(h, tod, p.n_rhs, n_map, stream=s2)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
    finally:
        lib.mm_destroy(h)
