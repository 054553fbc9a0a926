"""The allocation-free lag construction (mm_noise_lags_noalloc, static device scratch)
against mm_noise_lags in a torch workspace, through the C ABI: bit-identical lags on two
calls in a row, the second with a smaller input; requests beyond its scratch rejected."""

import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _lib():
    from paper_0906_1775_amd import _lib as L
    return L, L.load()


def _with_workspace(prm, fs, n_c, L_K, deriv):
    L, lib = _lib()
    n = ctypes.c_size_t(0)
    L.check(lib.mm_noise_lags_workspace_size(n_c, L_K, ctypes.byref(n)), lib)
    ws = torch.empty(int(n.value), dtype=torch.uint8, device="cuda:0")
    out = torch.empty((prm.shape[0], n_c), dtype=torch.float64, device="cuda:0")
    L.check(lib.mm_noise_lags(ctypes.c_void_p(prm.data_ptr()), prm.shape[0], fs, n_c, L_K, deriv,
                              ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                              ctypes.c_size_t(ws.numel()), None), lib)
    torch.cuda.synchronize()
    return out


def _no_alloc(prm, fs, n_c, L_K, deriv):
    L, lib = _lib()
    out = torch.full((prm.shape[0], n_c), float("nan"), dtype=torch.float64, device="cuda:0")
    L.check(lib.mm_noise_lags_noalloc(ctypes.c_void_p(prm.data_ptr()), prm.shape[0], fs, n_c, L_K, deriv,
                                      ctypes.c_void_p(out.data_ptr()), None), lib)
    torch.cuda.synchronize()
    return out


def test_no_alloc_lags_equal_the_workspace_variant_on_two_calls():
    from oracle import noise
    rng = np.random.default_rng(8)
    big = np.column_stack([rng.uniform(0.5, 2, 6), rng.uniform(0.05, 0.5, 6), rng.uniform(1, 2, 6)])
    prm_big = torch.from_numpy(big).cuda()
    prm_small = torch.from_numpy(big[:2].copy()).cuda()
    # first call: 6 filters, n_c 8192, 2^20 frequencies (three filters per pass of the 64 MiB scratch)
    a = _no_alloc(prm_big, 200.0, 8192, 1 << 20, 0)
    b = _with_workspace(prm_big, 200.0, 8192, 1 << 20, 0)
    assert torch.equal(a, b)
    want = noise.lags(8192, 200.0, *big[4], L=1 << 20)
    assert np.max(np.abs(a.cpu().numpy()[4] - want)) <= 1e-12 * np.max(np.abs(want))
    # second call, smaller: 2 filters, n_c 1024, 2^16 frequencies, the f_knee derivative
    a2 = _no_alloc(prm_small, 100.0, 1024, 1 << 16, 2)
    b2 = _with_workspace(prm_small, 100.0, 1024, 1 << 16, 2)
    assert torch.equal(a2, b2)
    want2 = noise.lag_derivatives(1024, 100.0, *big[1], L=1 << 16)["f_knee"]
    assert np.max(np.abs(a2.cpu().numpy()[1] - want2)) <= 1e-11 * np.max(np.abs(want2))


def test_no_alloc_rejects_requests_beyond_its_scratch():
    L, lib = _lib()
    prm = torch.tensor([[1.0, 0.2, 1.7]], dtype=torch.float64, device="cuda:0")
    out = torch.empty((1, 8192), dtype=torch.float64, device="cuda:0")
    st = lib.mm_noise_lags_noalloc(ctypes.c_void_p(prm.data_ptr()), 1, 200.0, 8192, 1 << 23, 0,
                                   ctypes.c_void_p(out.data_ptr()), None)   # 128 MiB for one filter
    assert st == L.MM_EINVAL
    assert "64" in lib.mm_last_error().decode() or "above" in lib.mm_last_error().decode()
