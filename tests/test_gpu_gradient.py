"""Adjoint gradients (torch.autograd through the C ABI) vs the CPU oracle's
reference gradient and vs central finite differences of the GPU solve.

Workload: the config-4 problem (config-1 T-only scan, 65,536 samples, one
interval, n_c = 1024) with the map loss L = sum_p w_p m_p^2, w ~ U(0.5, 1.5).
Finite differences use step 1e-4 on f_knee and alpha and along a direction of
unit infinity norm in the TOD; inner solves run to 1e-13 so that solve error /
step stays far below the 1e-6 agreement asked of the gradient.
"""

import numpy as np
import pytest
import torch

import synth
from gpu_helpers import oracle_for, plan_for, rel_err, tod_tensor
from oracle import gradient

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C4():
    p = synth.make_problem("c4")
    o = oracle_for(p)
    ref = gradient.map_loss_gradients(o, p.tod[0], p.meta["loss_w"], tol=1e-13, max_iter=3000)
    return p, ref


def _loss_and_grads(p, params=None, tod=None, precision="fp64", n_f=0):
    from paper_0906_1775_amd import MapMaker, solve_map
    prm = p.filter_params if params is None else params
    dev = torch.device("cuda:0")
    mm = MapMaker(torch.from_numpy(p.pix).to(dev), None, p.n_pix, 1, p.iv_start, p.iv_filter,
                  filter_params=prm, f_samp=p.f_samp, n_c=p.n_c, precision=precision, n_f=n_f)
    d = (tod_tensor(p) if tod is None else tod).clone().requires_grad_(True)
    th = torch.tensor(prm, dtype=torch.float64, requires_grad=True)
    m = solve_map(d, mm, th, tol=1e-13, max_iter=3000)
    lw = torch.from_numpy(p.meta["loss_w"]).to(dev)[None]
    L = (lw * m * m).sum()
    L.backward()
    return float(L), d.grad.detach().cpu().numpy()[0], th.grad.numpy()[0]


@pytest.mark.parametrize("n_f", [0, 1 << 17])
def test_adjoint_matches_cpu_reference_gradient(C4, n_f):
    """n_f = 2^17: the float64 filter and its derivative symbols run through the
    four-step transform (symbols in row order)."""
    p, ref = C4
    L, gd, gth = _loss_and_grads(p, n_f=n_f)
    assert abs(L - ref["loss"]) <= 1e-10 * abs(ref["loss"])
    assert rel_err(gd, ref["grad_d"]) <= 1e-8
    assert abs(gth[1] - ref["grad_f_knee"][0]) <= 1e-7 * abs(ref["grad_f_knee"][0])
    assert abs(gth[2] - ref["grad_alpha"][0]) <= 1e-7 * abs(ref["grad_alpha"][0])
    # one detector, one sigma: the map does not change with a common rescaling of N
    assert abs(gth[0]) <= 1e-7 * (abs(gth[1]) + abs(gth[2]))
    assert abs(gth[0] - ref["grad_sigma"][0]) <= 1e-7 * (abs(gth[1]) + abs(gth[2]))


def test_adjoint_matches_central_differences(C4):
    p, _ = C4
    L0, gd, gth = _loss_and_grads(p)
    h = 1e-4
    for idx in (1, 2):
        pp = p.filter_params.copy()
        pm = p.filter_params.copy()
        pp[0, idx] += h
        pm[0, idx] -= h
        fd = (_loss_and_grads(p, params=pp)[0] - _loss_and_grads(p, params=pm)[0]) / (2 * h)
        print(f"theta[{idx}]: adjoint {gth[idx]:.9e} central difference {fd:.9e}")
        assert abs(fd - gth[idx]) <= 1e-6 * max(1.0, abs(fd))
    v = np.random.default_rng(17).uniform(-1, 1, p.n_samples)
    v /= np.abs(v).max()
    dv = torch.from_numpy(v[None]).cuda()
    base = tod_tensor(p)
    fd = (_loss_and_grads(p, tod=base + h * dv)[0] - _loss_and_grads(p, tod=base - h * dv)[0]) / (2 * h)
    print(f"TOD direction: adjoint {gd @ v:.9e} central difference {fd:.9e}")
    assert abs(fd - gd @ v) <= 1e-6 * max(1.0, abs(fd))


def test_mixed_precision_adjoint_float32_tod(C4):
    p, ref = C4
    t32 = tod_tensor(p).float()
    L, gd, gth = _loss_and_grads(p, tod=t32, precision="mixed")
    assert gd.dtype == np.float32
    # the oracle gradient of the float32-rounded TOD
    from oracle import Oracle
    o = Oracle.from_problem(p)
    r32 = gradient.map_loss_gradients(o, t32.cpu().numpy()[0].astype(np.float64), p.meta["loss_w"],
                                      tol=1e-13, max_iter=3000)
    assert rel_err(gd, r32["grad_d"]) <= 1e-5
    assert abs(gth[1] - r32["grad_f_knee"][0]) <= 1e-5 * abs(r32["grad_f_knee"][0])
    assert abs(gth[2] - r32["grad_alpha"][0]) <= 1e-5 * abs(r32["grad_alpha"][0])


def test_noise_gradient_needs_parameters():
    from paper_0906_1775_amd import MMError
    p = synth.make_custom(1, grid=(8, 8), det_lens=(3000,), n_c=32, f_samp=20.0, seed=3)
    o = oracle_for(p, 1 << 14)
    mm = plan_for(p, explicit_lags=o.lag_tab)
    u = tod_tensor(p)
    m = torch.zeros((1, p.n_pix, p.n_stokes), dtype=torch.float64, device="cuda:0")
    with pytest.raises(MMError, match="EUNSUPPORTED"):
        mm.noise_gradient(u, m, m)


def test_noise_gradient_sums_the_right_hand_sides(C4):
    """Two TOD rows in one plan: the library's dL/dtheta is the sum of the CPU reference
    gradients of the two maps (the loss is the sum of the per-map losses)."""
    from paper_0906_1775_amd import MapMaker, solve_map
    p, ref = C4
    dev = torch.device("cuda:0")
    d1 = np.roll(p.tod[0], 12345) * 0.7
    tods = np.stack([p.tod[0], d1])
    mm = MapMaker(torch.from_numpy(p.pix).to(dev), None, p.n_pix, 1, p.iv_start, p.iv_filter,
                  filter_params=p.filter_params, f_samp=p.f_samp, n_c=p.n_c, n_rhs=2)
    d = torch.from_numpy(tods).to(dev).requires_grad_(True)
    th = torch.tensor(p.filter_params, dtype=torch.float64, requires_grad=True)
    m = solve_map(d, mm, th, tol=1e-13, max_iter=3000)
    lw = torch.from_numpy(p.meta["loss_w"]).to(dev)[None]
    (lw * m * m).sum().backward()
    o = oracle_for(p)
    ref1 = gradient.map_loss_gradients(o, d1, p.meta["loss_w"], tol=1e-13, max_iter=3000)
    g = th.grad.numpy()[0]
    for k, name in ((1, "grad_f_knee"), (2, "grad_alpha")):
        want = ref[name][0] + ref1[name][0]
        assert abs(g[k] - want) <= 1e-7 * (abs(ref[name][0]) + abs(ref1[name][0]))
    gd = d.grad.detach().cpu().numpy()
    assert rel_err(gd[0], ref["grad_d"]) <= 1e-8
    assert rel_err(gd[1], ref1["grad_d"]) <= 1e-8
