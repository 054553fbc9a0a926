"""Template-extended pointing [P B] on the GPU against the oracle ("Using MADmap"
section, eqs. eDSN1, PmatExt, HWPmat).

Workloads: small TQU / T scans with ragged stationary intervals and 1/f noise
(n_c = 24), plus destriping offsets, ground-synchronous azimuth bins and the
32-column HWP block per detector segment; and a destriping run with white
noise (n_c = 1, the diagonal weighting path).  Map-shaped tensors are the
extended vector [map; amplitudes].

Checks: P x, P^T y, H x and b element by element (float64 1e-12, mixed 1e-5);
PCG iterates compared through their fitted TOD [P B] x (fixed iterations:
float64 1e-10; converged: float64 1e-7, mixed 1e-5), with the unknowns
themselves to 1e-8 at fixed iterations.  The
extended system is singular along the temperature-monopole / offset
direction and nearly singular along uniform Q, U against the 4w HWP harmonic
(exactly degenerate in real numbers; the float32 angles leave eigenvalues
~1e-14 of the preconditioned H), so rounding is amplified in those directions
of the unknowns while the fitted TOD, which the data determine, is not.  Also:
two right-hand sides; amplitudes no sample touches stay 0.
"""

import numpy as np
import pytest
import torch

import synth
from gpu_helpers import max_rel
from oracle import Oracle
from oracle import templates as tm
from synth import templates as st

pytestmark = pytest.mark.gpu


def _problem(n_stokes=3, n_c=24, filters=((1.0, 0.3, 1.5),), kinds=("offsets", "azimuth", "hwp"), n_rhs=1,
             extra_amp=0, seed=8):
    p = synth.make_custom(n_stokes, grid=(10, 10), det_lens=(2600, 2100), n_c=n_c, f_samp=20.0,
                          filters=filters, interval_lens=[[900, 1700], [2100]], seed=seed, n_rhs=n_rhs)
    p, ti = st.add_templates(p, offsets=300 if "offsets" in kinds else 0,
                             azimuth_bins=5 if "azimuth" in kinds else 0, hwp="hwp" in kinds,
                             amplitude=0.5, seed=seed)
    tl, dev = [], []
    if ti.offsets is not None:
        idx, n = ti.offsets
        tl.append(tm.OneHot(idx, n + extra_amp))
        dev.append(dict(kind="onehot", idx=torch.from_numpy(idx).cuda(), n_amp=n + extra_amp))
    if ti.azimuth is not None:
        idx, n = ti.azimuth
        idx = idx.copy()
        idx[::7] = -1                   # samples without a bin
        tl.append(tm.OneHot(idx, n))
        dev.append(dict(kind="onehot", idx=torch.from_numpy(idx).cuda(), n_amp=n))
    if ti.hwp is not None:
        om, seg = ti.hwp
        tl.append(tm.HWP(om, seg))
        dev.append(dict(kind="hwp", omega=torch.from_numpy(om).cuda(), seg_start=seg))
    o = Oracle.from_problem(p, templates=tl, L_K=1 << 12)
    return p, o, dev


def _plan(p, o, dev, precision="fp64", n_rhs=None):
    from paper_0906_1775_amd import MapMaker
    d = torch.device("cuda:0")
    w = None if p.w is None else torch.from_numpy(p.w).to(d)
    return MapMaker(torch.from_numpy(p.pix).to(d), w, p.n_pix, p.n_stokes, p.iv_start, p.iv_filter,
                    filter_lags=o.lag_tab, n_c=p.n_c, precision=precision,
                    n_rhs=p.n_rhs if n_rhs is None else n_rhs, templates=dev)


def _to_oracle(o, x):
    """GPU map-shaped row [n_pix * ns + n_tmpl] -> oracle unknowns."""
    x = np.asarray(x, dtype=np.float64)
    nm = o.n_pix * o.n_stokes
    return o.to_observed(x[:nm].reshape(o.n_pix, o.n_stokes), x[nm:])


def _to_gpu(o, xo):
    return np.concatenate([o.to_global(xo).ravel(), o.amplitudes(xo)])


def _random_ext(o, rng):
    xo = rng.standard_normal(o.n_unknowns)
    return _to_gpu(o, xo), xo


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
@pytest.mark.parametrize("n_stokes", [1, 3])
def test_template_operators_match_the_oracle(precision, tol, n_stokes):
    p, o, dev = _problem(n_stokes=n_stokes)
    mm = _plan(p, o, dev, precision)
    assert mm.n_tmpl == o.n_tmpl
    rng = np.random.default_rng(3)
    xg, xo = _random_ext(o, rng)
    x = torch.from_numpy(xg[None]).cuda()
    y = mm.unpoint(x).cpu().numpy()[0]
    assert max_rel(y, o.apply_A(xo)) <= tol
    v = rng.standard_normal(p.n_samples)
    pt = mm.point(torch.from_numpy(v[None]).cuda()).cpu().numpy()[0]
    assert max_rel(pt, _to_gpu(o, o.apply_At(v))) <= tol
    hx = mm.apply_A(x).cpu().numpy()[0]
    assert max_rel(hx, _to_gpu(o, o.apply_H(xo))) <= tol
    b = mm.rhs(torch.from_numpy(np.ascontiguousarray(p.tod)).cuda()).cpu().numpy()[0]
    assert max_rel(b, _to_gpu(o, o.rhs(p.tod[0]))) <= tol


def test_fixed_iterations_match_the_oracle_pcg():
    p, o, dev = _problem()
    mm = _plan(p, o, dev)
    m, info = mm.solve(torch.from_numpy(np.ascontiguousarray(p.tod)).cuda(), fixed_iters=10)
    xo, oinfo = o.pcg(o.rhs(p.tod[0]), fixed_iters=10)
    assert info["iters"][0] == 10
    _same_iterate(o, m.cpu().numpy()[0], xo)


def _same_iterate(o, x_gpu, xo):
    """Fitted TOD to 1e-10, the unknowns to 1e-8 (see the module docstring)."""
    assert max_rel(o.apply_A(_to_oracle(o, x_gpu)), o.apply_A(xo)) <= 1e-10
    assert max_rel(x_gpu, _to_gpu(o, xo)) <= 1e-8


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_converged_fit_matches_the_oracle(precision):
    p, o, dev = _problem()
    mm = _plan(p, o, dev, precision)
    m, info = mm.solve(torch.from_numpy(np.ascontiguousarray(p.tod)).cuda(), tol=1e-10, max_iter=2000)
    print(f"templates {precision}: {info['iters'][0]} iterations, true residual {info['true_rel_res'][0]:.3e}")
    assert info["status"] == "MM_OK"
    xo, oinfo = o.pcg(o.rhs(p.tod[0]), tol=1e-12, max_iter=5000)
    fit_gpu = o.apply_A(_to_oracle(o, m.cpu().numpy()[0]))
    fit_or = o.apply_A(xo)
    # mixed: float32 rounding enters the near-null directions, invisible to the residual
    # (lambda |v|) but not to the fit (sqrt(lambda) |v|); the mixed-path bound is 1e-5
    assert max_rel(fit_gpu, fit_or) <= (1e-7 if precision == "fp64" else 1e-5)


def test_destriping_with_white_noise_uses_no_transform():
    p, o, dev = _problem(n_stokes=1, n_c=1, filters=((1.3, 0.0, 1.0),), kinds=("offsets",))
    mm = _plan(p, o, dev)
    rng = np.random.default_rng(5)
    xg, xo = _random_ext(o, rng)
    hx = mm.apply_A(torch.from_numpy(xg[None]).cuda()).cpu().numpy()[0]
    assert max_rel(hx, _to_gpu(o, o.apply_H(xo))) <= 1e-12
    m, info = mm.solve(torch.from_numpy(np.ascontiguousarray(p.tod)).cuda(), fixed_iters=8)
    xr, _ = o.pcg(o.rhs(p.tod[0]), fixed_iters=8)
    _same_iterate(o, m.cpu().numpy()[0], xr)
    for dt in (torch.float64, torch.float32):
        y = torch.from_numpy(rng.standard_normal((1, p.n_samples))).cuda().to(dt)
        wy = mm.weight(y).double().cpu().numpy()[0]
        want = o.apply_ninv(y.double().cpu().numpy()[0])
        assert max_rel(wy, want) <= (1e-15 if dt == torch.float64 else 1e-7)


def test_two_right_hand_sides_and_untouched_amplitudes():
    p, o, dev = _problem(n_rhs=2, extra_amp=3)
    mm = _plan(p, o, dev)
    assert mm.n_tmpl == o.n_tmpl
    tod = torch.from_numpy(np.ascontiguousarray(p.tod)).cuda()
    b = mm.rhs(tod).cpu().numpy()
    for r in range(2):
        assert max_rel(b[r], _to_gpu(o, o.rhs(p.tod[r]))) <= 1e-12
    m, info = mm.solve(tod, fixed_iters=6)
    for r in range(2):
        xr, _ = o.pcg(o.rhs(p.tod[r]), fixed_iters=6)
        _same_iterate(o, m.cpu().numpy()[r], xr)
    _, amps = mm.split(m)
    assert torch.all(amps[0][:, -3:] == 0)      # offsets past the last used one
