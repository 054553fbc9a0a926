"""Pins of the template-extended oracle ("Using MADmap" section, eqs. eDSN1,
PmatExt and HWPmat) against closed forms and independent constructions.

* the HWP columns span the paper's parametric signal: a signal simulated by
  the generator from the sum over harmonics (time in seconds, its own
  coefficients) is fitted exactly by least squares on the oracle's columns;
* discrete orthogonality: with w_t = 2 pi t / P and whole turns per segment,
  the 16 untimed columns have Gram matrix (L/2) I;
* noiseless destriping and ground-bin recovery: d = A z + B y gives a
  solution whose fitted TOD equals d, whose polarisation maps equal the input
  and whose temperature map and amplitudes differ from the input by c and
  -g c for one constant c, g being the weight of I in a row of A (the
  monopole-amplitude degeneracy of the extended system);
* the PCG solution of a small 1/f problem with all three templates has the
  same fitted TOD as the least-squares solution of the whitened system
  L^T [A B] x = L^T d, with N^-1 = L L^T built entry by entry;
* with templates the extended H stays symmetric positive semi-definite.
"""

import numpy as np
import pytest

import synth
from oracle import Oracle
from oracle import templates as tm
from synth import templates as st


def _oracle(p, ti, **kw):
    tl = []
    if ti.offsets is not None:
        tl.append(tm.OneHot(*ti.offsets))
    if ti.azimuth is not None:
        tl.append(tm.OneHot(*ti.azimuth))
    if ti.hwp is not None:
        tl.append(tm.HWP(*ti.hwp))
    return Oracle.from_problem(p, templates=tl, **kw), tl


def test_hwp_columns_span_the_parametric_signal():
    lens = [3000, 2500]
    seg = np.array([0, 3000, 5500], dtype=np.int64)
    om = st.hwp_angle(lens, 2.0, 37.0)
    coef = np.random.default_rng(4).standard_normal((2, 32))
    coef[:, 8:16] *= 0.05
    coef[:, 24:32] *= 0.05
    psi = st.hwp_signal(om, seg, coef, 37.0)
    B = tm.hwp_block(tm.HWP(om, seg), 5500).toarray()
    y, *_ = np.linalg.lstsq(B, psi, rcond=None)
    assert np.linalg.norm(B @ y - psi) <= 1e-10 * np.linalg.norm(psi)


def test_hwp_untimed_columns_are_orthogonal_over_whole_turns():
    P, L = 64, 64 * 40
    om = (2.0 * np.pi * np.arange(L) / P).astype(np.float32)
    B = tm.hwp_block(tm.HWP(om, np.array([0, L])), L).toarray()
    C = B[:, list(range(8)) + list(range(16, 24))]
    G = C.T @ C
    # float32 angles: the closed form holds to their rounding
    assert np.allclose(G, (L / 2) * np.eye(16), atol=2e-3 * L)


def test_scaled_time_is_centred_and_bounded():
    tau = tm.scaled_time(np.array([0, 5, 5, 12]), 12)
    assert np.allclose(tau[:5], [-0.8, -0.4, 0.0, 0.4, 0.8])
    assert np.isclose(tau[5:].sum(), 0.0) and np.all(np.abs(tau) < 1)


def _noiseless(n_stokes, **tk):
    p = synth.make_custom(n_stokes, grid=(12, 12), det_lens=(5000, 4200), n_c=1,
                          filters=((1.0, 0.0, 1.0),), f_samp=50.0, noiseless=True, seed=21)
    return st.add_templates(p, amplitude=0.7, seed=5, **tk)


@pytest.mark.parametrize("n_stokes", [1, 3])
@pytest.mark.parametrize("kind", ["offsets", "azimuth"])
def test_noiseless_one_hot_recovery_up_to_the_monopole(n_stokes, kind):
    tk = dict(offsets=250) if kind == "offsets" else dict(azimuth_bins=6)
    p, ti = _noiseless(n_stokes, **tk)
    o, tl = _oracle(p, ti, L_K=1 << 12)
    x, info = o.pcg(o.rhs(p.tod[0]), tol=1e-13, max_iter=3000)
    assert info.converged
    fit = o.apply_A(x)
    assert np.abs(fit - p.tod[0]).max() <= 1e-9 * np.abs(p.tod[0]).max()
    m = o.to_global(x)
    obs = o.obs2glob
    dz = m[obs] - p.sky[obs]
    c = dz[:, 0].mean()
    assert np.abs(dz[:, 0] - c).max() <= 1e-8
    if n_stokes == 3:
        assert np.abs(dz[:, 1:]).max() <= 1e-8
    y = o.amplitudes(x)
    truth = ti.truth[kind]
    used = np.bincount(tl[0].idx[tl[0].idx >= 0], minlength=tl[0].n_amp) > 0
    g = 1.0 if n_stokes == 1 else 0.5          # weight of I in a row of A
    assert np.abs((y - truth)[used] + g * c).max() <= 1e-8
    assert np.all(y[~used] == 0)


def test_noiseless_hwp_signal_is_fitted_exactly():
    # The 4w harmonic is degenerate with a uniform Q/U map; the float32 rounding
    # of the polarisation pairs and of the HWP angles turns that exact null
    # direction into an eigenvalue ~1e-14 of the preconditioned H, along which
    # the fit settles at ~1e-8.  A wrong column set misfits by O(1).
    p, ti = _noiseless(3, hwp=True)
    o, _ = _oracle(p, ti, L_K=1 << 12)
    x, info = o.pcg(o.rhs(p.tod[0]), tol=1e-13, max_iter=3000)
    assert info.converged
    fit = o.apply_A(x)
    assert np.abs(fit - p.tod[0]).max() <= 1e-6 * np.abs(p.tod[0]).max()


def test_pcg_fit_matches_whitened_least_squares_with_all_templates():
    p = synth.make_custom(3, grid=(6, 6), det_lens=(700, 560), n_c=24, f_samp=20.0,
                          filters=((1.0, 0.05, 1.5),), interval_lens=[[300, 400], [560]], seed=8)
    p, ti = st.add_templates(p, offsets=90, azimuth_bins=4, hwp=True, amplitude=0.5, seed=2)
    o, _ = _oracle(p, ti, L_K=1 << 12)
    d = p.tod[0].astype(np.float64)
    Ad = o.A.toarray()
    Lc = np.linalg.cholesky(o.dense_ninv())        # N^-1 = L L^T, built entry by entry
    xw = np.linalg.lstsq(Lc.T @ Ad, Lc.T @ d, rcond=None)[0]
    x, info = o.pcg(o.rhs(d), tol=1e-13, max_iter=5000)
    assert info.converged
    assert np.abs(Ad @ x - Ad @ xw).max() <= 1e-7 * np.abs(Ad @ xw).max()


def test_extended_H_is_symmetric_positive_semidefinite():
    p = synth.make_custom(3, grid=(6, 6), det_lens=(600,), n_c=16, f_samp=20.0, seed=9)
    p, ti = st.add_templates(p, offsets=100, hwp=True, seed=3)
    o, _ = _oracle(p, ti, L_K=1 << 12)
    H = o.dense_H()
    assert np.allclose(H, H.T, atol=1e-12 * np.abs(H).max())
    ev = np.linalg.eigvalsh(0.5 * (H + H.T))
    assert ev.min() >= -1e-10 * ev.max()
    rng = np.random.default_rng(0)
    u, v = rng.standard_normal((2, o.n_unknowns))
    assert np.isclose(u @ o.apply_H(v), v @ o.apply_H(u), rtol=1e-12)
