"""Pins of the oracle's map-loss gradients (CPU only).

Central finite differences of the oracle's own solve (a check of the adjoint
algebra, independent of it), the white-noise closed form dL/dd_t =
2 w_p m_p / hits_p, and the invariance of the map under a common rescaling
of N (dL/dsigma = 0 for one detector with one sigma).
"""

import numpy as np
import pytest

import synth
from oracle import Oracle, gradient


def small_t(white=False):
    fk = 0.0 if white else 0.8
    return synth.make_custom(1, grid=(8, 8), det_lens=(3000,), interval_lens=[[1200, 1800]],
                             filters=((1.0, fk, 1.5),), n_c=48, f_samp=20.0, seed=21)


def _loss_at(prob, d, lw, params, L=1 << 14):
    o = Oracle(prob.pix, prob.w, prob.n_pix, prob.n_stokes, prob.iv_start, prob.iv_filter,
               params, prob.f_samp, prob.n_c, L_K=L)
    return gradient.map_loss(o, d, lw, tol=1e-14, max_iter=3000)


def test_gradients_match_central_differences():
    prob = small_t()
    rng = np.random.default_rng(3)
    lw = rng.uniform(0.5, 1.5, (prob.n_pix, 1))
    o = Oracle.from_problem(prob, L_K=1 << 14)
    g = gradient.map_loss_gradients(o, prob.tod[0], lw, tol=1e-14, max_iter=3000)
    h = 1e-4
    # TOD direction with unit infinity norm
    v = rng.uniform(-1, 1, prob.n_samples)
    v /= np.max(np.abs(v))
    fp = _loss_at(prob, prob.tod[0] + h * v, lw, prob.filter_params)
    fm = _loss_at(prob, prob.tod[0] - h * v, lw, prob.filter_params)
    fd = (fp - fm) / (2 * h)
    assert abs(fd - g["grad_d"] @ v) <= 1e-6 * max(1.0, abs(fd))
    for name, idx in (("grad_f_knee", 1), ("grad_alpha", 2), ("grad_sigma", 0)):
        pp = prob.filter_params.copy()
        pm = prob.filter_params.copy()
        pp[0, idx] += h
        pm[0, idx] -= h
        fd = (_loss_at(prob, prob.tod[0], lw, pp) - _loss_at(prob, prob.tod[0], lw, pm)) / (2 * h)
        assert abs(fd - g[name][0]) <= 1e-5 * max(1.0, abs(fd)), (name, fd, g[name][0])


def test_white_noise_tod_gradient_closed_form():
    prob = small_t(white=True)
    lw = np.random.default_rng(4).uniform(0.5, 1.5, (prob.n_pix, 1))
    o = Oracle.from_problem(prob, L_K=1 << 14)
    g = gradient.map_loss_gradients(o, prob.tod[0], lw)
    m = g["map"][:, 0]
    ok = prob.pix >= 0
    p = prob.pix[ok]
    expect = np.zeros(prob.n_samples)
    expect[ok] = 2 * lw[p, 0] * m[p] / o.hits[p]
    assert np.allclose(g["grad_d"], expect, rtol=1e-10, atol=1e-12)


def test_sigma_gradient_vanishes_for_a_common_scale():
    prob = small_t()
    lw = np.ones((prob.n_pix, 1))
    o = Oracle.from_problem(prob, L_K=1 << 14)
    g = gradient.map_loss_gradients(o, prob.tod[0], lw)
    assert abs(g["grad_sigma"][0]) < 1e-8 * (abs(g["grad_f_knee"][0]) + abs(g["grad_alpha"][0]) + 1)
