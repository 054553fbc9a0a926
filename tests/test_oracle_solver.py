"""Pins of the oracle's system, preconditioner, PCG and FFT-length rule (CPU only).

Pins: a dense direct solve of the dense system on tiny inputs; the white-noise
closed forms (binned average for T, per-pixel 3x3 solve for TQU) and one-step
convergence of the block-preconditioned iteration there; unbiasedness on
noiseless data; symmetry and positive definiteness of H; the monotone
H-norm error of conjugate gradients; the lowest-residual return rule; the
FFT-length rule against the continuous optimum and Appendix A.
"""

import math

import numpy as np
import pytest
import scipy.optimize

import synth
from oracle import Oracle, fftlen, noise


def tiny(ns, noiseless=False, white=False, seed=11):
    filters = ((1.0, 0.0, 1.5), (0.8, 0.0, 1.2)) if white else ((1.0, 0.6, 1.5), (0.8, 1.1, 1.2))
    if ns == 1:
        return synth.make_custom(1, grid=(6, 6), det_lens=(420, 333),
                                 interval_lens=[[150, 270], [1, 40, 292]], filters=filters,
                                 n_c=20, f_samp=20.0, noiseless=noiseless, seed=seed)
    return synth.make_custom(3, grid=(4, 4), det_lens=(500, 460, 380),
                             interval_lens=[[200, 300], [460], [17, 363]], filters=filters,
                             n_c=24, f_samp=20.0, noiseless=noiseless, seed=seed)


def oracle_for(prob, L=1 << 14):
    return Oracle.from_problem(prob, L_K=L)


@pytest.mark.parametrize("ns", [1, 3])
def test_pcg_matches_dense_direct_solve(ns):
    prob = tiny(ns)
    o = oracle_for(prob)
    H = o.dense_H()
    b = o.A.toarray().T @ o.dense_ninv() @ prob.tod[0]
    x_dense = np.linalg.solve(H, b)
    x, info = o.pcg(o.rhs(prob.tod[0]), tol=1e-14, max_iter=500)
    assert np.linalg.norm(x - x_dense) <= 1e-10 * np.linalg.norm(x_dense)
    assert info.converged
    # Implementation section: without rounding CG reaches the solution within n_z steps
    assert info.iters <= o.n_unknowns


@pytest.mark.parametrize("ns", [1, 3])
def test_H_is_symmetric_positive_definite_and_matches_dense(ns):
    prob = tiny(ns)
    o = oracle_for(prob)
    H = o.dense_H()
    assert np.allclose(H, H.T, atol=1e-12)
    assert np.linalg.eigvalsh(H).min() > 0
    rng = np.random.default_rng(1)
    u, v = rng.standard_normal((2, o.n_unknowns))
    assert np.allclose(o.apply_H(u), H @ u, atol=1e-12)
    assert abs(u @ o.apply_H(v) - v @ o.apply_H(u)) < 1e-10
    assert v @ o.apply_H(v) > 0


def test_white_noise_T_map_is_the_binned_average():
    prob = tiny(1, white=True)
    o = oracle_for(prob)
    m, info = o.solve(prob.tod[0], tol=1e-13, max_iter=50)
    # average of the samples in each pixel, weighted by the white weight 1/sigma^2 of their interval
    num = np.zeros(prob.n_pix)
    den = np.zeros(prob.n_pix)
    for b in range(prob.n_intervals):
        sg = prob.filter_params[prob.iv_filter[b], 0]
        for t in range(prob.iv_start[b], prob.iv_start[b + 1]):
            p = prob.pix[t]
            if p >= 0:
                num[p] += prob.tod[0, t] / sg ** 2
                den[p] += 1 / sg ** 2
    seen = den > 0
    assert np.allclose(m[seen, 0], num[seen] / den[seen], rtol=1e-12, atol=1e-12)
    assert np.all(m[~seen] == 0)
    assert info.iters == 1   # block preconditioner is the exact inverse


def test_white_noise_TQU_map_is_the_per_pixel_3x3_solve():
    prob = tiny(3, white=True)
    o = oracle_for(prob)
    m, info = o.solve(prob.tod[0], tol=1e-13, max_iter=50)
    blocks = np.zeros((prob.n_pix, 3, 3))
    rhs = np.zeros((prob.n_pix, 3))
    for b in range(prob.n_intervals):
        wgt = 1.0 / prob.filter_params[prob.iv_filter[b], 0] ** 2
        for t in range(prob.iv_start[b], prob.iv_start[b + 1]):
            p = prob.pix[t]
            if p < 0:
                continue
            a = 0.5 * np.array([1.0, float(prob.w[t, 0]), float(prob.w[t, 1])])
            blocks[p] += wgt * np.outer(a, a)
            rhs[p] += wgt * a * prob.tod[0, t]
    for p in range(prob.n_pix):
        if o.hits[p] > 0:
            assert np.allclose(m[p], np.linalg.solve(blocks[p], rhs[p]), rtol=1e-10, atol=1e-10)
    assert info.iters == 1


@pytest.mark.parametrize("ns", [1, 3])
def test_noiseless_data_recover_the_input_sky(ns):
    # unbiasedness: with d = A z exactly, m = H^-1 A^T N^-1 A z = z for any positive definite N
    prob = tiny(ns, noiseless=True)
    o = oracle_for(prob)
    m, info = o.solve(prob.tod[0], tol=1e-14, max_iter=500)
    seen = o.hits > 0
    assert np.allclose(m[seen], prob.sky[seen], rtol=0, atol=1e-10)


def test_H_norm_error_never_increases():
    prob = tiny(3)
    o = oracle_for(prob)
    b = o.rhs(prob.tod[0])
    H = o.dense_H()
    xs = np.linalg.solve(H, b)
    errs = []

    def cb(it, x, r):
        e = x - xs
        errs.append(e @ H @ e)
    o.pcg(b, fixed_iters=25, callback=cb)
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-9) + 1e-25 for i in range(len(errs) - 1))


def test_returns_the_lowest_residual_iterate():
    # Implementation section: the residual of CG need not decrease monotonically, and the
    # iterate with the lowest relative residual is returned.  An explicit SPD matrix with
    # eigenvalues spread over three decades gives a non-monotone history.
    prob = tiny(3)
    o = oracle_for(prob)
    n = o.n_unknowns
    rng = np.random.default_rng(0)
    ev = np.logspace(0, 3, n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    H = Q @ np.diag(ev) @ Q.T
    b = rng.standard_normal(n)
    seen = {}

    def cb(it, x, r):
        seen[it] = x.copy()
    x, info = o.pcg(b, fixed_iters=30, precond="none", apply_H=lambda v: H @ v, callback=cb)
    assert np.any(np.diff(info.history) > 0)
    k = int(np.argmin(info.history))
    assert 0 < k < 30
    assert info.best_iter == k
    assert np.array_equal(x, seen[k])
    assert info.best_rel_res == info.history[k]


def test_block_and_jacobi_agree_for_one_T_filter():
    # T pointing with one filter: A^T W^-1 A = f(0) A^T A, so the two preconditioners differ
    # by a constant factor and PCG produces the same iterates
    prob = synth.make_custom(1, grid=(6, 6), det_lens=(600,), interval_lens=[[250, 350]],
                             filters=((1.0, 0.6, 1.5),), n_c=20, f_samp=20.0)
    o = oracle_for(prob)
    b = o.rhs(prob.tod[0])
    xa, ia = o.pcg(b, fixed_iters=8, precond="block")
    xb, ib = o.pcg(b, fixed_iters=8, precond="jacobi")
    assert np.allclose(xa, xb, rtol=1e-10, atol=1e-12)
    assert np.allclose(ia.history, ib.history, rtol=1e-8)


def test_relative_residual_definition():
    prob = tiny(1)
    o = oracle_for(prob)
    b = o.rhs(prob.tod[0])
    xs = {}

    def cb(it, x, r):
        xs[it] = x.copy()
    _, info = o.pcg(b, fixed_iters=4, callback=cb)
    for it in range(1, 5):
        true = np.linalg.norm(b - o.apply_H(xs[it])) / np.linalg.norm(b)
        assert abs(true - info.history[it]) <= 1e-9 * max(true, 1e-12)


# ---------------------------------------------------------------- FFT length

def _golden_rows():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "fft_length_rule.txt")
    rows = []
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            rows.append(tuple(int(v) for v in line.split()))
    return rows


@pytest.mark.parametrize("nc,longest,nf", _golden_rows())
def test_fft_length_rule_golden_and_bracket(nc, longest, nf):
    assert fftlen.paper_fft_length(nc, longest) == nf
    assert nf & (nf - 1) == 0 and nf > 2 * nc
    start = 1 << max(0, (longest - 1).bit_length())
    assert nf <= max(start, nf)
    # continuous optimum n* solves n - 2 n_c (1 + ln n) = 0
    nstar = scipy.optimize.brentq(lambda n: n - 2 * nc * (1 + math.log(n)), 2 * nc + 1e-9, 1e12)
    if start >= nstar and nf > 4 * nc:
        assert nf / 2 < nstar <= nf


def test_fft_length_values_for_the_workloads():
    assert fftlen.paper_fft_length(1024, 65536) == 32768
    assert fftlen.paper_fft_length(8192, 1 << 20) == 262144
    assert fftlen.paper_fft_length(8192, 1 << 21) == 262144


@pytest.mark.parametrize("nc", [4, 64, 1024, 8192, 100000])
def test_appendix_a_critical_point_is_a_minimum(nc):
    nstar = scipy.optimize.brentq(lambda n: n - 2 * nc * (1 + math.log(n)), 2 * nc + 1e-9, 1e15)
    assert abs(fftlen.h_prime(nstar, nc)) < 1e-12 * fftlen.h(nstar, nc)
    assert fftlen.h_second(nstar, nc) > 0
    # h' and h'' against central differences of h
    for n in (nstar * 0.7, nstar, nstar * 1.6):
        e = n * 1e-5
        fd1 = (fftlen.h(n + e, nc) - fftlen.h(n - e, nc)) / (2 * e)
        fd2 = (fftlen.h(n + e, nc) - 2 * fftlen.h(n, nc) + fftlen.h(n - e, nc)) / (e * e)
        assert abs(fd1 - fftlen.h_prime(n, nc)) < 1e-6 * abs(fftlen.h(n, nc)) / n
        assert abs(fd2 - fftlen.h_second(n, nc)) < 1e-3 * abs(fftlen.h_second(n, nc)) + 1e-12
