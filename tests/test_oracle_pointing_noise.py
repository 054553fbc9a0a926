"""Pins of the oracle's pointing matrix and inverse-noise filter (CPU only).

Each check ties the oracle to something other than itself: values of the
paper's polarised-signal equation at hand-evaluated angles, brute-force
counting, the independently simulated signal of the input generator, a
numerical quadrature of the inverse power spectrum, a dense Toeplitz matrix,
and the response of N^-1 to a pure sinusoid.
"""

import math

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg

import synth
from oracle import noise, pointing


# ---------------------------------------------------------------- pointing

def test_hits_match_brute_force_count():
    rng = np.random.default_rng(0)
    pix = rng.integers(-1, 37, size=5000).astype(np.int32)
    h = pointing.hits(pix, 40)
    brute = [0] * 40
    for p in pix.tolist():
        if p >= 0:
            brute[p] += 1
    assert h.tolist() == brute


@pytest.mark.parametrize("alpha_deg, expect", [
    (0.0, (0.5, 0.0, 0.5)),      # sin 0 = 0, cos 0 = 1
    (45.0, (0.5, 0.5, 0.0)),     # 2a = 90 deg
    (90.0, (0.5, 0.0, -0.5)),    # 2a = 180 deg
    (135.0, (0.5, -0.5, 0.0)),   # 2a = 270 deg
])
def test_polarised_row_follows_the_formalism_equation(alpha_deg, expect):
    # zeta_t = 1/2 [i + q sin(2a) + u cos(2a)]  (Formalism section)
    a = math.radians(alpha_deg)
    w = np.array([[math.sin(2 * a), math.cos(2 * a)]], dtype=np.float32)
    A = pointing.pointing_matrix(np.array([2], np.int32), w, 4, 3).toarray()
    row = A[0, 6:9]
    assert np.allclose(row, expect, atol=1e-7)
    assert np.count_nonzero(np.abs(A[0]) > 1e-7) == np.count_nonzero(np.abs(expect) > 0)


def test_temperature_row_is_unit_and_excised_rows_are_zero():
    A = pointing.pointing_matrix(np.array([1, -1, 3], np.int32), None, 5, 1).toarray()
    assert A.tolist() == [[0, 1, 0, 0, 0], [0, 0, 0, 0, 0], [0, 0, 0, 1, 0]]


@pytest.mark.parametrize("ns", [1, 3])
def test_pointing_reproduces_the_generators_noiseless_signal(ns):
    prob = synth.make_custom(ns, grid=(8, 8), det_lens=(3000, 2000), noiseless=True)
    A = pointing.pointing_matrix(prob.pix, prob.w, prob.n_pix, ns)
    sig = A @ prob.sky.ravel()
    assert np.allclose(sig, prob.tod[0], rtol=0, atol=1e-12)


def test_uniform_angles_give_the_closed_form_block():
    # n equally spaced polarisation angles over [0, pi): sum a a^T = n/4 diag(1, 1/2, 1/2)
    n = 12
    ang = np.arange(n) * np.pi / n
    w = np.stack([np.sin(2 * ang), np.cos(2 * ang)], 1)
    A = pointing.pointing_matrix(np.zeros(n, np.int32), w, 1, 3).toarray()
    assert np.allclose(A.T @ A, n / 4 * np.diag([1.0, 0.5, 0.5]), atol=1e-12)


# ---------------------------------------------------------------- noise filter

def test_white_noise_lags_are_a_scaled_delta():
    f = noise.lags(64, 100.0, 1.7, 0.0, 1.5, L=1 << 12)
    assert abs(f[0] - 1 / 1.7 ** 2) < 1e-15
    assert np.max(np.abs(f[1:])) < 1e-15


@pytest.mark.parametrize("tau", [0, 1, 7, 60, 400])
def test_lags_match_quadrature_of_the_inverse_spectrum(tau):
    # f~(tau) = (1/f_s) int_{-f_s/2}^{f_s/2} cos(2 pi nu tau / f_s) / p(nu) d nu
    fs, sg, fk, al = 100.0, 1.3, 0.4, 1.5
    n_c = 1024
    f = noise.lags(n_c, fs, sg, fk, al)
    g = lambda nu: 1.0 / noise.psd(nu, sg, fk, al) if nu > 0 else 0.0
    if tau == 0:
        val, _ = scipy.integrate.quad(g, 0, fs / 2, limit=500, epsabs=1e-13, epsrel=1e-12,
                                      points=[fk])
    else:
        val, _ = scipy.integrate.quad(g, 0, fs / 2, weight="cos", wvar=2 * np.pi * tau / fs,
                                      limit=2000, epsabs=1e-13)
    expect = 2.0 * val / fs * (1 - tau / n_c)
    assert abs(f[tau] - expect) < 1e-8 * abs(f[0])


@pytest.mark.parametrize("sg,fk,al,n_c", [(1.0, 0.1, 1.5, 1024), (1.0, 0.2, 1.7, 8192),
                                          (0.6, 0.5, 2.0, 8192), (2.0, 0.05, 1.0, 256)])
def test_filter_symbol_is_positive(sg, fk, al, n_c):
    f = noise.lags(n_c, 100.0 if n_c == 1024 else 200.0, sg, fk, al)
    n = 1 << 18
    c = np.zeros(n)
    c[:n_c] = f
    c[n - n_c + 1:] = f[1:][::-1]
    sym = np.fft.rfft(c).real
    assert sym.min() > 0


def test_ninv_on_a_sinusoid_returns_the_inverse_power():
    # deep inside a long interval, N^-1 acts on cos(2 pi nu t / f_s) as multiplication by
    # its symbol, which approximates 1/p(nu) away from nu = 0 (Fejer smoothing of width f_s/n_c)
    fs, sg, fk, al, n_c = 100.0, 1.0, 0.1, 1.5, 1024
    f = noise.lags(n_c, fs, sg, fk, al)
    n = 20000
    t = np.arange(n)
    for nu, tol in ((0.5, 1e-2), (2.0, 2e-3), (11.0, 2e-3), (37.0, 2e-3)):
        y = np.cos(2 * np.pi * nu * t / fs)
        out = noise.apply_ninv(y, np.array([0, n]), np.array([0]), f[None, :])
        mid = slice(n_c, n - n_c)
        ratio = np.dot(out[mid], y[mid]) / np.dot(y[mid], y[mid])
        assert abs(ratio * noise.psd(nu, sg, fk, al) - 1) < tol, nu


@pytest.mark.parametrize("lens", [[1, 5, 63, 64, 65, 200], [257, 31, 33, 2], [700]])
def test_ninv_fft_equals_direct_equals_dense_toeplitz(lens):
    rng = np.random.default_rng(5)
    n_c = 64
    tabs = np.stack([noise.lags(n_c, 50.0, 1.0, 0.3, 1.2, L=1 << 14),
                     noise.lags(n_c, 50.0, 0.7, 1.0, 1.9, L=1 << 14)])
    iv = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    filt = np.arange(len(lens)) % 2
    y = rng.standard_normal(iv[-1])
    a = noise.apply_ninv(y, iv, filt, tabs)
    b = noise.apply_ninv_direct(y, iv, filt, tabs)
    # dense: one Toeplitz block per interval, first column [f(0), ..., f(n_c-1), 0, ...]
    blocks = []
    for k, n in enumerate(lens):
        col = np.zeros(n)
        m = min(n, n_c)
        col[:m] = tabs[filt[k]][:m]
        blocks.append(scipy.linalg.toeplitz(col))
    c = scipy.linalg.block_diag(*blocks) @ y
    assert np.allclose(a, c, rtol=0, atol=1e-13)
    assert np.allclose(b, c, rtol=0, atol=1e-13)


@pytest.mark.parametrize("n_c", [1, 16, 64])
def test_single_sample_ninv_matches_direct_and_dense_toeplitz(n_c):
    """apply_ninv_at (one output sample from the banded-Toeplitz definition) at every
    sample of ragged intervals, including lengths 1, 2, n_c - 1, n_c, n_c + 1 and an
    empty interval, against the direct convolution and the dense block-Toeplitz product."""
    rng = np.random.default_rng(11 + n_c)
    tabs = np.stack([noise.lags(n_c, 50.0, 1.0, 0.3, 1.2, L=1 << 12),
                     noise.lags(n_c, 50.0, 0.7, 1.0, 1.9, L=1 << 12)])
    lens = sorted({1, 2, max(n_c - 1, 1), n_c, n_c + 1, 3 * n_c + 5}) + [0, 7]
    iv = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    filt = np.arange(len(lens)) % 2
    y = rng.standard_normal(int(iv[-1]))
    direct = noise.apply_ninv_direct(y, iv, filt, tabs)
    blocks = []
    for k, n in enumerate(lens):
        col = np.zeros(n)
        m = min(n, n_c)
        col[:m] = tabs[filt[k]][:m]
        blocks.append(scipy.linalg.toeplitz(col) if n else np.zeros((0, 0)))
    dense = scipy.linalg.block_diag(*blocks) @ y
    at = np.empty_like(y)
    for b in range(len(lens)):
        a, e = int(iv[b]), int(iv[b + 1])
        for t in range(a, e):
            at[t] = noise.apply_ninv_at(lambda lo, hi: y[lo:hi], t, a, e, tabs[filt[b]])
    assert np.allclose(at, direct, rtol=0, atol=1e-13)
    assert np.allclose(at, dense, rtol=0, atol=1e-13)


def test_ninv_batches_rows_independently():
    rng = np.random.default_rng(6)
    f = noise.lags(32, 50.0, 1.0, 0.3, 1.2, L=1 << 12)[None, :]
    iv = np.array([0, 100, 250])
    y = rng.standard_normal((3, 250))
    out = noise.apply_ninv(y, iv, np.array([0, 0]), f)
    for r in range(3):
        assert np.allclose(out[r], noise.apply_ninv(y[r], iv, np.array([0, 0]), f))


def test_lag_derivatives_match_finite_differences():
    fs, sg, fk, al, n_c = 100.0, 1.2, 0.3, 1.4, 128
    L = 1 << 16
    d = noise.lag_derivatives(n_c, fs, sg, fk, al, L=L)
    h = 1e-5
    for name, idx in (("sigma", 0), ("f_knee", 1), ("alpha", 2)):
        pp = [sg, fk, al]
        pm = [sg, fk, al]
        pp[idx] += h
        pm[idx] -= h
        fd = (noise.lags(n_c, fs, *pp, L=L) - noise.lags(n_c, fs, *pm, L=L)) / (2 * h)
        assert np.allclose(d[name], fd, rtol=0, atol=1e-8 * np.max(np.abs(fd))), name
