"""Inverse-noise weighting N^-1 (oracle; test infrastructure only).

Algorithm section: the noise power spectrum is p(f) = sigma^2 [1 + (f_k/f)^alpha].
Weighting section: for piecewise-stationary noise N^-1 is block diagonal with one
banded Toeplitz block per stationary interval,
    (N^-1)_{t,t'} = f(|t - t'|)  if |t - t'| < n_c  (same interval),  else 0.

The paper does not say how f is obtained from p.  Reading used here (and by
the library): f is the inverse correlation function -- the inverse discrete
Fourier transform of 1/p sampled on a fine grid of L_K = 2^20 frequencies
nu_j = j f_samp / L_K -- multiplied by the triangular (Bartlett) taper
(1 - tau/n_c) on 0 <= tau < n_c.  1/p at nu = 0 is its limit (0 when
f_knee > 0).  The taper makes the symbol of each Toeplitz block a
Fejer-smoothed copy of 1/p >= 0, so every block is positive definite.

N^-1 is applied by plain linear convolution of each interval with the
symmetric kernel [f(n_c-1) .. f(1), f(0), f(1) .. f(n_c-1)], zero outside the
interval.  ``apply_ninv`` does that convolution with a library FFT of the
whole interval (no chunking); ``apply_ninv_direct`` does it by direct
summation for small inputs.
"""

from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.signal

L_K_DEFAULT = 1 << 20


def psd(nu, sigma: float, f_knee: float, alpha: float):
    """p(nu) = sigma^2 (1 + (f_knee / nu)^alpha), the 1/f model of the Algorithm section."""
    nu = np.asarray(nu, dtype=np.float64)
    return sigma * sigma * (1.0 + (f_knee / nu) ** alpha)


def inverse_psd_grid(L: int, f_samp: float, sigma: float, f_knee: float, alpha: float) -> np.ndarray:
    """s_j = 1/p(nu_j) for j = 0 .. L/2, nu_j = j f_samp / L; s_0 is the nu -> 0 limit."""
    nu = np.arange(L // 2 + 1, dtype=np.float64) * (f_samp / L)
    s = np.empty_like(nu)
    s[1:] = 1.0 / psd(nu[1:], sigma, f_knee, alpha)
    s[0] = 0.0 if f_knee > 0 else 1.0 / (sigma * sigma)
    return s


def taper(n_c: int) -> np.ndarray:
    """Bartlett taper 1 - tau/n_c on tau = 0 .. n_c - 1."""
    return 1.0 - np.arange(n_c, dtype=np.float64) / n_c


def lags(n_c: int, f_samp: float, sigma: float, f_knee: float, alpha: float,
         L: int = L_K_DEFAULT) -> np.ndarray:
    """f(tau), tau = 0 .. n_c - 1: tapered inverse DFT of 1/p on L frequencies."""
    s = inverse_psd_grid(L, f_samp, sigma, f_knee, alpha)
    return np.fft.irfft(s, n=L)[:n_c] * taper(n_c)


def inverse_psd_grid_derivatives(L: int, f_samp: float, sigma: float, f_knee: float,
                                 alpha: float) -> dict:
    """d s_j / d theta for theta in (sigma, f_knee, alpha), j = 0 .. L/2.

    With x = (f_knee/nu)^alpha and s = 1/p:
      ds/dsigma = -2 s / sigma,
      ds/df_knee = -s^2 sigma^2 alpha x / f_knee,
      ds/dalpha = -s^2 sigma^2 x ln(f_knee / nu).
    The nu = 0 entry is a constant (0 or 1/sigma^2) in f_knee and alpha.
    """
    nu = np.arange(L // 2 + 1, dtype=np.float64) * (f_samp / L)
    s = inverse_psd_grid(L, f_samp, sigma, f_knee, alpha)
    out = {k: np.zeros_like(s) for k in ("sigma", "f_knee", "alpha")}
    out["sigma"] = -2.0 * s / sigma
    if f_knee > 0:
        x = (f_knee / nu[1:]) ** alpha
        s2 = s[1:] ** 2 * sigma * sigma
        out["f_knee"][1:] = -s2 * alpha * x / f_knee
        out["alpha"][1:] = -s2 * x * np.log(f_knee / nu[1:])
    return out


def lag_derivatives(n_c: int, f_samp: float, sigma: float, f_knee: float, alpha: float,
                    L: int = L_K_DEFAULT) -> dict:
    """d f(tau) / d theta for theta in (sigma, f_knee, alpha)."""
    ds = inverse_psd_grid_derivatives(L, f_samp, sigma, f_knee, alpha)
    tp = taper(n_c)
    return {k: np.fft.irfft(v, n=L)[:n_c] * tp for k, v in ds.items()}


def lag_table(filter_params: np.ndarray, f_samp: float, n_c: int, L: int = L_K_DEFAULT) -> np.ndarray:
    """Lags of every filter: array [n_filters, n_c]."""
    return np.stack([lags(n_c, f_samp, *map(float, fp), L=L) for fp in np.atleast_2d(filter_params)])


def symmetric_kernel(f: np.ndarray) -> np.ndarray:
    """[f(n_c-1) .. f(1), f(0), f(1) .. f(n_c-1)] (length 2 n_c - 1, centre at n_c - 1)."""
    return np.concatenate([f[:0:-1], f])


def _convolve_interval(y: np.ndarray, f: np.ndarray, direct: bool) -> np.ndarray:
    n = y.shape[-1]
    if n == 0:
        return np.zeros_like(y)
    k = symmetric_kernel(f)
    c = f.shape[0] - 1
    if direct:
        full = np.convolve(y, k, mode="full")
    else:
        full = scipy.signal.fftconvolve(y, k, mode="full")
    return full[c:c + n]


def apply_ninv(y: np.ndarray, iv_start: np.ndarray, iv_filter: np.ndarray, lag_tab: np.ndarray,
               direct: bool = False) -> np.ndarray:
    """(N^-1 y)_t = sum_{t' in interval(t), |t-t'| < n_c} f_b(|t - t'|) y_t'.

    ``y`` may carry leading batch dimensions ([..., n_t]); every row is filtered
    independently.
    """
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros_like(y)
    flat_in = y.reshape(-1, y.shape[-1])
    flat_out = out.reshape(-1, y.shape[-1])
    with scipy.fft.set_workers(-1):
        for b in range(iv_filter.shape[0]):
            a, e = int(iv_start[b]), int(iv_start[b + 1])
            f = lag_tab[int(iv_filter[b])]
            for r in range(flat_in.shape[0]):
                flat_out[r, a:e] = _convolve_interval(flat_in[r, a:e], f, direct)
    return out


def apply_ninv_direct(y, iv_start, iv_filter, lag_tab):
    """Same operator as ``apply_ninv`` by direct summation (small inputs)."""
    return apply_ninv(y, iv_start, iv_filter, lag_tab, direct=True)


def white_weights(iv_start: np.ndarray, iv_filter: np.ndarray, lag_tab: np.ndarray,
                  n_t: int) -> np.ndarray:
    """diag(N^-1): f_b(0) of the interval holding each sample (the W^-1 of MADpre)."""
    out = np.zeros(n_t)
    for b in range(iv_filter.shape[0]):
        out[int(iv_start[b]):int(iv_start[b + 1])] = lag_tab[int(iv_filter[b]), 0]
    return out


def apply_ninv_at(y_window, t: int, a: int, e: int, f: np.ndarray) -> float:
    """(N^-1 y)_t by the definition, for one sample t of the interval [a, e).

    ``y_window(lo, hi)`` returns y[lo:hi] (float64); only samples with
    |t' - t| < n_c inside the interval contribute, with weight f(|t' - t|).
    """
    n_c = f.shape[0]
    lo, hi = max(a, t - n_c + 1), min(e, t + n_c)
    ys = np.asarray(y_window(lo, hi), dtype=np.float64)
    return float(np.dot(f[np.abs(np.arange(lo, hi) - t)], ys))
