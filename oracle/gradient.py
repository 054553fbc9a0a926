"""Gradients of a quadratic map loss (oracle; test infrastructure only).

The map is m = H^-1 b with H = A^T N^-1 A, b = A^T N^-1 d (eq. pcgSystem).
For L = sum_p w_p m_p^2:
  * dL/dm = g = 2 w * m; H is symmetric (Algorithm section), so the adjoint
    of m = H^-1 b is lambda = H^-1 g;
  * dL/dd = N^-1 A lambda (N^-1 is symmetric);
  * for a parameter theta of N^-1: dm = H^-1 A^T dN^-1 (d - A m), hence
    dL/dtheta = (A lambda)^T (dN^-1/dtheta) (d - A m), where dN^-1/dtheta is
    the banded Toeplitz operator whose lags are df(tau)/dtheta, restricted to
    the intervals using that parameter's filter.
"""

from __future__ import annotations

import numpy as np

from . import noise
from .solver import Oracle


def map_loss(orc: Oracle, d: np.ndarray, loss_w: np.ndarray, **pcg_kw) -> float:
    """L(d) = sum_p w_p m_p^2 over observed pixels and Stokes."""
    x, _ = orc.pcg(orc.rhs(d), **pcg_kw)
    wo = orc.to_observed(loss_w)
    return float(np.sum(wo * x * x))


def map_loss_gradients(orc: Oracle, d: np.ndarray, loss_w: np.ndarray, tol: float = 1e-13,
                       max_iter: int = 2000, precond: str = "block") -> dict:
    """L, dL/dd and dL/d(sigma, f_knee, alpha) per filter, by one extra adjoint solve."""
    if orc.filter_params is None:
        raise ValueError("noise-parameter gradients need filter_params")
    d = np.asarray(d, dtype=np.float64)
    x, info = orc.pcg(orc.rhs(d), tol=tol, max_iter=max_iter, precond=precond)
    wo = orc.to_observed(loss_w)
    L = float(np.sum(wo * x * x))
    g = 2.0 * wo * x
    lam, info_adj = orc.pcg(g, tol=tol, max_iter=max_iter, precond=precond)
    a_lam = orc.apply_A(lam)
    grad_d = orc.apply_ninv(a_lam)
    resid = d - orc.apply_A(x)

    n_f = orc.filter_params.shape[0]
    grads = {k: np.zeros(n_f) for k in ("sigma", "f_knee", "alpha")}
    for k in range(n_f):
        sg, fk, al = map(float, orc.filter_params[k])
        dl = noise.lag_derivatives(orc.n_c, orc.f_samp, sg, fk, al, L=orc.L_K)
        sel = np.flatnonzero(orc.iv_filter == k)
        if sel.size == 0:
            continue
        for name in grads:
            tab = np.zeros((1, orc.n_c))
            tab[0] = dl[name]
            total = 0.0
            for b in sel:
                a, e = int(orc.iv_start[b]), int(orc.iv_start[b + 1])
                conv = noise.apply_ninv(resid[a:e], np.array([0, e - a]), np.array([0]), tab)
                total += float(a_lam[a:e] @ conv)
            grads[name][k] = total
    return dict(loss=L, map=orc.to_global(x), grad_d=grad_d, grad_sigma=grads["sigma"],
                grad_f_knee=grads["f_knee"], grad_alpha=grads["alpha"], lam=lam,
                iters=info.iters, iters_adjoint=info_adj.iters)
