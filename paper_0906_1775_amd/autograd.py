"""Differentiable map-making: a torch.autograd.Function around the PCG solve.

The map m = H^-1 P^T N^-1 d is linear in the TOD d, and H = P^T N^-1 P is
symmetric (Algorithm section of the MADmap paper), so for any loss L(m):
  lambda = H^-1 dL/dm                       (one more PCG solve, same operator)
  dL/dd  = N^-1 P lambda
  dL/dtheta = (P lambda)^T (dN^-1/dtheta) (d - P m)   for theta = sigma, f_knee, alpha.
Every operator runs in libmm; this module only wires the calls.
"""

from __future__ import annotations

import torch

from .mapmaker import MapMaker


class _MapSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, tod, params, plan: MapMaker, tol: float, max_iter: int):
        m, info = plan.solve(tod.detach().contiguous(), tol=tol, max_iter=max_iter)
        ctx.plan, ctx.tol, ctx.max_iter = plan, tol, max_iter
        ctx.save_for_backward(tod, m)
        ctx.info = info
        return m

    @staticmethod
    def backward(ctx, g):
        tod, m = ctx.saved_tensors
        plan = ctx.plan
        lam, _ = plan.solve_rhs(g.detach().to(torch.float64).contiguous(), tol=ctx.tol, max_iter=ctx.max_iter)
        grad_tod = grad_params = None
        if ctx.needs_input_grad[0]:
            u = plan.unpoint(lam, dtype=torch.float64)                    # P lambda
            grad_tod = plan.weight(u.to(tod.dtype))                       # N^-1 P lambda
        if ctx.needs_input_grad[1]:
            grad_params = torch.from_numpy(plan.noise_gradient(tod.detach().contiguous(), m, lam))
        return grad_tod, grad_params, None, None, None


def solve_map(tod: torch.Tensor, plan: MapMaker, params: torch.Tensor | None = None, tol: float = 1e-10,
              max_iter: int = 1000) -> torch.Tensor:
    """Differentiable maximum-likelihood map.

    tod: CUDA tensor [n_rhs, n_samples] (float32 or float64).
    params: optional CPU float64 tensor [n_filters, 3] = (sigma, f_knee, alpha); it must hold the
      parameters ``plan`` was built with and receives dL/d(sigma, f_knee, alpha) when it requires grad.
    Returns the map [n_rhs, n_pix, n_stokes] (float64, CUDA); for a plan with templates, the
    extended vector [n_rhs, n_pix * n_stokes + n_tmpl] (map values, then template amplitudes),
    the amplitudes being marginalised in the gradients.  The adjoint solve needs dL/dm in the
    range of H: with templates that make H singular (offsets against the temperature
    monopole), a loss must not depend on the degenerate direction.
    """
    if params is None:
        params = torch.zeros(plan.n_filters, 3, dtype=torch.float64)
    return _MapSolve.apply(tod, params, plan, tol, max_iter)
