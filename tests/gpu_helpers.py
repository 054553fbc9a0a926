"""Helpers shared by the GPU tests: build a library plan and an oracle from one synthetic problem."""

from __future__ import annotations

import numpy as np
import torch

from oracle import Oracle


def plan_for(prob, precision="fp64", precond="block", n_f=0, n_rhs=None, lag_dft_len=0,
             explicit_lags=None):
    from paper_0906_1775_amd import MapMaker
    dev = torch.device("cuda:0")
    pix = torch.from_numpy(prob.pix).to(dev)
    w = None if prob.w is None else torch.from_numpy(prob.w).to(dev)
    kw = dict(filter_params=None if explicit_lags is not None else prob.filter_params,
              filter_lags=explicit_lags)
    return MapMaker(pix, w, prob.n_pix, prob.n_stokes, prob.iv_start, prob.iv_filter,
                    f_samp=prob.f_samp, n_c=prob.n_c, n_f=n_f, lag_dft_len=lag_dft_len,
                    precision=precision, precond=precond,
                    n_rhs=prob.n_rhs if n_rhs is None else n_rhs, **kw)


def oracle_for(prob, L_K=None):
    kw = {} if L_K is None else dict(L_K=L_K)
    return Oracle.from_problem(prob, **kw)


def tod_tensor(prob, rows=None):
    t = prob.tod if rows is None else prob.tod[rows]
    return torch.from_numpy(np.ascontiguousarray(t)).to("cuda:0")


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def max_rel(a, b):
    """max |a - b| / max |b| (elementwise comparison scaled by the output's size)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    s = np.max(np.abs(b)) if b.size else 0.0
    return float(np.max(np.abs(a - b)) / (s if s > 0 else 1.0)) if b.size else 0.0
