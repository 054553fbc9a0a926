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


def sampled_AtNinv(fetch, hit_samples, n_stokes, iv_start, iv_filter, lag_tab, n_c, y_window):
    """(A^T N^-1 y)_p at a few pixels p, sample by sample from the oracle's definitions.

    fetch(lo, hi) -> (pix [hi-lo], w [hi-lo, 2] or None) as host arrays;
    hit_samples: sorted indices of the samples that fall in the chosen pixels;
    y_window(lo, hi, pix, rows) -> y[lo:hi] (float64) given that range's pixel
    indices and rows of A.  Every hit sample t adds a_t (N^-1 y)_t to its pixel,
    (N^-1 y)_t taking y on the 2 n_c - 1 samples around t inside t's interval.
    With y = A x this is (H x)_p; with y = d it is b_p.
    Returns {pixel: [n_stokes] float64}.
    """
    from oracle import noise, pointing
    hit_samples = np.asarray(hit_samples, dtype=np.int64)
    b_of = np.searchsorted(iv_start, hit_samples, side="right") - 1
    lo = np.maximum(iv_start[b_of], hit_samples - n_c + 1)
    hi = np.minimum(iv_start[b_of + 1], hit_samples + n_c)
    ranges = []                       # overlapping windows merged, each fetched once
    for a, e in zip(lo.tolist(), hi.tolist()):
        if ranges and a <= ranges[-1][1]:
            ranges[-1][1] = max(ranges[-1][1], e)
        else:
            ranges.append([a, e])
    out = {}
    for ra, re_ in ranges:
        pix, w = fetch(ra, re_)
        pix = np.asarray(pix)
        rows = pointing.row_weights(pix, w, n_stokes)
        y = np.asarray(y_window(ra, re_, pix, rows), dtype=np.float64)
        sel = (hit_samples >= ra) & (hit_samples < re_)
        for t, b in zip(hit_samples[sel].tolist(), b_of[sel].tolist()):
            a, e = int(iv_start[b]), int(iv_start[b + 1])
            z = noise.apply_ninv_at(lambda l, h: y[l - ra:h - ra], t, a, e, lag_tab[int(iv_filter[b])])
            p = int(pix[t - ra])
            out[p] = out.get(p, np.zeros(n_stokes)) + rows[t - ra] * z
    return out
