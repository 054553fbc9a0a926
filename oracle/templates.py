"""Template-extended pointing [A B] (oracle; test infrastructure only).

Section "Using MADmap" (eqs. eDSN1 and PmatExt): a parasitic signal that is
linear in a few amplitudes y adds B y to the data model, d = A z + B y + n.
Appending B's columns to A and y to z gives a system of the same form as the
map-making system, solved by the same PCG.  The estimate vector is [z; y].

Kinds of B built here:

* one-hot templates -- signals synchronous with a binned parameter (case 1
  of that section) and destriping offsets (case 3).  Sample t carries an
  amplitude index idx_t (or -1 for none) and B[t, idx_t] = 1.
* the half-wave-plate parametric block (case 2, eq. HWPmat).  For every
  segment g of samples (for instance one detector's samples) there are 32
  columns, in this order for k = 1 .. 8:
      columns  0 ..  7: cos(k w_t)
      columns  8 .. 15: tau_t cos(k w_t)
      columns 16 .. 23: sin(k w_t)
      columns 24 .. 31: tau_t sin(k w_t)
  with w_t the polarizer angle of sample t.

Reading of the time factor: the paper multiplies by the time t.  Here
tau_t = (2 (t - s_g) - (L_g - 1)) / L_g, the sample index centred on segment
g = [s_g, s_g + L_g) and scaled to (-1, 1).  tau_t is an affine function of t
within a segment, so the span of {cos, tau cos, sin, tau sin} is the span of
the paper's columns: the fitted parasitic signal, and the map, are the same;
only the coefficients of the t-columns are rescaled and the constant columns
absorb the shift.

Amplitude layout: templates in the order given; a one-hot template holds
n_amp amplitudes (global ids 0 .. n_amp - 1); an HWP template holds 32 per
segment, segment-major.

Preconditioner for the amplitudes (the paper gives none): the diagonal of
B^T W^-1 B with W^-1 = diag(N^-1), inverted; zero where that diagonal is 0.
The pixel part keeps the block preconditioner of the Implementation section.
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

HWP_HARMONICS = 8
HWP_COLUMNS = 4 * HWP_HARMONICS


@dataclasses.dataclass
class OneHot:
    idx: np.ndarray                  # int32 [n_t]: amplitude of each sample, -1 = none
    n_amp: int

    @property
    def n_cols(self) -> int:
        return int(self.n_amp)


@dataclasses.dataclass
class HWP:
    omega: np.ndarray                # float32 [n_t]: polarizer angle (radians)
    seg_start: np.ndarray            # int64 [n_seg + 1]: segments tile [0, n_t)

    @property
    def n_seg(self) -> int:
        return int(np.asarray(self.seg_start).shape[0] - 1)

    @property
    def n_cols(self) -> int:
        return HWP_COLUMNS * self.n_seg


def scaled_time(seg_start: np.ndarray, n_t: int) -> np.ndarray:
    """tau_t for every sample (see the module docstring)."""
    seg_start = np.asarray(seg_start, dtype=np.int64)
    if seg_start[0] != 0 or seg_start[-1] != n_t or np.any(np.diff(seg_start) < 0):
        raise ValueError("HWP segments must tile [0, n_t)")
    tau = np.zeros(n_t)
    for g in range(seg_start.shape[0] - 1):
        a, e = int(seg_start[g]), int(seg_start[g + 1])
        L = e - a
        if L > 0:
            tau[a:e] = (2.0 * (np.arange(L, dtype=np.float64)) - (L - 1)) / L
    return tau


def hwp_block(t: HWP, n_t: int) -> sp.csr_matrix:
    """The HWP columns of eq. HWPmat for every segment: [n_t, 32 n_seg]."""
    om = np.asarray(t.omega, dtype=np.float64)
    tau = scaled_time(t.seg_start, n_t)
    seg = np.searchsorted(np.asarray(t.seg_start), np.arange(n_t), side="right") - 1
    k = np.arange(1, HWP_HARMONICS + 1, dtype=np.float64)
    ck = np.cos(om[:, None] * k[None, :])
    sk = np.sin(om[:, None] * k[None, :])
    vals = np.concatenate([ck, tau[:, None] * ck, sk, tau[:, None] * sk], axis=1)   # [n_t, 32]
    rows = np.repeat(np.arange(n_t), HWP_COLUMNS)
    cols = (HWP_COLUMNS * seg[:, None] + np.arange(HWP_COLUMNS)[None, :]).ravel()
    return sp.csr_matrix((vals.ravel(), (rows, cols)), shape=(n_t, t.n_cols))


def onehot_block(t: OneHot, n_t: int) -> sp.csr_matrix:
    idx = np.asarray(t.idx, dtype=np.int64)
    if idx.shape[0] != n_t or np.any(idx < -1) or np.any(idx >= t.n_amp):
        raise ValueError("one-hot index outside [-1, n_amp)")
    ok = idx >= 0
    rows = np.flatnonzero(ok)
    return sp.csr_matrix((np.ones(rows.shape[0]), (rows, idx[ok])), shape=(n_t, t.n_cols))


def template_matrix(templates: List, n_t: int) -> sp.csr_matrix:
    """B = [B_1 B_2 ...] for the templates in order: [n_t, sum of their columns]."""
    blocks = []
    for t in templates:
        if isinstance(t, OneHot):
            blocks.append(onehot_block(t, n_t))
        elif isinstance(t, HWP):
            blocks.append(hwp_block(t, n_t))
        else:
            raise TypeError(type(t))
    if not blocks:
        return sp.csr_matrix((n_t, 0))
    return sp.hstack(blocks).tocsr()


def amplitude_diagonal(B: sp.csr_matrix, wdiag: np.ndarray) -> np.ndarray:
    """diag(B^T W^-1 B) = sum_t f_b(t)(0) B[t, j]^2 for every amplitude j."""
    B2 = B.multiply(B)
    return np.asarray(B2.T @ wdiag).ravel()


def split(x: np.ndarray, n_map: int, templates: List) -> tuple:
    """[map part, [amplitudes of each template]] of an extended vector."""
    x = np.asarray(x)
    out, pos = [], n_map
    for t in templates:
        out.append(x[..., pos:pos + t.n_cols])
        pos += t.n_cols
    return x[..., :n_map], out


def total_columns(templates: Optional[List]) -> int:
    return int(sum(t.n_cols for t in templates)) if templates else 0
