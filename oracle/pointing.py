"""Pointing matrix A and hit counts (oracle; test infrastructure only).

Formalism section: the data model is gamma = nu + A z.  For a total-power
(temperature) detector the row of sample t has one unit weight in the column
of the pixel the detector points at; for an ideal polarisation-sensitive
detector the signal is zeta_t = (1/2)[i_p + q_p sin(2 a_t) + u_p cos(2 a_t)],
so the row holds the three weights (1/2, sin(2 a_t)/2, cos(2 a_t)/2) in the
(I, Q, U) columns of pixel p.  Algorithm section (gap filling): rows of
samples whose pixel was excised are zero; such samples carry index -1.

The polarisation input is the pair (sin 2a_t, cos 2a_t) per sample.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def hits(pix: np.ndarray, n_pix: int) -> np.ndarray:
    """Number of samples falling in each global pixel (excised samples skipped)."""
    ok = pix >= 0
    return np.bincount(pix[ok].astype(np.int64), minlength=n_pix).astype(np.int64)


def observed_pixels(pix: np.ndarray, n_pix: int) -> np.ndarray:
    """Sorted global ids of the pixels hit at least once (the observed index scheme)."""
    return np.flatnonzero(hits(pix, n_pix) > 0)


def row_weights(pix: np.ndarray, w, n_stokes: int) -> np.ndarray:
    """Non-zero values of each row of A: [n_t, n_stokes] (zero rows for pix = -1).

    T: 1.  TQU: (1/2, sin(2a)/2, cos(2a)/2), the weights of (I, Q, U).
    """
    ok = (np.asarray(pix) >= 0)[:, None]
    if n_stokes == 1:
        return np.where(ok, 1.0, 0.0)
    if n_stokes != 3:
        raise ValueError("n_stokes must be 1 or 3")
    s = np.asarray(w[:, 0], dtype=np.float64)
    c = np.asarray(w[:, 1], dtype=np.float64)
    return np.where(ok, 0.5 * np.stack([np.ones_like(s), s, c], axis=1), 0.0)


def pointing_matrix(pix: np.ndarray, w, n_pix: int, n_stokes: int,
                    obs2glob: np.ndarray | None = None) -> sp.csr_matrix:
    """A as a CSR matrix of shape (n_t, n_cols * n_stokes), float64.

    Columns are the observed pixels (in ``obs2glob`` order) when given, else
    all ``n_pix`` global pixels.  Column index = pixel * n_stokes + stokes.
    """
    n_t = pix.shape[0]
    pix = pix.astype(np.int64)
    ok = pix >= 0
    if obs2glob is not None:
        glob2obs = np.full(n_pix, -1, dtype=np.int64)
        glob2obs[obs2glob] = np.arange(obs2glob.shape[0])
        col_pix = np.where(ok, glob2obs[np.maximum(pix, 0)], -1)
        if np.any(ok & (col_pix < 0)):
            raise ValueError("a sample points at a pixel outside obs2glob")
        n_cols = obs2glob.shape[0]
    else:
        col_pix = pix
        n_cols = n_pix
    rows = np.flatnonzero(ok)
    vals = row_weights(pix, w, n_stokes)[ok]
    r = np.repeat(rows, n_stokes)
    cols = (n_stokes * col_pix[ok][:, None] + np.arange(n_stokes)[None, :]).ravel()
    return sp.csr_matrix((vals.ravel(), (r, cols)), shape=(n_t, n_cols * n_stokes))
