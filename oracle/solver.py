"""Map-making system and PCG solve (oracle; test infrastructure only).

Algorithm section, eq. pcgSystem: the maximum-likelihood map x solves
H x = b with H = A^T N^-1 A and b = A^T N^-1 d (eq. eMLM gives x = H^-1 b).
The unknowns are the observed pixels only (Implementation section, observed
index scheme); unobserved pixels are reported as 0.

Implementation section:
  * preconditioner: MADpre's (A^T W^-1 A)^-1 with W^-1 = diag(N^-1) (block
    diagonal with one 1x1 or 3x3 block per pixel, because every row of A
    touches one pixel), or the default point-Jacobi diag(A^T A)^-1;
  * termination after n_i iterations or at relative residual epsilon
    (defaults 50 and 1e-6), returning the iterate with the lowest relative
    residual seen so far.

With templates ("Using MADmap" section, eq. PmatExt) the pointing matrix is
[A B] and the unknowns are [z; y]: the observed map followed by the template
amplitudes (``templates.py``).

The iteration is the textbook preconditioned conjugate gradient method the
paper cites (Barrett et al.; Shewchuk), in its usual order.  Relative
residual = ||r_k||_2 / ||b||_2 with r_k the recurrence residual.
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.sparse as sp

from . import noise, pointing
from . import templates as tmpl


@dataclasses.dataclass
class PCGInfo:
    iters: int                 # number of H applications performed
    best_iter: int             # iteration whose iterate is returned (0 = x0)
    best_rel_res: float
    history: np.ndarray        # relative residual after each iteration (index 0 = start)
    converged: bool


class Oracle:
    """Plain FP64 statement of the map-making operators for one workload."""

    def __init__(self, pix, w, n_pix, n_stokes, iv_start, iv_filter, filter_params=None,
                 f_samp=None, n_c=None, lag_tab=None, L_K: int = noise.L_K_DEFAULT, templates=None):
        self.n_pix = int(n_pix)
        self.n_stokes = int(n_stokes)
        self.n_t = int(pix.shape[0])
        self.iv_start = np.asarray(iv_start, dtype=np.int64)
        self.iv_filter = np.asarray(iv_filter, dtype=np.int32)
        if self.iv_start[0] != 0 or self.iv_start[-1] != self.n_t or np.any(np.diff(self.iv_start) < 0):
            raise ValueError("intervals must tile [0, n_t)")
        if lag_tab is None:
            lag_tab = noise.lag_table(filter_params, f_samp, n_c, L=L_K)
        self.lag_tab = np.asarray(lag_tab, dtype=np.float64)
        self.filter_params = None if filter_params is None else np.asarray(filter_params, np.float64)
        self.f_samp = f_samp
        self.n_c = self.lag_tab.shape[1]
        self.L_K = L_K
        self.pix = np.asarray(pix)
        self.w = None if w is None else np.asarray(w)
        self.hits = pointing.hits(self.pix, self.n_pix)
        self.obs2glob = np.flatnonzero(self.hits > 0)
        self.n_obs = int(self.obs2glob.shape[0])
        self.A_sky = pointing.pointing_matrix(self.pix, self.w, self.n_pix, self.n_stokes, self.obs2glob)
        self.templates = list(templates) if templates else []
        self.n_tmpl = tmpl.total_columns(self.templates)
        if self.templates:
            self.B = tmpl.template_matrix(self.templates, self.n_t)
            self.A = sp.hstack([self.A_sky, self.B]).tocsr()
        else:
            self.B = None
            self.A = self.A_sky
        self.At = self.A.T.tocsr()

    @classmethod
    def from_problem(cls, prob, **kw):
        return cls(prob.pix, prob.w, prob.n_pix, prob.n_stokes, prob.iv_start, prob.iv_filter,
                   prob.filter_params, prob.f_samp, prob.n_c, **kw)

    # ---- operators -------------------------------------------------------
    @property
    def n_unknowns(self) -> int:
        return self.n_obs * self.n_stokes + self.n_tmpl

    @property
    def n_map(self) -> int:
        return self.n_obs * self.n_stokes

    def apply_A(self, x: np.ndarray) -> np.ndarray:
        """Unpointing: map (observed layout) -> TOD."""
        return self.A @ x

    def apply_At(self, y: np.ndarray) -> np.ndarray:
        """Pointing: TOD -> map (observed layout)."""
        return self.At @ y

    def apply_ninv(self, y: np.ndarray, direct: bool = False) -> np.ndarray:
        return noise.apply_ninv(y, self.iv_start, self.iv_filter, self.lag_tab, direct=direct)

    def apply_H(self, x: np.ndarray) -> np.ndarray:
        """H x = A^T N^-1 A x."""
        return self.apply_At(self.apply_ninv(self.apply_A(x)))

    def rhs(self, d: np.ndarray) -> np.ndarray:
        """b = A^T N^-1 d."""
        return self.apply_At(self.apply_ninv(np.asarray(d, dtype=np.float64)))

    # ---- layouts ---------------------------------------------------------
    def to_global(self, x: np.ndarray) -> np.ndarray:
        """Observed-layout unknowns -> [n_pix, n_stokes] map with zeros elsewhere
        (the map part only; ``amplitudes`` returns the template part)."""
        out = np.zeros((self.n_pix, self.n_stokes))
        out[self.obs2glob] = np.asarray(x)[:self.n_map].reshape(self.n_obs, self.n_stokes)
        return out

    def amplitudes(self, x: np.ndarray) -> np.ndarray:
        """The template amplitudes of an unknown vector (all templates, in order)."""
        return np.asarray(x)[self.n_map:]

    def to_observed(self, m: np.ndarray, amps=None) -> np.ndarray:
        xm = np.asarray(m, dtype=np.float64).reshape(self.n_pix, self.n_stokes)[self.obs2glob].ravel()
        if self.n_tmpl == 0:
            return xm
        a = np.zeros(self.n_tmpl) if amps is None else np.asarray(amps, dtype=np.float64).ravel()
        return np.concatenate([xm, a])

    # ---- preconditioners -------------------------------------------------
    def precond_blocks(self) -> np.ndarray:
        """Blocks of A^T W^-1 A with W^-1 = diag(N^-1): array [n_obs, n_s, n_s].

        B_p = sum over samples t in pixel p of f_b(t)(0) a_t a_t^T, with a_t the
        non-zero weights of row t of A.
        """
        wdiag = noise.white_weights(self.iv_start, self.iv_filter, self.lag_tab, self.n_t)
        ok = self.pix >= 0
        glob2obs = np.full(self.n_pix, -1, dtype=np.int64)
        glob2obs[self.obs2glob] = np.arange(self.n_obs)
        p = glob2obs[self.pix[ok]]
        a = pointing.row_weights(self.pix, self.w, self.n_stokes)[ok]
        ns = self.n_stokes
        out = np.zeros((self.n_obs, ns, ns))
        for i in range(ns):
            for j in range(ns):
                out[:, i, j] = np.bincount(p, weights=wdiag[ok] * a[:, i] * a[:, j],
                                           minlength=self.n_obs)
        return out

    def preconditioner(self, kind: str = "block"):
        """Return M as a function r -> M r."""
        ns = self.n_stokes
        if kind == "none":
            return lambda r: r.copy()
        if kind == "jacobi":
            d = np.asarray((self.At @ self.A).diagonal())
            dinv = np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0)
            return lambda r: r * dinv
        if kind != "block":
            raise ValueError(kind)
        Minv = np.linalg.inv(self.precond_blocks())
        nm = self.n_map
        if self.n_tmpl:
            wdiag = noise.white_weights(self.iv_start, self.iv_filter, self.lag_tab, self.n_t)
            dg = tmpl.amplitude_diagonal(self.B, wdiag)
            dinv = np.where(dg > 0, 1.0 / np.where(dg > 0, dg, 1.0), 0.0)
        else:
            dinv = np.zeros(0)

        def apply(r):
            zm = np.einsum("pij,pj->pi", Minv, r[:nm].reshape(-1, ns)).ravel()
            return np.concatenate([zm, dinv * r[nm:]]) if self.n_tmpl else zm
        return apply

    # ---- solver ----------------------------------------------------------
    def pcg(self, b: np.ndarray, tol: float = 1e-6, max_iter: int = 50, precond: str = "block",
            x0: Optional[np.ndarray] = None, fixed_iters: Optional[int] = None,
            apply_H=None, callback=None):
        """Preconditioned CG on H x = b; returns (lowest-residual iterate, PCGInfo).

        ``fixed_iters`` runs exactly that many iterations (no tolerance test).
        """
        apply_H = apply_H or self.apply_H
        M = self.preconditioner(precond)
        b = np.asarray(b, dtype=np.float64)
        bnorm = np.linalg.norm(b)
        x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
        r = b - apply_H(x) if x0 is not None else b.copy()
        rel = np.linalg.norm(r) / bnorm if bnorm > 0 else 0.0
        hist = [rel]
        best_x, best_rel, best_it = x.copy(), rel, 0
        n_max = fixed_iters if fixed_iters is not None else max_iter
        if bnorm == 0 or (fixed_iters is None and rel <= tol):
            return best_x, PCGInfo(0, 0, rel, np.array(hist), True)
        z = M(r)
        p = z.copy()
        rho = r @ z
        converged = False
        it = 0
        for it in range(1, n_max + 1):
            q = apply_H(p)
            alpha = rho / (p @ q)
            x = x + alpha * p
            r = r - alpha * q
            rel = np.linalg.norm(r) / bnorm
            hist.append(rel)
            if callback is not None:
                callback(it, x, r)
            if rel < best_rel:
                best_x, best_rel, best_it = x.copy(), rel, it
            if fixed_iters is None and rel <= tol:
                converged = True
                break
            z = M(r)
            rho_new = r @ z
            beta = rho_new / rho
            p = z + beta * p
            rho = rho_new
        return best_x, PCGInfo(it, best_it, best_rel, np.array(hist), converged)

    def solve(self, d: np.ndarray, **kw):
        """Global [n_pix, n_stokes] map from TOD d, plus PCG info."""
        x, info = self.pcg(self.rhs(d), **kw)
        return self.to_global(x), info

    # ---- dense forms (tiny problems) ---------------------------------------
    def dense_ninv(self) -> np.ndarray:
        """N^-1 as a dense n_t x n_t matrix, built entry by entry from f(|t - t'|)."""
        out = np.zeros((self.n_t, self.n_t))
        for b in range(self.iv_filter.shape[0]):
            a, e = int(self.iv_start[b]), int(self.iv_start[b + 1])
            f = self.lag_tab[self.iv_filter[b]]
            for i in range(a, e):
                lo, hi = max(a, i - self.n_c + 1), min(e, i + self.n_c)
                out[i, lo:hi] = f[np.abs(np.arange(lo, hi) - i)]
        return out

    def dense_H(self) -> np.ndarray:
        Ad = self.A.toarray()
        return Ad.T @ self.dense_ninv() @ Ad
