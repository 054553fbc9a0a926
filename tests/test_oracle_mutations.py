"""Plant plausible mistakes in the oracle (on the CPU) and check that a pin catches each.

Every case patches one oracle function with a wrong variant (a dropped term, a
wrong sign, a swapped operand, an off-by-one) and re-runs one of the pin
tests, which must then fail.
"""

import numpy as np
import pytest

import oracle
from oracle import fftlen, noise, pointing, solver

import test_oracle_pointing_noise as pn
import test_oracle_solver as sv


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_swapped_q_u_weights_are_caught(monkeypatch):
    orig = pointing.row_weights

    def swapped(pix, w, ns):
        r = orig(pix, w, ns)
        if ns == 3:
            r = r[:, [0, 2, 1]]
        return r
    monkeypatch.setattr(pointing, "row_weights", swapped)
    _fails(pn.test_polarised_row_follows_the_formalism_equation, 45.0, (0.5, 0.5, 0.0))
    _fails(pn.test_pointing_reproduces_the_generators_noiseless_signal, 3)


def test_dropped_half_factor_is_caught(monkeypatch):
    orig = pointing.row_weights
    monkeypatch.setattr(pointing, "row_weights", lambda p, w, ns: orig(p, w, ns) * (2.0 if ns == 3 else 1.0))
    _fails(pn.test_uniform_angles_give_the_closed_form_block)


def test_missing_taper_is_caught(monkeypatch):
    monkeypatch.setattr(noise, "taper", lambda n_c: np.ones(n_c))
    _fails(pn.test_lags_match_quadrature_of_the_inverse_spectrum, 400)


def test_psd_instead_of_inverse_psd_is_caught(monkeypatch):
    orig = noise.inverse_psd_grid

    def wrong(L, fs, sg, fk, al):
        s = orig(L, fs, sg, fk, al)
        out = np.zeros_like(s)
        out[s > 0] = 1.0 / s[s > 0]
        return out
    monkeypatch.setattr(noise, "inverse_psd_grid", wrong)
    _fails(pn.test_ninv_on_a_sinusoid_returns_the_inverse_power)


def test_convolution_off_by_one_is_caught(monkeypatch):
    def shifted(y, f, direct):
        n = y.shape[-1]
        if n == 0:
            return np.zeros_like(y)
        k = noise.symmetric_kernel(f)
        full = np.convolve(y, k, mode="full")
        c = f.shape[0] - 2
        return full[c:c + n]
    monkeypatch.setattr(noise, "_convolve_interval", shifted)
    _fails(pn.test_ninv_fft_equals_direct_equals_dense_toeplitz, [257, 31, 33, 2])


def test_single_sample_window_off_by_one_is_caught(monkeypatch):
    def short_window(y_window, t, a, e, f):
        n_c = f.shape[0]
        lo, hi = max(a, t - n_c + 1), min(e, t + n_c - 1)
        ys = np.asarray(y_window(lo, hi), dtype=np.float64)
        return float(np.dot(f[np.abs(np.arange(lo, hi) - t)], ys))
    monkeypatch.setattr(noise, "apply_ninv_at", short_window)
    _fails(pn.test_single_sample_ninv_matches_direct_and_dense_toeplitz, 16)


def test_single_sample_wrong_interval_edge_is_caught(monkeypatch):
    orig = noise.apply_ninv_at
    monkeypatch.setattr(noise, "apply_ninv_at", lambda y_window, t, a, e, f: orig(y_window, t, max(a - 1, 0), e, f))
    _fails(pn.test_single_sample_ninv_matches_direct_and_dense_toeplitz, 16)


def test_pcg_beta_sign_error_is_caught(monkeypatch):
    def bad_pcg(self, b, tol=1e-6, max_iter=50, precond="block", **kw):
        M = self.preconditioner(precond)
        x = np.zeros_like(b)
        r = b.copy()
        z = M(r)
        p = z.copy()
        rho = r @ z
        for it in range(max_iter):
            q = self.apply_H(p)
            a = rho / (p @ q)
            x = x + a * p
            r = r - a * q
            if np.linalg.norm(r) <= tol * np.linalg.norm(b):
                break
            z = M(r)
            rho_new = r @ z
            p = z - (rho_new / rho) * p          # planted: wrong sign of beta
            rho = rho_new
        return x, solver.PCGInfo(it + 1, it + 1, 0.0, np.zeros(1), True)
    monkeypatch.setattr(solver.Oracle, "pcg", bad_pcg)
    _fails(sv.test_pcg_matches_dense_direct_solve, 3)


def test_unweighted_preconditioner_is_caught(monkeypatch):
    # dropping W^-1 from (A^T W^-1 A) breaks one-step convergence with two noise levels
    orig = noise.white_weights
    monkeypatch.setattr(noise, "white_weights", lambda *a: np.ones_like(orig(*a)))
    _fails(sv.test_white_noise_T_map_is_the_binned_average)


def test_wrong_h_prime_is_caught(monkeypatch):
    monkeypatch.setattr(fftlen, "h_prime",
                        lambda nf, nc: (1.0 + np.log(nf)) / (nf - 2.0 * nc))
    _fails(sv.test_appendix_a_critical_point_is_a_minimum, 1024)


def test_best_iterate_rule_is_caught(monkeypatch):
    orig = solver.Oracle.pcg

    def last_iterate(self, b, **kw):
        cb_x = {}
        user_cb = kw.pop("callback", None)

        def cb(it, x, r):
            cb_x["x"] = x.copy()
            if user_cb:
                user_cb(it, x, r)
        x, info = orig(self, b, callback=cb, **kw)
        info.best_iter = info.iters
        return cb_x.get("x", x), info
    monkeypatch.setattr(solver.Oracle, "pcg", last_iterate)
    _fails(sv.test_returns_the_lowest_residual_iterate)


# ---------------------------------------------------------------- templates
import scipy.sparse as sp

import test_oracle_templates as tt
from oracle import templates as otm


def test_hwp_harmonic_off_by_one_is_caught(monkeypatch):
    orig = otm.hwp_block

    def shifted(t, n_t):
        om = np.asarray(t.omega, dtype=np.float64)
        return orig(otm.HWP((om * 9.0 / 8.0).astype(np.float32), t.seg_start), n_t)
    monkeypatch.setattr(otm, "hwp_block", shifted)
    _fails(tt.test_hwp_columns_span_the_parametric_signal)


def test_hwp_missing_time_factor_is_caught(monkeypatch):
    monkeypatch.setattr(otm, "scaled_time", lambda seg, n_t: np.zeros(n_t))
    _fails(tt.test_hwp_columns_span_the_parametric_signal)


def test_hwp_sin_cos_swap_is_caught(monkeypatch):
    # a swap keeps the column span, so the span pin passes; the layout closed form catches it
    orig = otm.hwp_block

    def swapped(t, n_t):
        B = orig(t, n_t).tocsc()
        cols = np.array(list(range(16, 32)) + list(range(0, 16)))
        return sp.hstack([B[:, 32 * g + cols] for g in range(t.n_seg)]).tocsr()
    monkeypatch.setattr(otm, "hwp_block", swapped)
    _fails(_hwp_layout_check)


def _hwp_layout_check():
    """Columns 0..7 of a segment are cos(k w) (closed form at w = 0: all ones)."""
    om = np.zeros(4, dtype=np.float32)
    B = otm.hwp_block(otm.HWP(om, np.array([0, 4])), 4).toarray()
    assert np.allclose(B[:, :8], 1.0) and np.allclose(B[:, 16:24], 0.0)


def test_hwp_layout_check_passes_unmutated():
    _hwp_layout_check()


def test_one_hot_index_shift_is_caught(monkeypatch):
    orig = otm.onehot_block

    def shifted(t, n_t):
        idx = np.asarray(t.idx).copy()
        ok = idx >= 0
        idx[ok] = (idx[ok] + 1) % t.n_amp
        return orig(otm.OneHot(idx, t.n_amp), n_t)
    monkeypatch.setattr(otm, "onehot_block", shifted)
    _fails(tt.test_noiseless_one_hot_recovery_up_to_the_monopole, 1, "offsets")


def test_template_preconditioner_on_wrong_weights_is_caught(monkeypatch):
    # B^T B instead of B^T W^-1 B: caught by the closed form at sigma = 2
    monkeypatch.setattr(otm, "amplitude_diagonal", lambda B, w: np.asarray(B.multiply(B).sum(axis=0)).ravel())
    _fails(_template_precond_check)


def _template_precond_check():
    import synth
    from synth import templates as st
    p = synth.make_custom(1, grid=(6, 6), det_lens=(800,), n_c=1, filters=((2.0, 0.0, 1.0),),
                          f_samp=20.0, seed=4)
    p, ti = st.add_templates(p, offsets=100, seed=1)
    o, _ = tt._oracle(p, ti, L_K=1 << 12)
    # the diagonal of B^T W^-1 B is (number of samples) / sigma^2 for every offset
    M = o.preconditioner("block")
    r = np.zeros(o.n_unknowns)
    r[o.n_map:] = 1.0
    z = M(r)[o.n_map:]
    counts = np.bincount(ti.offsets[0], minlength=ti.offsets[1])
    assert np.allclose(z, 4.0 / counts)


def test_template_precond_check_passes_unmutated():
    _template_precond_check()
