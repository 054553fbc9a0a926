"""Operator parity: HIP library (through the C ABI) vs the FP64 CPU oracle.

Inputs are seeded synthetic problems shared bit-for-bit by both sides.  Sizes
span several overlap-save transforms per interval, ragged interval tails,
empty and length-1 intervals, excised samples, non-power-of-two n_c and
several forced FFT lengths.  Tolerances: float64 path <= 1e-12 of the
output's scale (rounding of O(n_c log n_f) operations); float32 filtering
<= 2e-6; hit counts bit-exact.
"""

import numpy as np
import pytest
import torch

import synth
from gpu_helpers import max_rel, oracle_for, plan_for, rel_err, tod_tensor

pytestmark = pytest.mark.gpu

L_K = 1 << 14


def prob_t(n_rhs=1):
    return synth.make_custom(
        1, grid=(16, 16), det_lens=(20000, 13001),
        interval_lens=[[1, 0, 5, 63, 64, 65, 9000, 10802], [13001]],
        filters=((1.0, 0.5, 1.5), (0.7, 1.2, 1.8)), det_filter=[0, 1], n_c=64, f_samp=20.0,
        n_rhs=n_rhs, seed=31)


def prob_tqu(n_rhs=1, tod_dtype=np.float64):
    p = synth.make_custom(
        3, grid=(12, 12), det_lens=(9000, 7000, 5000, 3000),
        interval_lens=[[4000, 5000], [7000], [1, 2, 997, 4000], [3000]],
        filters=((1.0, 0.3, 1.6), (1.4, 0.8, 1.2)), n_c=100, f_samp=20.0, n_rhs=n_rhs,
        tod_dtype=tod_dtype, seed=32)
    return p


def with_excised(p, frac=0.02, seed=5):
    rng = np.random.default_rng(seed)
    p.pix = p.pix.copy()
    p.pix[rng.random(p.pix.shape[0]) < frac] = -1
    return p


@pytest.fixture(scope="module")
def T():
    p = prob_t()
    return p, oracle_for(p, L_K)


@pytest.fixture(scope="module")
def TQU():
    p = with_excised(prob_tqu())
    return p, oracle_for(p, L_K)


@pytest.mark.parametrize("which", ["T", "TQU"])
def test_hits_bit_exact(which, T, TQU):
    p, o = T if which == "T" else TQU
    mm = plan_for(p, lag_dft_len=L_K)
    h = mm.hits().cpu().numpy()
    assert np.array_equal(h, o.hits.astype(np.int32))
    info = mm.info()
    assert info["n_obs"] == o.n_obs
    assert info["n_valid"] == int((p.pix >= 0).sum())


@pytest.mark.parametrize("which", ["T", "TQU"])
def test_lags_match_oracle(which, T, TQU):
    p, o = T if which == "T" else TQU
    mm = plan_for(p, lag_dft_len=L_K)
    assert max_rel(mm.lags(), o.lag_tab) < 1e-12


def test_lags_full_resolution_c1():
    p = synth.make_problem("c1")
    o = oracle_for(p)          # L_K = 2^20
    mm = plan_for(p)
    assert max_rel(mm.lags(), o.lag_tab) < 1e-12


@pytest.mark.parametrize("which", ["T", "TQU"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_unpoint_and_point(which, dtype, T, TQU):
    p, o = T if which == "T" else TQU
    mm = plan_for(p, lag_dft_len=L_K)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((1, p.n_pix, p.n_stokes))
    y = mm.unpoint(torch.from_numpy(x).cuda(), dtype=dtype).cpu().numpy()
    ref = o.apply_A(o.to_observed(x[0]))
    tol = 1e-15 if dtype == torch.float64 else 1e-6
    assert max_rel(y[0], ref) < tol
    yy = rng.standard_normal((1, p.n_samples))
    yt = torch.from_numpy(yy).to(dtype).cuda()
    xm = mm.point(yt).cpu().numpy()
    ref = o.to_global(o.apply_At(yt.cpu().double().numpy()[0]))
    assert max_rel(xm[0], ref) < (1e-13 if dtype == torch.float64 else 1e-6)


# 24,000 TQU samples on grids of 144, 256, 576 and 2304 pixels: about 167, 94, 42 and
# 10 hits per observed pixel, so the scatter reads the plain pixel-major layout
# (128 or more on average; a TOD this small is far below the plan's size bound for it)
# and the sliced one with 4, 2 and 1 wavefronts per slice
@pytest.mark.parametrize("grid", [(12, 12), (16, 16), (24, 24), (48, 48)])
@pytest.mark.parametrize("n_rhs", [1, 3])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_point_on_every_scatter_layout(grid, n_rhs, dtype):
    p = with_excised(synth.make_custom(
        3, grid=grid, det_lens=(9000, 7000, 5000, 3000),
        interval_lens=[[4000, 5000], [7000], [1, 2, 997, 4000], [3000]],
        filters=((1.0, 0.3, 1.6),), n_c=100, f_samp=20.0, n_rhs=n_rhs, seed=33))
    o = oracle_for(p, L_K)
    mm = plan_for(p, lag_dft_len=L_K)
    info = mm.info()
    assert (info["n_sliced"] == info["n_valid"]) == (info["n_valid"] >= 128 * info["n_obs"])
    yy = np.random.default_rng(12).standard_normal((n_rhs, p.n_samples))
    yt = torch.from_numpy(yy).to(dtype).cuda()
    xm = mm.point(yt).cpu().numpy()
    for r in range(n_rhs):
        ref = o.to_global(o.apply_At(yt[r].cpu().double().numpy()))
        assert max_rel(xm[r], ref) < (1e-13 if dtype == torch.float64 else 1e-6)


# Plans built again from the same pointing scatter bit-identically: the radix sort,
# the layouts and every summation order are fixed, so nothing depends on timing.  The
# 2^24-sample workload sorts 4,096 tiles in two 9-bit passes (pixel-major scatter);
# the small TQU problem is sorted in one pass.
@pytest.mark.parametrize("which", ["TQU", "c2"])
def test_plans_scatter_bit_identically(which, TQU):
    p = TQU[0] if which == "TQU" else synth.make_problem("c2")
    y = torch.from_numpy(np.random.default_rng(13).standard_normal((1, p.n_samples)).astype(np.float32)).cuda()
    outs = []
    for _ in range(3):
        mm = plan_for(p, n_rhs=1, precision="mixed", lag_dft_len=L_K if which == "TQU" else 0)
        outs.append(mm.point(y).cpu().numpy())
        mm.close()
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


# 2^20 pixels (21-bit keys: three 8-bit sort passes), 100,000 samples in a strip of the
# map, ~4 hits per observed pixel (sliced scatter, one wavefront per slice): P^T against
# the oracle, and bit-identical across plans
def test_point_wide_keys_parity_and_reproducible():
    p = with_excised(synth.make_custom(
        3, grid=(1024, 1024), det_lens=(60000, 40000), interval_lens=[[60000], [17, 39983]],
        filters=((1.0, 0.3, 1.6),), n_c=100, f_samp=20.0, n_rhs=1, seed=34))
    o = oracle_for(p, L_K)
    yy = np.random.default_rng(14).standard_normal((1, p.n_samples))
    for dtype, tol in ((torch.float64, 1e-13), (torch.float32, 1e-6)):
        yt = torch.from_numpy(yy).to(dtype).cuda()
        ref = o.to_global(o.apply_At(yt[0].cpu().double().numpy()))
        outs = []
        for _ in range(2):
            mm = plan_for(p, lag_dft_len=L_K)
            info = mm.info()
            outs.append(mm.point(yt).cpu().numpy())
            mm.close()
        assert info["n_sliced"] % 64 == 0 and info["n_sliced"] >= info["n_valid"]
        assert max_rel(outs[0][0], ref) < tol
        assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("which", ["T", "TQU"])
@pytest.mark.parametrize("n_f", [0, 256, 512, 2048])
def test_weight_fp64(which, n_f, T, TQU):
    p, o = T if which == "T" else TQU
    mm = plan_for(p, n_f=n_f, lag_dft_len=L_K)
    y = np.random.default_rng(8).standard_normal((1, p.n_samples))
    out = mm.weight(torch.from_numpy(y).cuda()).cpu().numpy()
    ref = o.apply_ninv(y[0])
    assert max_rel(out[0], ref) < 1e-12


@pytest.mark.parametrize("which", ["T", "TQU"])
@pytest.mark.parametrize("n_f", [0, 2048, 1 << 16])
def test_weight_mixed(which, n_f, T, TQU):
    p, o = T if which == "T" else TQU
    mm = plan_for(p, precision="mixed", lag_dft_len=L_K, n_f=n_f)
    y = np.random.default_rng(9).standard_normal((1, p.n_samples)).astype(np.float32)
    out = mm.weight(torch.from_numpy(y).cuda()).cpu().numpy()
    ref = o.apply_ninv(y[0].astype(np.float64))
    assert max_rel(out[0], ref) < 2e-6


@pytest.mark.parametrize("which", ["T", "TQU"])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 2e-6)])
def test_apply_A_and_rhs(which, precision, tol, T, TQU):
    p, o = T if which == "T" else TQU
    mm = plan_for(p, precision=precision, lag_dft_len=L_K)
    x = np.random.default_rng(10).standard_normal((1, p.n_pix, p.n_stokes))
    hx = mm.apply_A(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = o.to_global(o.apply_H(o.to_observed(x[0])))
    assert max_rel(hx[0], ref) < tol
    b = mm.rhs(tod_tensor(p)).cpu().numpy()
    refb = o.to_global(o.rhs(p.tod[0]))
    assert max_rel(b[0], refb) < tol


def test_multi_rhs_operators_match_single(T):
    p, _ = T
    x = np.random.default_rng(11).standard_normal((3, p.n_pix, 1))
    mm3 = plan_for(p, n_rhs=3, lag_dft_len=L_K)
    mm1 = plan_for(p, n_rhs=1, lag_dft_len=L_K)
    h3 = mm3.apply_A(torch.from_numpy(x).cuda()).cpu().numpy()
    for r in range(3):
        h1 = mm1.apply_A(torch.from_numpy(x[r:r + 1].copy()).cuda()).cpu().numpy()
        assert np.array_equal(h3[r], h1[0])


def test_operator_is_symmetric_and_positive(TQU):
    p, _ = TQU
    mm = plan_for(p, lag_dft_len=L_K)
    rng = np.random.default_rng(12)
    u = rng.standard_normal((1, p.n_pix, 3))
    v = rng.standard_normal((1, p.n_pix, 3))
    hits = mm.hits().cpu().numpy() > 0
    u[0, ~hits] = 0
    v[0, ~hits] = 0
    hu = mm.apply_A(torch.from_numpy(u).cuda()).cpu().numpy()
    hv = mm.apply_A(torch.from_numpy(v).cuda()).cpu().numpy()
    a, b = np.sum(u * hv), np.sum(v * hu)
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))
    assert np.sum(v * hv) > 0


def test_invalid_pixel_is_rejected():
    from paper_0906_1775_amd import MMError
    p = prob_t()
    p.pix = p.pix.copy()
    p.pix[17] = p.n_pix   # out of range
    with pytest.raises(MMError, match="EINVAL"):
        plan_for(p, lag_dft_len=L_K)


def test_forced_fft_length_beyond_chip_is_unsupported():
    from paper_0906_1775_amd import MMError
    p = prob_t()
    with pytest.raises(MMError, match="EUNSUPPORTED"):
        plan_for(p, n_f=1 << 20, lag_dft_len=L_K)


def test_explicit_lags_equal_parametric(T):
    p, o = T
    mm = plan_for(p, explicit_lags=o.lag_tab)
    y = np.random.default_rng(13).standard_normal((1, p.n_samples))
    out = mm.weight(torch.from_numpy(y).cuda()).cpu().numpy()
    assert max_rel(out[0], o.apply_ninv(y[0])) < 1e-12
