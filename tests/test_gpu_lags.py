"""The plan-free lag construction (mm_noise_lags) against the oracle's lags and their
parameter derivatives (Weighting section; the 1/f model of the Algorithm section),
and against the lags a plan built from the same parameters holds."""

import numpy as np
import pytest
import torch

from oracle import noise

pytestmark = pytest.mark.gpu

PARAMS = np.array([[1.0, 0.2, 1.7], [0.5, 0.05, 1.0], [2.0, 0.5, 2.0], [1.3, 0.0, 1.5]])


@pytest.mark.parametrize("n_c,L", [(8192, 1 << 20), (1024, 1 << 16), (37, 1 << 12), (1, 256)])
def test_lags_and_derivatives_match_the_oracle(n_c, L):
    from paper_0906_1775_amd import noise_lags
    fs = 200.0
    prm = torch.from_numpy(PARAMS).cuda()
    got = noise_lags(prm, fs, n_c, L).cpu().numpy()
    for k, fp in enumerate(PARAMS):
        want = noise.lags(n_c, fs, *fp, L=L)
        assert np.max(np.abs(got[k] - want)) <= 1e-12 * np.max(np.abs(want))
    for deriv, name in ((1, "sigma"), (2, "f_knee"), (3, "alpha")):
        got = noise_lags(prm, fs, n_c, L, deriv=deriv).cpu().numpy()
        for k, fp in enumerate(PARAMS):
            want = noise.lag_derivatives(n_c, fs, *fp, L=L)[name]
            scale = max(np.max(np.abs(want)), 1e-300)
            assert np.max(np.abs(got[k] - want)) <= 1e-11 * scale, (name, k)


def test_plan_lags_are_the_plan_free_lags():
    import synth
    from gpu_helpers import plan_for
    from paper_0906_1775_amd import noise_lags
    p = synth.make_custom(3, grid=(8, 8), det_lens=(3000, 2400), filters=((1.0, 0.3, 1.6), (0.8, 0.1, 1.2)),
                          n_c=64, f_samp=20.0, seed=4)
    mm = plan_for(p, lag_dft_len=1 << 14)
    free = noise_lags(torch.from_numpy(p.filter_params).cuda(), p.f_samp, p.n_c, 1 << 14).cpu().numpy()
    assert np.array_equal(mm.lags(), free)
