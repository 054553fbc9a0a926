"""The two large workloads, generated on the device, against the oracle.

* Batched uneven intervals: 64 detectors x 2^22 samples (2^28), intervals
  log-uniform in [2^14, 2^21], 2^20 TQU pixels, per-detector noise.
* Large batch: 256 detectors x 2^22 samples (2^30), intervals log-uniform in
  [2^16, 2^22], 12 x 2048^2 TQU pixels, 8 noise realisations.

At full size the mixed-precision maps (float64 residual replacement, converged
to 1e-10) are also compared with the float64 GPU maps converged to 1e-10, whose
residual the oracle checks at sampled pixels (both workloads; 2 realisations
of the large batch).

Slices of each recipe (a few detectors) are small enough for the oracle's
full operators and PCG: hits bit-exact, H x and b element by element, and a
fixed-iteration solve.  At full size the oracle evaluates (H x)_p and b_p at a
few pixels sample by sample from the definitions (outputs it can compute one
by one), hits at those pixels are counted exactly, and the converged maps'
residual H m - b at those pixels is checked against the oracle's H and b.
"""

import gc

import numpy as np
import pytest
import torch

from gpu_helpers import max_rel, sampled_AtNinv
from oracle import Oracle
from oracle import noise as onoise

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-5}


def _gen(name, **kw):
    from synth.gpu import make_device_problem
    print(f"generating {name} {kw}", flush=True)
    # start from an empty cache: inputs carved out of an earlier test's cached segments
    # would pin those segments, and the plan's workspace (up to ~190 GiB) needs the rest
    gc.collect()
    torch.cuda.empty_cache()
    p = make_device_problem(name, device="cuda:0", **kw)
    torch.cuda.empty_cache()          # generation temporaries
    return p


def _plan(p, precision, n_f=0, fft_shape=0):
    from paper_0906_1775_amd import MapMaker
    return MapMaker(p.pix, p.w, p.n_pix, 3, p.iv_start, p.iv_filter, filter_params=p.filter_params,
                    f_samp=p.f_samp, n_c=p.n_c, n_f=n_f, precision=precision, n_rhs=p.n_rhs,
                    fft_shape=fft_shape)


def _host_oracle(p):
    return Oracle(p.pix.cpu().numpy(), p.w.cpu().numpy(), p.n_pix, 3, p.iv_start, p.iv_filter,
                  p.filter_params, p.f_samp, p.n_c)


def _random_map(n_rhs, n_pix, seed):
    g = torch.Generator(device="cuda:0")
    g.manual_seed(seed)
    return torch.randn((n_rhs, n_pix, 3), generator=g, device="cuda:0", dtype=torch.float64)


# ---------------------------------------------------------------- slices

SLICES = {
    "c3": dict(n_det=2, det_len=1 << 20),
    "c5": dict(n_det=8, det_len=1 << 20, n_rhs=2),
}


@pytest.fixture(scope="module", params=sorted(SLICES))
def slice_case(request):
    p = _gen(request.param, **SLICES[request.param])
    o = _host_oracle(p)
    assert o.n_obs > 1000
    tod = p.tod.double().cpu().numpy()
    b = np.stack([o.rhs(tod[r]) for r in range(p.n_rhs)])
    x = _random_map(p.n_rhs, p.n_pix, 11)
    xo = np.stack([o.to_observed(x[r].cpu().numpy()) for r in range(p.n_rhs)])
    hx = np.stack([o.to_global(o.apply_H(xo[r])) for r in range(p.n_rhs)])
    fixed = [o.to_global(o.pcg(b[r], fixed_iters=5)[0]) for r in range(p.n_rhs)]
    return request.param, p, o, dict(b=b, x=x, hx=hx, fixed=fixed)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_slice_operators_and_fixed_iterations(slice_case, precision):
    name, p, o, ref = slice_case
    print(f"{name} slice, {precision}", flush=True)
    mm = _plan(p, precision)
    assert np.array_equal(mm.hits().cpu().numpy(), o.hits.astype(np.int32))
    tol = TOL[precision]
    hx = mm.apply_A(ref["x"]).cpu().numpy()
    assert max_rel(hx, ref["hx"]) <= tol
    b = mm.rhs(p.tod).cpu().numpy()
    for r in range(p.n_rhs):
        assert max_rel(b[r], o.to_global(ref["b"][r])) <= tol
    m, info = mm.solve(p.tod, fixed_iters=5, refine=False)
    m = m.cpu().numpy()
    for r in range(p.n_rhs):
        err = max_rel(m[r], ref["fixed"][r])
        print(f"  5 fixed iterations, rhs {r}: max rel {err:.3e}", flush=True)
        assert err <= TOL[precision]


# ---------------------------------------------------------------- full size

def _pick_pixels(p, k, seed):
    """k distinct observed pixels chosen at seeded sample positions."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < k:
        t = int(rng.integers(0, p.n_samples))
        q = int(p.pix[t].item())
        if q >= 0 and q not in out:
            out.append(q)
    return np.asarray(sorted(out), dtype=np.int64)


def _fetch(p):
    def f(lo, hi):
        return p.pix[lo:hi].cpu().numpy(), p.w[lo:hi].cpu().numpy()
    return f


def _hit_samples(p, pixels):
    sel = torch.isin(p.pix, torch.from_numpy(pixels.astype(np.int32)).to(p.pix.device))
    return torch.nonzero(sel).flatten().cpu().numpy()


def _default_nf(p, precision):
    """The library's default FFT length for n_c = 8192 workloads: 2^15 (the smallest power of
    two above 2 n_c), or in float32 2^16 when its chunks, one 2^15-point workgroup each at
    2.25 times the work of a 2^14-point one, take fewer full rounds over the compute units."""
    assert p.n_c == 8192
    if precision == "fp64":
        return 1 << 15
    cu = torch.cuda.get_device_properties(0).multi_processor_count
    iv = np.asarray(p.iv_start, dtype=np.int64)
    lens = iv[1:] - iv[:-1]

    def rounds(nf):
        m = nf - 2 * p.n_c
        return -(-int(np.sum((lens + m - 1) // m)) * p.n_rhs // cu)
    return 1 << 16 if 2.25 * rounds(1 << 16) < rounds(1 << 15) else 1 << 15


def _check_full(p, precision, n_f=0):
    lag_tab = onoise.lag_table(p.filter_params, p.f_samp, p.n_c)
    pixels = _pick_pixels(p, 4, 5)
    ts = _hit_samples(p, pixels)
    mm = _plan(p, precision, n_f=n_f)
    print(f"{p.name} full: plan {mm.info()}", flush=True)
    if n_f == 0:
        assert mm.info()["n_f"] == _default_nf(p, precision)
    h = mm.hits()[torch.from_numpy(pixels).cuda()].cpu().numpy()
    assert np.array_equal(h, np.array([np.count_nonzero(p.pix[ts].cpu().numpy() == q) for q in pixels]))
    rs = sorted({0, p.n_rhs - 1})
    x = _random_map(p.n_rhs, p.n_pix, 13)
    hx = mm.apply_A(x)
    tol = TOL[precision]
    for r in rs:
        xr = x[r]
        ref = sampled_AtNinv(_fetch(p), ts, 3, p.iv_start, p.iv_filter, lag_tab, p.n_c,
                             lambda lo, hi, pix, rows: np.sum(
                                 rows * xr[torch.from_numpy(np.maximum(pix, 0)).cuda()].cpu().numpy(), axis=1))
        got = hx[r, torch.from_numpy(pixels).cuda()].cpu().numpy()
        want = np.stack([ref[int(q)] for q in pixels])
        print(f"  H x rhs {r}: max rel {max_rel(got, want):.3e}", flush=True)
        assert max_rel(got, want) <= tol
    del x, hx
    torch.cuda.empty_cache()
    # converged maps: oracle residual (H m - b) at the chosen pixels
    m, info = mm.solve(p.tod, tol=1e-8, max_iter=300)
    print(f"  solve {info['status']} iters {info['iters']} best {info['best_rel_res']}", flush=True)
    assert info["status"] == "MM_OK"
    for r in rs:
        mr = m[r]
        hm = sampled_AtNinv(_fetch(p), ts, 3, p.iv_start, p.iv_filter, lag_tab, p.n_c,
                            lambda lo, hi, pix, rows: np.sum(
                                rows * mr[torch.from_numpy(np.maximum(pix, 0)).cuda()].cpu().numpy(), axis=1))
        tod_r = p.tod[r]
        bb = sampled_AtNinv(_fetch(p), ts, 3, p.iv_start, p.iv_filter, lag_tab, p.n_c,
                            lambda lo, hi, pix, rows: tod_r[lo:hi].double().cpu().numpy())
        res = np.stack([hm[int(q)] - bb[int(q)] for q in pixels])
        bs = np.stack([bb[int(q)] for q in pixels])
        print(f"  residual at sampled pixels rhs {r}: {np.abs(res).max() / np.abs(bs).max():.3e}", flush=True)
        assert np.abs(res).max() <= 1e-6 * np.abs(bs).max()
    mm.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_uneven_full_size_sampled(precision):
    p = _gen("c3")
    assert p.n_samples == 1 << 28
    if precision == "mixed":
        assert _default_nf(p, precision) == 1 << 16   # 5,829 chunks against 16,779 at 2^15
    _check_full(p, precision)


def _sampled_residual(p, m, r, pixels, ts, lag_tab):
    """max |H m - b| / max |b| at the chosen pixels, from the oracle's definitions."""
    mr = m[r]
    hm = sampled_AtNinv(_fetch(p), ts, 3, p.iv_start, p.iv_filter, lag_tab, p.n_c,
                        lambda lo, hi, pix, rows: np.sum(
                            rows * mr[torch.from_numpy(np.maximum(pix, 0)).cuda()].cpu().numpy(), axis=1))
    tod_r = p.tod[r]
    bb = sampled_AtNinv(_fetch(p), ts, 3, p.iv_start, p.iv_filter, lag_tab, p.n_c,
                        lambda lo, hi, pix, rows: tod_r[lo:hi].double().cpu().numpy())
    res = np.stack([hm[int(q)] - bb[int(q)] for q in pixels])
    bs = np.stack([bb[int(q)] for q in pixels])
    return float(np.abs(res).max() / np.abs(bs).max())


@pytest.mark.parametrize("name,kw", [("c3", {}), ("c5", dict(n_rhs=2))])
def test_full_size_mixed_map_matches_the_fp64_map(name, kw):
    """Protocol (iii) at full size: the float64 GPU map, converged to 1e-10 and checked by the
    oracle's residual at sampled pixels, against the mixed-precision map with float64
    residual replacement converged to 1e-10: within 1e-5, in norm and element by element."""
    p = _gen(name, **kw)
    lag_tab = onoise.lag_table(p.filter_params, p.f_samp, p.n_c)
    pixels = _pick_pixels(p, 4, 7)
    ts = _hit_samples(p, pixels)
    mm = _plan(p, "fp64")
    m64, info = mm.solve(p.tod, tol=1e-10, max_iter=1000)
    print(f"{name} fp64: {info['status']} iters {info['iters']}", flush=True)
    assert info["status"] == "MM_OK"
    mm.close()
    del mm
    for r in range(p.n_rhs):
        res = _sampled_residual(p, m64, r, pixels, ts, lag_tab)
        print(f"  fp64 residual at sampled pixels, rhs {r}: {res:.3e}", flush=True)
        assert res <= 1e-8
    mx = _plan(p, "mixed")
    m32, info = mx.solve(p.tod, tol=1e-10, max_iter=1000, map_error=True)
    print(f"{name} mixed: {info['status']} iters {info['iters']} map error estimate {info['map_error']}",
          flush=True)
    assert info["status"] == "MM_OK"
    mx.close()
    for r in range(p.n_rhs):
        norm = float(torch.linalg.norm(m32[r] - m64[r]) / torch.linalg.norm(m64[r]))
        elem = float((m32[r] - m64[r]).abs().max() / m64[r].abs().max())
        print(f"  mixed vs fp64, rhs {r}: norm {norm:.3e}, max element {elem:.3e}", flush=True)
        assert norm <= 1e-5 and elem <= 1e-5
        assert info["map_error"][r] <= 1e-5


def test_large_batch_full_size_sampled():
    p = _gen("c5")
    assert p.n_samples == 1 << 30 and p.n_rhs == 8
    assert _default_nf(p, "mixed") == 1 << 16
    _check_full(p, "mixed")


# ---------------------------------------------------------------- autotuner

@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotuned_transform_length(precision):
    """n_f = -1 times every admissible length; operators match the oracle whatever it picks."""
    p = _gen("c3", n_det=2, det_len=1 << 18)
    o = _host_oracle(p)
    mm = _plan(p, precision, n_f=-1)
    nf = mm.info()["n_f"]
    assert nf & (nf - 1) == 0 and nf > 2 * p.n_c
    assert mm.info()["fft_shape"] in (tuple(range(1, 11)) if precision == "mixed" else (1, 3, 6, 8))
    x = _random_map(1, p.n_pix, 17)
    hx = mm.apply_A(x).cpu().numpy()[0]
    want = o.to_global(o.apply_H(o.to_observed(x[0].cpu().numpy())))
    assert max_rel(hx, want) <= TOL[precision]


@pytest.mark.parametrize("n_f,shape", [(32768, s) for s in range(1, 11)] + [(65536, 1), (65536, 2), (65536, 3),
                                                                          (65536, 10)])
def test_forced_transform_shapes_match_the_oracle(n_f, shape):
    """Each workgroup shape of the float32 transforms of 2^14 and 2^15 complex points
    gives the oracle's H x; float64 plans use the shapes that exist in float64 (1, 3, 6, 8)
    and fall back to shape 1 otherwise."""
    p = _gen("c3", n_det=2, det_len=1 << 18)
    o = _host_oracle(p)
    mm = _plan(p, "mixed", n_f=n_f, fft_shape=shape)
    assert mm.info()["fft_shape"] == shape and mm.info()["n_f"] == n_f
    x = _random_map(1, p.n_pix, 19)
    hx = mm.apply_A(x).cpu().numpy()[0]
    want = o.to_global(o.apply_H(o.to_observed(x[0].cpu().numpy())))
    assert max_rel(hx, want) <= TOL["mixed"]
    y = p.tod[:1].contiguous()
    wy = mm.weight(y).double().cpu().numpy()[0]
    assert max_rel(wy, o.apply_ninv(y.double().cpu().numpy()[0])) <= 1e-5
    wy = mm.weight(y.double()).cpu().numpy()[0]          # float64 TOD into the float32 transform
    assert max_rel(wy, o.apply_ninv(y.double().cpu().numpy()[0])) <= 1e-5
    if n_f == 65536:
        return                          # beyond the largest float64 transform
    m64 = _plan(p, "fp64", n_f=32768, fft_shape=shape)
    assert m64.info()["fft_shape"] == (shape if shape in (1, 3, 6, 8) else 1)
    assert max_rel(m64.apply_A(x).cpu().numpy()[0], want) <= TOL["fp64"]
    wy = m64.weight(y.double()).cpu().numpy()[0]
    assert max_rel(wy, o.apply_ninv(y.double().cpu().numpy()[0])) <= 1e-12


@pytest.mark.parametrize("n_f", [1 << 17, 1 << 18])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_four_step_transform_lengths_match_the_oracle(n_f, precision):
    """The paper's FFT lengths beyond one workgroup (batched four-step transform): N^-1 and H x
    against the oracle at n_f = 2^17 and 2^18, in float32 and float64."""
    p = _gen("c3", n_det=2, det_len=1 << 18)
    o = _host_oracle(p)
    mm = _plan(p, precision, n_f=n_f)
    assert mm.info()["n_f"] == n_f
    x = _random_map(1, p.n_pix, 23)
    hx = mm.apply_A(x).cpu().numpy()[0]
    want = o.to_global(o.apply_H(o.to_observed(x[0].cpu().numpy())))
    assert max_rel(hx, want) <= TOL[precision]
    y = p.tod[:1].contiguous()
    if precision == "fp64":
        y = y.double()
    wy = mm.weight(y).double().cpu().numpy()[0]
    err = max_rel(wy, o.apply_ninv(y.double().cpu().numpy()[0]))
    print(f"n_f {n_f} {precision}: N^-1 max rel {err:.3e}", flush=True)
    assert err <= (1e-5 if precision == "mixed" else 1e-12)
    m, _ = mm.solve(p.tod, fixed_iters=4, refine=False)
    b = o.rhs(p.tod.double().cpu().numpy()[0])
    xo, _ = o.pcg(b, fixed_iters=4)
    assert max_rel(m.cpu().numpy()[0], o.to_global(xo)) <= TOL[precision]


def test_four_step_transform_on_ragged_intervals():
    """Intervals of 1 to 300,000 samples (one chunk, several chunks, shorter than the halo)
    through the 2^17-point four-step transform, two filters, against the direct convolution."""
    import synth
    from gpu_helpers import plan_for, oracle_for, tod_tensor
    lens = [[1, 7, 300, 70000, 150000], [131000, 3]]
    p = synth.make_custom(3, grid=(64, 64), det_lens=tuple(sum(l) for l in lens), interval_lens=lens,
                          filters=((1.0, 0.3, 1.6), (0.8, 0.1, 1.2)), n_c=512, f_samp=50.0, seed=31)
    o = oracle_for(p, 1 << 16)
    for precision, tol in (("fp64", 1e-12), ("mixed", 1e-5)):
        mm = plan_for(p, precision=precision, n_f=1 << 17, lag_dft_len=1 << 16)
        y = tod_tensor(p)
        wy = mm.weight(y if precision == "fp64" else y.float()).double().cpu().numpy()[0]
        assert max_rel(wy, o.apply_ninv(p.tod[0])) <= tol, precision
