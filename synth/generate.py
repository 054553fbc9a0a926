"""Synthetic scan-and-noise workloads (inputs only).

The paper validates on Planck and EBEX simulations that are not available
here; these generators stand in for them with the same structure: one or more
detectors scanning a pixelised sky in a raster with cross-linking, a rotating
half-wave plate for polarisation sensitivity, stationary intervals of uneven
length and 1/f noise with the power spectrum of the Algorithm section
(sigma, knee frequency, slope).

Pointing is returned the way a pointing library hands it to a map-maker: a
pixel index per sample (-1 marks a sample whose pixel was excised) and, for
polarisation, the pair (sin 2a_t, cos 2a_t) of the polarisation angle a_t,
rounded to float32.  How those numbers enter the pointing matrix is the
map-maker's business, not this module's.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# component tags for SeedSequence spawning
_SKY, _NOISE, _INTERVALS, _FILTERS, _EXTRA = 1, 2, 3, 4, 5


@dataclasses.dataclass
class Problem:
    """One synthetic map-making workload."""

    name: str
    n_stokes: int
    n_pix: int
    pix: np.ndarray            # int32 [n_t], -1 = sample with no sky pixel
    w: Optional[np.ndarray]    # float32 [n_t, 2] = (sin 2a, cos 2a), None for T-only
    iv_start: np.ndarray       # int64 [n_b + 1], covers [0, n_t)
    iv_filter: np.ndarray      # int32 [n_b]
    filter_params: np.ndarray  # float64 [n_filters, 3] = (sigma, f_knee, alpha)
    f_samp: float
    n_c: int
    tod: np.ndarray            # [n_rhs, n_t] float32 or float64
    sky: np.ndarray            # float64 [n_pix, n_stokes]
    det_start: np.ndarray      # int64 [n_det + 1] detector boundaries in the TOD
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_samples(self) -> int:
        return int(self.pix.shape[0])

    @property
    def n_intervals(self) -> int:
        return int(self.iv_filter.shape[0])

    @property
    def n_rhs(self) -> int:
        return int(self.tod.shape[0])


def _rng(seed: int, *tags: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed)] + [int(t) for t in tags]))


def raster(n: int, width: int, height: int, speed: float, drift: float,
           x0: float = 0.0, y0: float = 0.0, transpose: bool = False,
           t0: int = 0) -> np.ndarray:
    """Pixel index of a back-and-forth raster.

    The column coordinate is a triangle wave of amplitude ``width`` moving
    ``speed`` pixels per sample; the row coordinate advances ``drift`` rows
    per one-way traversal.  ``transpose`` swaps rows and columns (square grids
    only), which gives cross-linked passes.
    """
    t = np.arange(t0, t0 + n, dtype=np.float64)
    phase = np.mod(speed * t, 2.0 * width)
    x = np.where(phase < width, phase, 2.0 * width - phase)
    ix = np.minimum(np.floor(x), width - 1).astype(np.int64)
    ix = np.mod(ix + int(round(x0)), width)
    y = y0 + drift * speed * t / width
    iy = np.mod(np.floor(y).astype(np.int64), height)
    if transpose:
        if width != height:
            raise ValueError("transposed raster needs a square grid")
        return (ix * width + iy).astype(np.int32)
    return (iy * width + ix).astype(np.int32)


def log_uniform_intervals(total: int, lo: int, hi: int, rng: np.random.Generator) -> List[int]:
    """Interval lengths drawn log-uniformly in [lo, hi] that sum to ``total``.

    Draws until the sum reaches ``total``, truncates the last draw, and merges
    a remainder shorter than ``lo`` into the previous interval.
    """
    out: List[int] = []
    acc = 0
    while acc < total:
        n = int(math.exp(rng.uniform(math.log(lo), math.log(hi))))
        n = max(lo, min(hi, n))
        n = min(n, total - acc)
        out.append(n)
        acc += n
    if len(out) > 1 and out[-1] < lo:
        out[-2] += out[-1]
        out.pop()
    return out


def noise_realisation(n: int, f_samp: float, sigma: float, f_knee: float, alpha: float,
                      rng: np.random.Generator) -> np.ndarray:
    """Stationary 1/f + white noise of length n by Fourier shaping.

    White N(0, 1) samples of length L = pow2 >= 2n are transformed, every mode
    k > 0 is scaled by sqrt(sigma^2 (1 + (f_knee / nu_k)^alpha)) with
    nu_k = k f_samp / L, the constant mode is removed when f_knee > 0, and the
    first n samples of the inverse transform are kept.
    """
    if n == 0:
        return np.zeros(0)
    L = 1 << max(1, (2 * n - 1).bit_length())
    white = rng.standard_normal(L)
    spec = np.fft.rfft(white)
    nu = np.arange(L // 2 + 1, dtype=np.float64) * (f_samp / L)
    amp = np.empty_like(nu)
    with np.errstate(divide="ignore"):
        amp[1:] = sigma * np.sqrt(1.0 + (f_knee / nu[1:]) ** alpha)
    amp[0] = 0.0 if f_knee > 0 else sigma
    return np.fft.irfft(spec * amp, n=L)[:n]


def _excise(pix: np.ndarray, w: Optional[np.ndarray], n_pix: int, n_stokes: int,
            min_hits: int = 3, min_rcond: float = 1e-3) -> np.ndarray:
    """Mark samples of poorly conditioned polarisation pixels with -1.

    A pixel is excised (Algorithm section, polarisation degeneracy) when it has
    fewer than ``min_hits`` samples or when the eigenvalue ratio of
    sum_t (1, s_t, c_t)(1, s_t, c_t)^T over its samples is below ``min_rcond``.
    This happens before the TOD is simulated, so excised samples carry noise
    only, as after gap filling.
    """
    if n_stokes == 1:
        return pix
    ok = pix >= 0
    p = pix[ok].astype(np.int64)
    s = w[ok, 0].astype(np.float64)
    c = w[ok, 1].astype(np.float64)
    blocks = np.zeros((n_pix, 3, 3))
    rows = (np.ones_like(s), s, c)
    for i in range(3):
        for j in range(i, 3):
            v = np.bincount(p, weights=rows[i] * rows[j], minlength=n_pix)
            blocks[:, i, j] = v
            blocks[:, j, i] = v
    hits = np.bincount(p, minlength=n_pix)
    seen = hits > 0
    bad = np.zeros(n_pix, dtype=bool)
    ev = np.linalg.eigvalsh(blocks[seen])
    with np.errstate(divide="ignore", invalid="ignore"):
        rc = np.where(ev[:, 2] > 0, ev[:, 0] / ev[:, 2], 0.0)
    bad[np.flatnonzero(seen)] = (hits[seen] < min_hits) | (rc < min_rcond)
    out = pix.copy()
    out[ok & bad[np.maximum(pix, 0)]] = -1
    return out


def _assemble(name: str, seed: int, n_stokes: int, n_pix: int,
              det_pix: Sequence[np.ndarray], det_angles: Sequence[Optional[np.ndarray]],
              det_intervals: Sequence[Sequence[int]], det_filter: Sequence[int],
              filter_params: np.ndarray, f_samp: float, n_c: int, tod_dtype,
              n_rhs: int, noiseless: bool = False, meta: Optional[dict] = None) -> Problem:
    pix = np.concatenate(det_pix).astype(np.int32)
    if n_stokes == 3:
        ang = np.concatenate(det_angles)
        w = np.stack([np.sin(2.0 * ang), np.cos(2.0 * ang)], axis=1).astype(np.float32)
    else:
        w = None
    pix = _excise(pix, w, n_pix, n_stokes)

    det_start = np.zeros(len(det_pix) + 1, dtype=np.int64)
    det_start[1:] = np.cumsum([len(p) for p in det_pix])
    starts = [0]
    filt = []
    for d, lens in enumerate(det_intervals):
        assert sum(lens) == len(det_pix[d])
        for n in lens:
            starts.append(starts[-1] + int(n))
            filt.append(int(det_filter[d]))
    iv_start = np.asarray(starts, dtype=np.int64)
    iv_filter = np.asarray(filt, dtype=np.int32)

    sky = _rng(seed, _SKY).standard_normal((n_pix, n_stokes))
    n_t = pix.shape[0]
    signal = np.zeros(n_t)
    ok = pix >= 0
    if n_stokes == 1:
        signal[ok] = sky[pix[ok], 0]
    else:
        s = w[ok, 0].astype(np.float64)
        c = w[ok, 1].astype(np.float64)
        sp = sky[pix[ok]]
        signal[ok] = 0.5 * (sp[:, 0] + s * sp[:, 1] + c * sp[:, 2])

    tod = np.empty((n_rhs, n_t), dtype=tod_dtype)
    for r in range(n_rhs):
        d = signal.copy()
        if not noiseless:
            for b in range(iv_filter.shape[0]):
                a, e = int(iv_start[b]), int(iv_start[b + 1])
                sg, fk, al = filter_params[iv_filter[b]]
                d[a:e] += noise_realisation(e - a, f_samp, sg, fk, al, _rng(seed, _NOISE, b, r))
        tod[r] = d.astype(tod_dtype)

    return Problem(name=name, n_stokes=n_stokes, n_pix=int(n_pix), pix=pix, w=w,
                   iv_start=iv_start, iv_filter=iv_filter,
                   filter_params=np.asarray(filter_params, dtype=np.float64),
                   f_samp=float(f_samp), n_c=int(n_c), tod=tod, sky=sky,
                   det_start=det_start, meta=dict(meta or {}))


def _hwp_angles(n: int, psi: float, f_hwp: float, f_samp: float) -> np.ndarray:
    t = np.arange(n, dtype=np.float64)
    return psi + 2.0 * (2.0 * np.pi * f_hwp * t / f_samp)


def make_c1(seed: int = 1, n_rhs: int = 1, noiseless: bool = False) -> Problem:
    """T-only, 1 detector, 65,536 samples on 32x32 pixels, one interval."""
    W = H = 32
    npass, plen = 4, 16384
    pix = np.concatenate([raster(plen, W, H, 0.25, 0.25, y0=0.37 * k, transpose=bool(k % 2))
                          for k in range(npass)])
    fp = np.array([[1.0, 0.1, 1.5]])
    return _assemble("c1", seed, 1, W * H, [pix], [None], [[npass * plen]], [0], fp,
                     100.0, 1024, np.float64, n_rhs, noiseless,
                     meta=dict(config=0, grid=(W, H)))


def make_c2(seed: int = 2, n_rhs: int = 1, n_det: int = 4, pass_len: int = 1 << 20,
            noiseless: bool = False) -> Problem:
    """TQU, 4 detectors at 0/45/90/135 deg with a 2 Hz half-wave plate, 4 x 2^22 samples."""
    W = H = 256
    f_samp, f_hwp = 200.0, 2.0
    det_pix, det_ang, det_iv = [], [], []
    for d in range(n_det):
        pix = np.concatenate([raster(pass_len, W, H, 0.5, 0.125, y0=4.0 * d + 0.37 * k,
                                     transpose=bool(k % 2)) for k in range(4)])
        det_pix.append(pix)
        det_ang.append(_hwp_angles(pix.shape[0], math.radians(45.0 * d), f_hwp, f_samp))
        det_iv.append([pass_len] * 4)
    fp = np.array([[1.0, 0.2, 1.7]])
    return _assemble("c2", seed, 3, W * H, det_pix, det_ang, det_iv, [0] * n_det, fp,
                     f_samp, 8192, np.float32, n_rhs, noiseless,
                     meta=dict(config=1, grid=(W, H)))


def _per_det_filters(seed: int, n_det: int) -> np.ndarray:
    r = _rng(seed, _FILTERS)
    fk = r.uniform(0.05, 0.5, n_det)
    al = r.uniform(1.0, 2.0, n_det)
    sg = r.uniform(0.5, 2.0, n_det)
    return np.stack([sg, fk, al], axis=1)


def make_c3(seed: int = 3, n_rhs: int = 1, n_det: int = 64, det_len: int = 1 << 22,
            noiseless: bool = False) -> Problem:
    """64 detectors, ~2^28 samples, 2^20 pixels x TQU, uneven intervals, per-detector noise."""
    W = H = 1024
    f_samp, f_hwp = 200.0, 2.0
    det_pix, det_ang, det_iv = [], [], []
    for d in range(n_det):
        det_pix.append(raster(det_len, W, H, 0.5, 0.5, x0=16.0 * (d % 8), y0=16.0 * (d // 8),
                              transpose=bool(d % 2)))
        det_ang.append(_hwp_angles(det_len, math.radians(45.0 * (d % 4)), f_hwp, f_samp))
        det_iv.append(log_uniform_intervals(det_len, 1 << 14, 1 << 21, _rng(seed, _INTERVALS, d)))
    fp = _per_det_filters(seed, n_det)
    return _assemble("c3", seed, 3, W * H, det_pix, det_ang, det_iv, list(range(n_det)), fp,
                     f_samp, 8192, np.float32, n_rhs, noiseless,
                     meta=dict(config=2, grid=(W, H)))


def make_c5(seed: int = 5, n_rhs: int = 8, n_det: int = 256, det_len: int = 1 << 22,
            noiseless: bool = False) -> Problem:
    """256 detectors, 2^30 samples, 12*2048^2 pixels x TQU, 8 noise realisations."""
    W, H = 4096, 12288
    f_samp, f_hwp = 200.0, 2.0
    det_pix, det_ang, det_iv = [], [], []
    for d in range(n_det):
        det_pix.append(raster(det_len, W, H, 1.0, 1.0, y0=48.0 * d))
        det_ang.append(_hwp_angles(det_len, math.radians(45.0 * (d % 4)), f_hwp, f_samp))
        det_iv.append(log_uniform_intervals(det_len, 1 << 16, 1 << 22, _rng(seed, _INTERVALS, d)))
    fp = _per_det_filters(seed, n_det)
    return _assemble("c5", seed, 3, W * H, det_pix, det_ang, det_iv, list(range(n_det)), fp,
                     f_samp, 8192, np.float32, n_rhs, noiseless,
                     meta=dict(config=4, grid=(W, H)))


CONFIGS = {"c1": make_c1, "c2": make_c2, "c3": make_c3, "c5": make_c5}


def make_problem(name: str, **kw) -> Problem:
    """Build a named workload (c1, c2, c3, c5; c4 is c1 with a map loss)."""
    if name == "c4":
        p = make_c1(seed=kw.pop("seed", 4), **kw)
        p.name = "c4"
        p.meta["loss_w"] = _rng(4, _EXTRA).uniform(0.5, 1.5, (p.n_pix, p.n_stokes))
        return p
    return CONFIGS[name](**kw)


def make_custom(n_stokes: int, grid=(16, 16), det_lens=(6000,), interval_lens=None,
                filters=((1.0, 0.5, 1.5),), det_filter=None, f_samp: float = 100.0,
                n_c: int = 64, speed: float = 0.5, drift: float = 0.5, tod_dtype=np.float64,
                n_rhs: int = 1, seed: int = 11, noiseless: bool = False,
                f_hwp: float = 2.0) -> Problem:
    """Small workloads for tests: any detector count, ragged intervals, any n_c.

    ``interval_lens[d]`` lists detector d's interval lengths (default: one
    interval per detector); ``det_filter[d]`` picks its noise filter.
    """
    W, H = grid
    det_pix, det_ang, det_iv = [], [], []
    for d, n in enumerate(det_lens):
        det_pix.append(raster(n, W, H, speed, drift, x0=3.0 * d, y0=1.7 * d,
                              transpose=bool(d % 2) and W == H))
        det_ang.append(_hwp_angles(n, math.radians(45.0 * (d % 4)), f_hwp, f_samp))
        det_iv.append(list(interval_lens[d]) if interval_lens is not None else [n])
    if det_filter is None:
        det_filter = [d % len(filters) for d in range(len(det_lens))]
    return _assemble("custom", seed, n_stokes, W * H, det_pix,
                     det_ang if n_stokes == 3 else [None] * len(det_lens), det_iv,
                     det_filter, np.asarray(filters, dtype=np.float64), f_samp, n_c,
                     tod_dtype, n_rhs, noiseless, meta=dict(grid=(W, H)))
