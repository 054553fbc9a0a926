"""Device-side generation of the large workloads (inputs only).

Same recipes as ``synth.generate`` (raster scans with detector offsets, a
2 Hz half-wave plate, log-uniform stationary intervals, per-detector 1/f noise
by Fourier shaping, N(0, 1) sky) but computed with torch on the GPU, so that
2^28-2^30-sample workloads with several noise realisations are produced in
seconds.  Random numbers come from torch generators seeded per (config,
component, detector/interval, realisation); interval lengths and noise
parameters come from the same NumPy streams as the host generator.

Returns a ``DeviceProblem`` whose pointing and TOD stay on the device; host
copies of slices (for the oracle) are made by the caller.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np
import torch

from .generate import (_FILTERS, _INTERVALS, _NOISE, _SKY, _per_det_filters, _rng,
                       log_uniform_intervals)


@dataclasses.dataclass
class DeviceProblem:
    name: str
    n_stokes: int
    n_pix: int
    pix: torch.Tensor          # int32 [n_t] (device)
    w: torch.Tensor            # float32 [n_t, 2] (device)
    tod: torch.Tensor          # float32 [n_rhs, n_t] (device)
    iv_start: np.ndarray       # int64 [n_b + 1]
    iv_filter: np.ndarray      # int32 [n_b]
    filter_params: np.ndarray  # float64 [n_filters, 3]
    f_samp: float
    n_c: int
    det_start: np.ndarray      # int64 [n_det + 1]
    meta: dict

    @property
    def n_samples(self) -> int:
        return int(self.pix.shape[0])

    @property
    def n_rhs(self) -> int:
        return int(self.tod.shape[0])


def _gen(device, *tags) -> torch.Generator:
    g = torch.Generator(device=device)
    seed = int(np.random.SeedSequence([int(t) for t in tags]).generate_state(1, dtype=np.uint64)[0] >> 1)
    g.manual_seed(seed)
    return g


def _raster(n, width, height, speed, drift, x0, y0, transpose, device):
    t = torch.arange(n, dtype=torch.float64, device=device)
    phase = torch.remainder(speed * t, 2.0 * width)
    x = torch.where(phase < width, phase, 2.0 * width - phase)
    ix = torch.clamp(torch.floor(x), max=width - 1).to(torch.int64)
    ix = torch.remainder(ix + int(round(x0)), width)
    yy = y0 + drift * speed * t / width
    iy = torch.remainder(torch.floor(yy).to(torch.int64), height)
    if transpose:
        return (ix * width + iy).to(torch.int32)
    return (iy * width + ix).to(torch.int32)


def _noise_fill(out: torch.Tensor, lens: List[int], params, f_samp, gen_tags, device):
    """Fill consecutive intervals of ``out`` (float32 view) with shaped 1/f noise."""
    pos = 0
    for k, n in enumerate(lens):
        sg, fk, al = params[k]
        L = 1 << max(1, (2 * n - 1).bit_length())
        g = _gen(device, *gen_tags, k)
        white = torch.randn(L, generator=g, device=device, dtype=torch.float32)
        spec = torch.fft.rfft(white)
        nu = torch.arange(L // 2 + 1, device=device, dtype=torch.float64) * (f_samp / L)
        amp = torch.empty_like(nu)
        amp[1:] = sg * torch.sqrt(1.0 + (fk / nu[1:]) ** al)
        amp[0] = 0.0 if fk > 0 else sg
        out[pos:pos + n] += torch.fft.irfft(spec * amp.to(torch.float32), n=L)[:n]
        pos += n


def _poorly_conditioned(blocks: torch.Tensor) -> torch.Tensor:
    """Pixels whose block [[n, S, C], [S, SS, SC], [C, SC, CC]] has min/max eigenvalue < 1e-3.

    Closed-form eigenvalues of a symmetric 3x3 matrix (trigonometric solution of
    its characteristic cubic), evaluated elementwise in float64.
    """
    a00, a01, a02, a11, a12, a22 = blocks[0], blocks[1], blocks[2], blocks[3], blocks[4], blocks[5]
    p1 = a01 * a01 + a02 * a02 + a12 * a12
    q = (a00 + a11 + a22) / 3.0
    p2 = (a00 - q) ** 2 + (a11 - q) ** 2 + (a22 - q) ** 2 + 2.0 * p1
    p = torch.sqrt(p2 / 6.0)
    safe = torch.where(p > 0, p, torch.ones_like(p))
    b00, b11, b22 = (a00 - q) / safe, (a11 - q) / safe, (a22 - q) / safe
    b01, b02, b12 = a01 / safe, a02 / safe, a12 / safe
    det = b00 * (b11 * b22 - b12 * b12) - b01 * (b01 * b22 - b12 * b02) + b02 * (b01 * b12 - b11 * b02)
    phi = torch.acos(torch.clamp(det / 2.0, -1.0, 1.0)) / 3.0
    e_max = q + 2.0 * p * torch.cos(phi)
    e_min = q + 2.0 * p * torch.cos(phi + 2.0 * math.pi / 3.0)
    seen = a00 > 0
    ratio = torch.where(e_max > 0, e_min / torch.where(e_max > 0, e_max, torch.ones_like(e_max)),
                        torch.zeros_like(e_max))
    return seen & (ratio < 1e-3)


def make_device_problem(name: str, device="cuda:0", n_det=None, n_rhs=None, det_len=None,
                        seed=None) -> DeviceProblem:
    """c3 (64 detectors, 2^28 samples, 2^20 pixels) or c5 (256 detectors, 2^30 samples,
    12 x 2048^2 pixels, 8 realisations); n_det / det_len shrink them for tests."""
    device = torch.device(device)
    if name == "c3":
        W = H = 1024
        speed, drift = 0.5, 0.5
        n_det = 64 if n_det is None else n_det
        det_len = (1 << 22) if det_len is None else det_len
        n_rhs = 1 if n_rhs is None else n_rhs
        seed = 3 if seed is None else seed
        lo, hi = 1 << 14, 1 << 21

        def geom(d):
            return dict(x0=16.0 * (d % 8), y0=16.0 * (d // 8), transpose=bool(d % 2))
    elif name == "c5":
        W, H = 4096, 12288
        speed, drift = 1.0, 1.0
        n_det = 256 if n_det is None else n_det
        det_len = (1 << 22) if det_len is None else det_len
        n_rhs = 8 if n_rhs is None else n_rhs
        seed = 5 if seed is None else seed
        lo, hi = 1 << 16, 1 << 22

        def geom(d):
            return dict(x0=0.0, y0=48.0 * d, transpose=False)
    else:
        raise ValueError(name)
    f_samp, f_hwp = 200.0, 2.0
    n_pix = W * H
    n_t = n_det * det_len
    fp = _per_det_filters(seed, n_det)

    pix = torch.empty(n_t, dtype=torch.int32, device=device)
    w = torch.empty((n_t, 2), dtype=torch.float32, device=device)
    iv_lens = []
    for d in range(n_det):
        a = d * det_len
        pix[a:a + det_len] = _raster(det_len, W, H, speed, drift, device=device, **geom(d))
        t = torch.arange(det_len, dtype=torch.float64, device=device)
        ang = math.radians(45.0 * (d % 4)) + 2.0 * (2.0 * math.pi * f_hwp * t / f_samp)
        w[a:a + det_len, 0] = torch.sin(2.0 * ang).to(torch.float32)
        w[a:a + det_len, 1] = torch.cos(2.0 * ang).to(torch.float32)
        iv_lens.append(log_uniform_intervals(det_len, lo, hi, _rng(seed, _INTERVALS, d)))

    # excision: fewer than 3 hits, or eigenvalue ratio of sum (1, s, c)(1, s, c)^T below 1e-3
    blocks = torch.zeros((6, n_pix), dtype=torch.float64, device=device)
    for d in range(n_det):
        a = d * det_len
        p64 = pix[a:a + det_len].to(torch.int64)
        s = w[a:a + det_len, 0].to(torch.float64)
        c = w[a:a + det_len, 1].to(torch.float64)
        for k, v in enumerate((torch.ones_like(s), s, c, s * s, s * c, c * c)):
            blocks[k].index_add_(0, p64, v)
    hits = blocks[0]
    bad = _poorly_conditioned(blocks) | ((hits > 0) & (hits < 3))
    del blocks
    for d in range(n_det):
        a = d * det_len
        seg = pix[a:a + det_len]
        seg[bad[seg.to(torch.int64)]] = -1

    starts = [0]
    filt = []
    for d, lens in enumerate(iv_lens):
        for n in lens:
            starts.append(starts[-1] + n)
            filt.append(d)
    iv_start = np.asarray(starts, dtype=np.int64)
    iv_filter = np.asarray(filt, dtype=np.int32)

    g = _gen(device, seed, _SKY)
    sky = torch.randn((n_pix, 3), generator=g, device=device, dtype=torch.float32).to(torch.float64)
    tod = torch.empty((n_rhs, n_t), dtype=torch.float32, device=device)
    for d in range(n_det):
        a = d * det_len
        pd = pix[a:a + det_len]
        ok = pd >= 0
        pv = torch.where(ok, pd, torch.zeros_like(pd)).to(torch.int64)
        sig = 0.5 * (sky[pv, 0] + w[a:a + det_len, 0].double() * sky[pv, 1]
                     + w[a:a + det_len, 1].double() * sky[pv, 2])
        sig = torch.where(ok, sig, torch.zeros_like(sig)).to(torch.float32)
        for r in range(n_rhs):
            tod[r, a:a + det_len].copy_(sig)
            _noise_fill(tod[r, a:a + det_len], iv_lens[d], [fp[d]] * len(iv_lens[d]), f_samp,
                        (seed, _NOISE, d, r), device)
    det_start = np.arange(n_det + 1, dtype=np.int64) * det_len
    return DeviceProblem(name=name, n_stokes=3, n_pix=n_pix, pix=pix, w=w, tod=tod, iv_start=iv_start,
                         iv_filter=iv_filter, filter_params=fp, f_samp=f_samp, n_c=8192,
                         det_start=det_start, meta=dict(grid=(W, H), sky=sky))
