"""Template inputs and simulated parasitic signals (inputs only).

For the template-extended pointing of the "Using MADmap" section this module
produces, from a problem's scan:

* destriping offset indices: consecutive offset intervals of fixed length
  inside each detector (case 3 of that section);
* ground-synchronous bin indices: the scan's azimuth (the raster's x
  coordinate) cut into equal bins (case 1);
* the half-wave-plate angle w_t = 2 pi f_hwp t / f_samp (mod 2 pi) of every
  sample and the detector segments (case 2);

and simulates the parasitic signals those templates model, added to the TOD:
an offset per offset interval, a ground profile per azimuth bin, and the HWP
signal of eq. HWPmat written as its sum over harmonics k = 1..8 with the time
t in seconds from the segment start.  It holds none of the map-maker's
arithmetic; the oracle and the library each build their own template matrix
from these arrays.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

from .generate import Problem, _rng

_TEMPLATES = 6


def offset_index(det_start: np.ndarray, length: int):
    """Offset interval of every sample: intervals of ``length`` samples restarting at
    every detector boundary (a detector's last interval may be shorter)."""
    det_start = np.asarray(det_start, dtype=np.int64)
    n_t = int(det_start[-1])
    idx = np.empty(n_t, dtype=np.int32)
    base = 0
    for d in range(det_start.shape[0] - 1):
        a, e = int(det_start[d]), int(det_start[d + 1])
        k = np.arange(e - a) // length
        idx[a:e] = base + k
        base += int(-(-(e - a) // length))
    return idx, base


def azimuth_index(det_lens, width: int, speed: float, n_bins: int):
    """Azimuth bin of every sample: the raster's triangle-wave x coordinate over
    ``width`` columns at ``speed`` columns per sample, cut into ``n_bins`` bins."""
    out = []
    for n in det_lens:
        t = np.arange(n, dtype=np.float64)
        phase = np.mod(speed * t, 2.0 * width)
        x = np.where(phase < width, phase, 2.0 * width - phase)
        out.append(np.minimum((x * n_bins / width).astype(np.int64), n_bins - 1))
    return np.concatenate(out).astype(np.int32), int(n_bins)


def hwp_angle(det_lens, f_hwp: float, f_samp: float) -> np.ndarray:
    """Polarizer angle of every sample, float32 in [0, 2 pi)."""
    out = []
    for n in det_lens:
        t = np.arange(n, dtype=np.float64)
        out.append(np.mod(2.0 * math.pi * f_hwp * t / f_samp, 2.0 * math.pi))
    return np.concatenate(out).astype(np.float32)


def hwp_signal(omega: np.ndarray, seg_start: np.ndarray, coef: np.ndarray, f_samp: float) -> np.ndarray:
    """psi(t) = sum_k (b_k + t b_{k+8}) cos(k w_t) + (b_{k+16} + t b_{k+24}) sin(k w_t),
    k = 1..8, with t in seconds from the start of the sample's segment and
    b = coef[g] (32 values, 0-based) for segment g."""
    om = np.asarray(omega, dtype=np.float64)
    out = np.zeros(om.shape[0])
    for g in range(seg_start.shape[0] - 1):
        a, e = int(seg_start[g]), int(seg_start[g + 1])
        t = np.arange(e - a, dtype=np.float64) / f_samp
        b = coef[g]
        for k in range(1, 9):
            out[a:e] += (b[k - 1] + t * b[k + 7]) * np.cos(k * om[a:e]) \
                + (b[k + 15] + t * b[k + 23]) * np.sin(k * om[a:e])
    return out


@dataclasses.dataclass
class TemplateInputs:
    offsets: Optional[tuple] = None      # (idx int32 [n_t], n_amp)
    azimuth: Optional[tuple] = None      # (idx int32 [n_t], n_amp)
    hwp: Optional[tuple] = None          # (omega float32 [n_t], seg_start int64 [n_seg + 1])
    truth: dict = dataclasses.field(default_factory=dict)


def add_templates(p: Problem, offsets: int = 0, azimuth_bins: int = 0, hwp: bool = False,
                  amplitude: float = 1.0, seed: int = 0, speed: float = 0.5,
                  f_hwp: float = 2.0) -> tuple:
    """Copy of ``p`` with parasitic signals added to every TOD row, plus their template inputs.

    offsets: offset-interval length (0 = none); azimuth_bins: number of azimuth bins
    (0 = none); hwp: add the HWP parametric signal.  Amplitudes are N(0, amplitude^2)
    (the HWP t-coefficients scaled by 1 / segment duration).  ``speed`` must be the
    raster speed the problem was generated with.
    """
    det_lens = np.diff(p.det_start).tolist()
    n_t = int(p.det_start[-1])
    extra = np.zeros(n_t)
    ti = TemplateInputs()
    if offsets:
        idx, n = offset_index(p.det_start, offsets)
        o = amplitude * _rng(seed, _TEMPLATES, 1).standard_normal(n)
        extra += o[idx]
        ti.offsets = (idx, n)
        ti.truth["offsets"] = o
    if azimuth_bins:
        W = p.meta["grid"][0]
        idx, n = azimuth_index(det_lens, W, speed, azimuth_bins)
        gprof = amplitude * _rng(seed, _TEMPLATES, 2).standard_normal(n)
        extra += gprof[idx]
        ti.azimuth = (idx, n)
        ti.truth["azimuth"] = gprof
    if hwp:
        om = hwp_angle(det_lens, f_hwp, p.f_samp)
        seg = np.asarray(p.det_start, dtype=np.int64)
        coef = amplitude * _rng(seed, _TEMPLATES, 3).standard_normal((seg.shape[0] - 1, 32))
        dur = np.maximum(np.diff(seg), 1) / p.f_samp
        coef[:, 8:16] /= dur[:, None]
        coef[:, 24:32] /= dur[:, None]
        extra += hwp_signal(om, seg, coef, p.f_samp)
        ti.hwp = (om, seg)
        ti.truth["hwp"] = coef
    tod = (p.tod.astype(np.float64) + extra[None, :]).astype(p.tod.dtype)
    q = dataclasses.replace(p, tod=tod, meta=dict(p.meta, parasitic=extra))
    return q, ti
