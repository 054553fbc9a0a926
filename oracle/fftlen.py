"""FFT length for the overlap-save filter (oracle; test infrastructure only).

Weighting section, eq. FFTcomplexity: filtering n_t samples with FFTs of length
n_f, each producing n_f - 2 n_c uncorrupted outputs, costs
ceil(n_t / (n_f - 2 n_c)) n_f log2 n_f.  Its continuous proxy is
h(n_f) = n_f ln n_f / (n_f - 2 n_c) (eq. FFTcomplexityFunction) whose
stationary point satisfies n_f - 2 n_c (1 + ln n_f) = 0; Appendix A shows it
is a minimum.

The rule: start at the smallest power of two not below the longest stationary
interval ("larger than" read as >=); if h' there is positive, halve n_f until
h'(n_f / 2) < 0 or n_f / 2 < 2 n_c.
"""

from __future__ import annotations

import math


def h(nf: float, nc: float) -> float:
    return nf * math.log(nf) / (nf - 2.0 * nc)


def h_prime(nf: float, nc: float) -> float:
    d = nf - 2.0 * nc
    return (1.0 + math.log(nf)) / d - nf * math.log(nf) / (d * d)


def h_second(nf: float, nc: float) -> float:
    d = nf - 2.0 * nc
    return (2.0 * nf * math.log(nf) / d ** 3 - 2.0 * (1.0 + math.log(nf)) / d ** 2
            + 1.0 / (nf * d))


def paper_fft_length(n_c: int, longest: int) -> int:
    """n_f chosen by the paper's halving rule for correlation length n_c."""
    nf = 1
    while nf < longest:
        nf *= 2
    if nf <= 2 * n_c:
        # every output of a transform this short is corrupted; the smallest
        # power of two above 2 n_c is the first admissible length
        nf = 1
        while nf <= 2 * n_c:
            nf *= 2
        return nf
    if h_prime(nf, n_c) > 0:
        while True:
            half = nf // 2
            if half < 2 * n_c or half == 2 * n_c or h_prime(half, n_c) < 0:
                break
            nf = half
    return nf
