"""MI355X-native maximum-likelihood CMB map-maker (MADmap's PCG hot path).

The solver lives in libmm.so (HIP kernels for gfx950 behind the C ABI of
include/mm.h); this package only binds it for torch device tensors.
"""

from ._lib import MMError, load  # noqa: F401
from .mapmaker import MapMaker, fft_length_rule, noise_lags  # noqa: F401
from .autograd import solve_map  # noqa: F401

__all__ = ["MapMaker", "MMError", "fft_length_rule", "load", "noise_lags", "solve_map"]
