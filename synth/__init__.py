"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This package only *produces inputs*: scan pointing (pixel index per sample and
the polarisation-angle pair sin 2a, cos 2a), stationary-interval tables, noise
parameters and simulated time-ordered data.  It holds none of the map-maker's
arithmetic (no pointing operators, no inverse-noise filter, no solver); both the
oracle and the HIP library take its arrays as given.

Every array is a deterministic function of (config, component, detector,
realisation) through ``numpy.random.SeedSequence``.
"""

from .generate import (  # noqa: F401
    CONFIGS,
    Problem,
    make_problem,
    make_custom,
    log_uniform_intervals,
)
