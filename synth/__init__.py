"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package holds no arithmetic of the method itself (no Dirac operator,
no smoother, no multigrid): only random gauge links, spinors, gauge
transforms and test vectors, drawn from numpy's PCG64 generator so both
sides of every parity comparison receive identical bits.
"""
from .fields import (  # noqa: F401
    seed_for, random_links, unit_links, random_spinors, gauge_transform,
    random_test_vectors, kappa_to_m0, device_gaussian_spinors,
)
