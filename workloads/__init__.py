"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the
benchmark.  No arithmetic of the method lives here."""
from .generators import (  # noqa: F401
    gaussian,
    gaussian_centered,
    planted_single,
    planted_block,
    gamma_fractions,
    gamma_absolute,
    random_orthonormal,
    serving_requests,
)
