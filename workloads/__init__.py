"""Seeded synthetic input generators (shared by tests, benchmark and oracle checks)."""
from .gen import (PAPER_SEED, Support, complex_normal, composite_support,  # noqa: F401
                  elementary_support, homogeneous_support, log_uniform_coefficients,
                  rng_for, sample_values)
