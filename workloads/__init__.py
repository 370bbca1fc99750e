"""Seeded synthetic input generators (shared by tests, benchmark and oracle checks)."""
from .gen import (PAPER_SEED, Support, arithmetic_progression, complex_normal,  # noqa: F401
                  composite_support, elementary_support, gap_support, homogeneous_support,
                  log_uniform_coefficients, rng_for, sample_values,
                  uneven_instances)
