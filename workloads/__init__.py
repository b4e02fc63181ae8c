"""Seeded synthetic HWPM inputs (shared by the tests, the oracle and the benchmark)."""
from .generators import (  # noqa: F401
    Workload, workload, random_matrix, stencil27, rmat, small_random, from_dense,
    option_a, equilibrated, magnitudes, with_weights, serving_matrix, poisson_arrivals,
    SERVING_SEED,
)
