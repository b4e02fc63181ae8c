"""Seeded synthetic HWPM inputs (shared by the tests, the oracle and the benchmark)."""
from .generators import (  # noqa: F401
    Workload, workload, random_matrix, stencil27, rmat, small_random, from_dense,
)
