"""HWPM oracle (test infrastructure only).

A plain sequential CPU implementation of the paper's method, used by the
tests, the smoke check and the benchmark's CPU-baseline leg to check the HIP
library.  Nothing in the product package imports it.
"""
from .oracle import (  # noqa: F401
    build_oracle,
    oracle_tree_sum,
    oracle_improve,
    oracle_greedy,
    oracle_mcm,
    oracle_match,
    OracleResult,
)
