"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package draws random matrices and vectors only; it holds none of the
solver's arithmetic (no partition, proposal, block update or residual).
"""
from .gen import (  # noqa: F401
    WORKLOADS,
    haar,
    log_spaced,
    dense_svd_system,
    dense_random_system,
    csr_system,
    make,
    to_bf16_bits,
    bf16_bits_to_f64,
)
