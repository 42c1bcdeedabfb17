"""FP64 CPU oracle for ROR-BK -- test infrastructure.

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the HIP library.
"""
from .oracle import *  # noqa: F401,F403
