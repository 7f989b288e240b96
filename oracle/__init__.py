"""FP64 CPU oracle for loopy belief propagation -- test infrastructure only.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the HIP implementation.
"""
from .oracle import OracleGraph, build_oracle, oracle_available  # noqa: F401
