"""FP64 CPU oracle for the LBM-IBM method (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path never does.
"""
from .oracle import *  # noqa: F401,F403
