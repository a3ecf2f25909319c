"""FP64 CPU oracle for multilevel NMF (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The HIP library never calls it and shares no code with it.
"""
from .nmf_oracle import *  # noqa: F401,F403
