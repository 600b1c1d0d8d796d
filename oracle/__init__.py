"""Plain FP64 CPU oracle for cascading-smoother multigrid.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the HIP library and its
Python binding never do, and nothing here imports them.
"""
from .cascade import *  # noqa: F401,F403
