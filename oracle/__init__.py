"""CPU reference oracle for one MPPI iteration — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It evaluates Algorithm 1 of arXiv 2409.07563 in binary64 (see
mppi_oracle.c) and shares no code with the GPU library.
"""
from .oracle import *  # noqa: F401,F403
