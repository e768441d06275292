"""CPU checker for the spectral network-formation hot path.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the package smoke
check and by the benchmark's CPU-baseline leg, never by the product path.
See ``oracle.nf_oracle`` for the implementation and its citations.
"""
from .nf_oracle import *  # noqa: F401,F403
