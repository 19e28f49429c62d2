"""CPU FP64 reference for the pseudo-spectral DNS right-hand side.

Test infrastructure only: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the library.
"""
from .psdns_oracle import *  # noqa: F401,F403
