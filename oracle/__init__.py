"""CPU FP64 oracle for Exp-ParaDiag -- test infrastructure only.

Imported by the test suite, the smoke check and the CPU-baseline leg of the
benchmark; never by the GPU library.
"""
from .expdiag_oracle import *  # noqa: F401,F403
