"""FP64 CPU oracle for the SPOD hot path: test infrastructure only.

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package; the HIP library and its binding never do.
"""
from .spod_oracle import *  # noqa: F401,F403
from .spod_oracle import __all__  # noqa: F401
