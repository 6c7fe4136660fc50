"""FP64 CPU oracle for the Active Set dual bound (test infrastructure only).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  It shares no code with the GPU library.
"""
from .asd_oracle import *  # noqa: F401,F403
