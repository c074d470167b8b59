"""FP64 CPU oracle for the ISDF-SMW dielectric inverse (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library.
"""
from .dielectric import *  # noqa: F401,F403
