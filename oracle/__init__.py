"""Plain FP64 CPU oracle of the ELBM step (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  The product path (the HIP library and its Python binding)
never does.
"""
from .oracle import *  # noqa: F401,F403
