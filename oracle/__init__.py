"""FP64 CPU oracle of the shift-and-stack search (test infrastructure only).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
use this package; the HIP library never imports or links it.
"""
from .core import *  # noqa: F401,F403
