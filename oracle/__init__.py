"""FP64 CPU oracle (test infrastructure only).

Imported by the tests, the smoke check and the benchmark's CPU-baseline leg; never by the
library. It shares no code with the device path.
"""
from .hmc import *  # noqa: F401,F403
from . import hmc, loops, philox, split  # noqa: F401
