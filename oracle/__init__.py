"""FP64 CPU checker for the SSI-COV path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke entry point and the
CPU-baseline leg of the benchmark, never by the library.  It shares no code
with the GPU path.
"""
from .ssicov_ref import *  # noqa: F401,F403
from . import philox  # noqa: F401
from . import stability  # noqa: F401
from . import fp8  # noqa: F401
