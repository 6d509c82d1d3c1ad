"""FP64 CPU oracle for the multimode Floquet hot path -- test infrastructure.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library."""
from .floquet import *  # noqa: F401,F403
from . import floquet  # noqa: F401
