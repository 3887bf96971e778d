"""FP64 CPU oracle for COPA. Test infrastructure only: imported by tests, the smoke check and the
benchmark's CPU-baseline leg; never by the library."""
from .copa_oracle import *  # noqa: F401,F403
