"""FP64 CPU oracle for QR-based CP-ALS.  Test infrastructure only: imported by
the test suite, the smoke check and the benchmark's CPU-baseline leg, never by
the product path."""
from .cpqr_oracle import *  # noqa: F401,F403
