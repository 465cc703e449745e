"""FP64 CPU oracle of online convolutional sparse coding.

Test infrastructure only: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the HIP product path.
"""
from .ocsc_oracle import *  # noqa: F401,F403
from .ocsc_oracle import OCSC  # noqa: F401
