"""FP64 CPU oracle for matching-based AMG-preconditioned CG.

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline
leg of the benchmark import this package. The GPU library never does.
"""

from .oracle import *  # noqa: F401,F403
from .oracle import __all__  # noqa: F401
