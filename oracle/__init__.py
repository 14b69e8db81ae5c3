"""CPU FP64 oracle for sketched GMRES -- test infrastructure only.

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the HIP implementation.
"""

from .oracle import *  # noqa: F401,F403
