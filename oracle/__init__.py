"""FP64 CPU oracle for the modified Born series (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product path never does.
"""

from .mbs_oracle import *  # noqa: F401,F403
