"""CPU FP64 oracle for the column interpolative decomposition.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything under ``oracle/``: only the test-suite, the package's
``smoke()`` check and the CPU-baseline leg of the benchmark use it.  It shares
no code with the HIP implementation.
"""
from .id_oracle import *  # noqa: F401,F403
