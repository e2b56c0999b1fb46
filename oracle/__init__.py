"""Plain FP64 CPU oracle of the powder-XRD pipeline.

TEST INFRASTRUCTURE ONLY: the checker for the GPU library.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
this package.  It shares no code with the library; the two meet only in the
seeded input generator, which holds none of the method's arithmetic.

The arithmetic lives in ``xrd_oracle.c`` (double precision, no FMA
contraction); this module loads it with ctypes and adds the orchestration
and the finite-difference loss used to check gradients.
"""

from .oracle import *  # noqa: F401,F403
