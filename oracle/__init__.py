"""CPU oracle for the blocked randomized QB factorisation (randQB_b, randQB_pb).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64 CPU
implementation written from the paper (Martinsson & Voronin, "A randomized
blocked algorithm for efficiently computing rank-revealing factorizations of
matrices", Sections 3-4, Figures 4 and 6).  Only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it.  The GPU
library never calls into it and shares no code, constants or helpers with it.

Modules
  philox    Philox4x32-10 counter-based generator (integer words)
  gaussian  53-bit uniforms, own log / sin-cos, Box-Muller -> Omega
  cholqr    Cholesky QR with column dropping, applied twice (orth)
  randqb    the blocked adaptive QB driver and its stopping rule
  checks    Eckart-Young optimum, expectation bound, orthonormality etc.

Parity status of each function is stated in its module header.
"""
from .philox import philox4x32_10  # noqa: F401
from .gaussian import omega_block, uniforms53, log_own, sincos_2pi  # noqa: F401
from .cholqr import chol_drop, cholqr, cholqr2  # noqa: F401
from .randqb import randqb_pb, QBResult, STOP, STATUS  # noqa: F401
