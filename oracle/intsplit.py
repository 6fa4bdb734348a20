"""Exact-range sampling product of the mixed-precision form (test
infrastructure only; see the package header).

Why it exists.  The sample Y = A^(i-1) Omega_i of Figure 4 step (3) decides
the subspace of Q_i.  Rounded in a low precision, Y = A Omega + dY leaves in
Q_i a component outside range(A) of the relative size of dY; once the rank
reaches min(m, n) < m no later block can remove it, and the error of the
factorisation floors at that size.  This module defines a sample that lies
in the range of A^(i-1) to float64 accuracy while its products run on
integers:

  Omega~ = clip(rint(16 Omega), -127, 127) / 16
      the sketch on a grid of 1/16 (an 8-bit signed integer per entry); any
      fixed full-rank sketch serves the range finder (Section 3.1);
  E      = ceil(e / 2) + 1,  where D = f 2^e, f in [1/2, 1)  (frexp of
      D = ||A^(i-1)||_F^2, the residual norm of the previous block, or
      ||A||_F^2 before the first block), so that every entry of A^(i-1)
      lies below 2^(E-1) in magnitude;
  A~     = rint(A^(i-1) 2^(55-E)) 2^(E-55)
      A^(i-1) on the fixed-point grid 2^(E-55): at most 2^(E-56) from it,
      and an integer below 2^54 in magnitude once scaled;
  Y      = A~ Omega~.

Then Y = A^(i-1) Omega~ + (A~ - A^(i-1)) Omega~ with the second term below
2^(E-56) |Omega~| per product term: at least as close to range(A^(i-1)) as
a float64 product.  The integer form computes A~ Omega~ exactly as
2^(E-59) sum_k a_k w_k with integers |a_k| < 2^54, |w_k| <= 127.  Here the
product is the float64 matmul of the two grid matrices (a plain definition:
the only rounding is float64's), and the GPU's integer form must agree with
it to float64 rounding.

Pinned by tests/test_oracle_intsplit.py: exact rational products (Python
integers) on small inputs, the grid and range bounds, the 1e-12 error this
sample reaches at k = n < m where a float32-rounded sample floors near
1e-6, and planted mutations of the exponent, the grid and the clip.
"""
from __future__ import annotations

import math

import numpy as np

SKETCH_SCALE = 16.0        # Omega~ on a grid of 1/16
SKETCH_CLIP = 127          # |16 Omega~| <= 127 (8-bit signed)
FRAC_BITS = 55             # A~ on the grid 2^(E - 55)


def split_exponent(D: float) -> int:
    """E with 2^(E-1) > sqrt(D) (so every entry of a matrix of Frobenius
    norm sqrt(D) lies below 2^(E-1)); 0 for D <= 0."""
    if not (D > 0.0):
        return 0
    _, e = math.frexp(D)          # D = f 2^e, f in [1/2, 1): sqrt(D) < 2^ceil(e/2)
    return -((-e) // 2) + 1


def quantize_sketch(Om: np.ndarray) -> np.ndarray:
    """Omega~ = clip(rint(16 Omega), -127, 127) / 16 (float64 values)."""
    q = np.clip(np.rint(np.asarray(Om, dtype=np.float64) * SKETCH_SCALE), -SKETCH_CLIP, SKETCH_CLIP)
    return q / SKETCH_SCALE


def fixed_point(R: np.ndarray, E: int) -> np.ndarray:
    """A~ = rint(R 2^(55-E)) 2^(E-55)."""
    R = np.asarray(R, dtype=np.float64)
    return np.ldexp(np.rint(np.ldexp(R, FRAC_BITS - E)), E - FRAC_BITS)


def sample_exact(R: np.ndarray, Om: np.ndarray, D: float) -> np.ndarray:
    """Y = A~ Omega~ with E from D (see the module header)."""
    E = split_exponent(D)
    return fixed_point(R, E) @ quantize_sketch(Om)
