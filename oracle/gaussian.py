"""Gaussian sketch Omega for the blocked scheme, built from Philox words.

The paper asks for an n x b matrix of iid standard normal entries per block
(Figure 4 step (2), Figure 6 step (2); eq. (OmegaBlock) in Section 4.1 shows
the blocks as slices of one n x (s b) Gaussian matrix).  The reading taken
here: entry (i, j) of the full sketch, for global column j = 0, 1, 2, ... ,
is a pure function of (seed, i, j), so block i is the column slice
[k, k + w) of the same matrix whatever the block size.  Rows 2t and 2t+1 of
column j come from one Philox call with counter (t, j, batch, 0):

    u1 = ((x0 << 21 | x1 >> 11) + 1) * 2^-53        in (0, 1], exact
    u2 = ((x2 << 21 | x3 >> 11) + 1) * 2^-53
    rho = sqrt(-2 log u1)
    Omega[2t, j] = rho cos(2 pi u2),  Omega[2t+1, j] = rho sin(2 pi u2)

(Box and Muller, 1958).  The logarithm and the sine/cosine are evaluated here
with only correctly rounded IEEE operations (+, -, *, /, sqrt, exact
scaling by powers of two), in a fixed order and without fused multiply-add,
so that any IEEE double implementation of the same steps gives the same bits:

  log u:  u = f 2^e with f in [sqrt(1/2), sqrt(2));  s = (f-1)/(f+1);
          log f = 2 s (1 + s^2/3 + s^4/5 + ... + s^20/21)  (atanh series);
          log u = e ln2_hi + (log f + e ln2_lo), ln2_hi holding 33 bits.
  cos/sin(2 pi u):  x = 4u,  q = rint(x),  r = x - q  (|r| <= 1/2, exact),
          phi = r * (pi/2), Taylor series of sin to phi^17 and cos to phi^18,
          then a quarter-turn rotation by q.

Parity pinned by: tests/test_oracle_gaussian.py (log and sin/cos against the
platform libm to a few ulp, Box-Muller moments and a Kolmogorov-Smirnov test
against N(0,1)); bitwise equality with the GPU is a GPU parity test.
"""
from __future__ import annotations

import struct
from decimal import Decimal, getcontext
from math import factorial

import numpy as np

from .philox import philox4x32_10, key_from_seed


# ---- constants, each derived here from its mathematical definition --------
def _nearest_double_of(dec: Decimal) -> float:
    return float(dec)  # Decimal -> float conversion is correctly rounded


getcontext().prec = 60
_LN2_DEC = Decimal(2).ln()
_LN2 = _nearest_double_of(_LN2_DEC)
_bits = struct.unpack("<Q", struct.pack("<d", _LN2))[0] & ~((1 << 20) - 1)
LN2_HI = struct.unpack("<d", struct.pack("<Q", _bits))[0]  # 33 significant bits
LN2_LO = _nearest_double_of(_LN2_DEC - Decimal(LN2_HI))
SQRT_HALF = _nearest_double_of(Decimal("0.5").sqrt())
# pi/2 from the Machin formula pi = 16 atan(1/5) - 4 atan(1/239), in Decimal


def _atan_inv(x: int) -> Decimal:
    x2 = x * x
    term = Decimal(1) / x
    total = term
    k = 1
    while True:
        term /= -x2
        add = term / (2 * k + 1)
        if abs(add) < Decimal(10) ** -58:
            break
        total += add
        k += 1
    return total


_PI_DEC = 16 * _atan_inv(5) - 4 * _atan_inv(239)
HALF_PI = _nearest_double_of(_PI_DEC / 2)

# atanh series coefficients 1/(2k+1), k = 0..10
ATANH_C = [1.0 / float(2 * k + 1) for k in range(11)]
# sin: (-1)^k / (2k+1)!, k = 0..8;  cos: (-1)^k / (2k)!, k = 0..9
SIN_C = [(-1.0) ** k / float(factorial(2 * k + 1)) for k in range(9)]
COS_C = [(-1.0) ** k / float(factorial(2 * k)) for k in range(10)]

TWO_M53 = 2.0 ** -53


def uniforms53(hi_word, lo_word) -> np.ndarray:
    """((hi << 21 | lo >> 11) + 1) * 2^-53  ->  doubles in (0, 1], exact."""
    hi = np.asarray(hi_word, dtype=np.uint64)
    lo = np.asarray(lo_word, dtype=np.uint64)
    v = ((hi << np.uint64(21)) | (lo >> np.uint64(11))) + np.uint64(1)
    return v.astype(np.float64) * TWO_M53


def log_own(u) -> np.ndarray:
    """Natural log of u > 0 (normal numbers), fixed-order evaluation."""
    u = np.asarray(u, dtype=np.float64)
    f, e = np.frexp(u)  # u = f 2^e, f in [1/2, 1)
    small = f < SQRT_HALF
    f = np.where(small, f * 2.0, f)
    e = np.where(small, e - 1, e).astype(np.float64)
    s = (f - 1.0) / (f + 1.0)
    z = s * s
    p = np.full_like(s, ATANH_C[10])
    for k in range(9, -1, -1):
        p = p * z + ATANH_C[k]
    logf = (s + s) * p
    return e * LN2_HI + (logf + e * LN2_LO)


def sincos_2pi(u):
    """(cos(2 pi u), sin(2 pi u)) for u in [0, 1], fixed-order evaluation."""
    u = np.asarray(u, dtype=np.float64)
    x = u * 4.0
    q = np.rint(x)
    r = x - q
    phi = r * HALF_PI
    z = phi * phi
    ps = np.full_like(z, SIN_C[8])
    for k in range(7, -1, -1):
        ps = ps * z + SIN_C[k]
    sn = phi * ps
    pc = np.full_like(z, COS_C[9])
    for k in range(8, -1, -1):
        pc = pc * z + COS_C[k]
    cs = pc
    qi = q.astype(np.int64) & 3
    cos_out = np.select([qi == 0, qi == 1, qi == 2], [cs, -sn, -cs], sn)
    sin_out = np.select([qi == 0, qi == 1, qi == 2], [sn, cs, -sn], -cs)
    return cos_out, sin_out


def omega_block(seed: int, n: int, col0: int, w: int, batch: int = 0) -> np.ndarray:
    """Columns [col0, col0 + w) of the n x inf Gaussian sketch, float64,
    column-major (Fortran) n x w."""
    out = np.empty((n, w), dtype=np.float64, order="F")
    if n == 0 or w == 0:
        return out
    k0, k1 = key_from_seed(seed)
    npairs = (n + 1) // 2
    t = np.arange(npairs, dtype=np.uint64)[:, None]
    j = (np.arange(w, dtype=np.uint64) + np.uint64(col0))[None, :]
    x0, x1, x2, x3 = philox4x32_10(t, j, np.uint64(batch), np.uint64(0), k0, k1)
    u1 = uniforms53(x0, x1)
    u2 = uniforms53(x2, x3)
    rho = np.sqrt(-2.0 * log_own(u1))
    c, s = sincos_2pi(u2)
    even = rho * c
    odd = rho * s
    out[0::2, :] = even
    out[1::2, :] = odd[: n // 2, :]
    return out
