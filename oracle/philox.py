"""Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11), written from its published definition.

The paper draws its sketch with Matlab's randn (Figures 3, 4 and 6); it does
not fix a generator.  This library fixes one counter-based generator so that the
sketch is a pure function of (seed, row, global column) and can be reproduced
bit for bit by the CPU oracle and by the GPU.

One round maps the counter (c0, c1, c2, c3) with round key (k0, k1) to
    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))
with the 32x32->64 bit products split into high and low words.  Between
rounds the key is advanced by the Weyl constants (W0, W1).  Ten rounds.

Pinned by: tests/test_oracle_philox.py against rocRAND's independent
philox4x32_10 engine (run on the host), plus avalanche / uniformity checks.
"""
from __future__ import annotations

import numpy as np

# multipliers and Weyl key increments of Philox4x32 (SC'11, Table 2 / Sec. 5)
M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Apply ten Philox4x32 rounds elementwise.

    All arguments are integers or integer arrays holding 32-bit values
    (broadcast together).  Returns a tuple of four uint32 arrays.
    """
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & _MASK for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & _MASK
            k1 = (k1 + W1) & _MASK
        p0 = M0 * c0  # < 2^64, exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def key_from_seed(seed: int):
    """64-bit seed -> Philox key words (low word, high word)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32
