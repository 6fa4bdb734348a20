"""Blocked adaptive randomized QB with a Frobenius tolerance: randQB_b
(Figure 4, Sections 4.1-4.3) and its power-iteration form randQB_pb
(Figure 6, Section 5.2).  Plain float64 CPU reference; test infrastructure.

For i = 1, 2, ... (A is overwritten by the residual A^(i), eq. def3):
  (2)  Omega_i = columns [k, k+w) of the Gaussian sketch     (gaussian.py)
  (3)  Q_i = orth(A Omega_i)                                   (cholqr.py)
  (4-7) P times: Q_i = orth(A^T Q_i); Q_i = orth(A Q_i)         (Fig. 6)
  (3') Q_i = orth(Q_i - Qbar Qbar^T Q_i)   re-projection, Section 4.3
  (4)  B_i = Q_i^T A
  (5)  A = A - Q_i B_i
  (6)  stop once the residual norm is at most eps (Section 4.2)
Output Q = [Q_1 ... Q_s], B = [B_1; ...; B_s].

Readings of points the paper leaves open (each also listed in the design
notes of the repository):
  * block width: w = min(b, kcap - k), kcap = min(kmax, min(m, n)), so the
    rank never exceeds min(m, n);
  * orth drops numerically dependent columns (cholqr.py); a block keeps
    w' <= w columns; when w' = 0 nothing is added and the run stops
    ("exhausted");
  * stopping quantity: the paper tests the norm of the updated A directly
    (Section 4.2 and step (6)).  Proposition 4.1 (a),(b) with Pythagoras
    gives ||A^(i)||^2 = ||A||^2 - sum_j ||B_j||^2, which is tracked as E_i.
    E_i cancels catastrophically near eps^2 when eps is close to
    sqrt(u)||A||, so the rule is hybrid: stop when E_i <= eps^2 - delta;
    continue when E_i > eps^2 + delta; otherwise stop iff the direct
    D_i = ||A^(i)||^2 <= eps^2, with delta = 1e-13 ||A||^2;
  * "at most eps" (non-strict), as in Algorithm 1 and Section 4.2; the same
    test is applied before the first block (k = 0 when ||A|| <= eps);
  * when the residual has fallen to the rounding level of the downdate,
    D_i <= (2^-46 ||A||)^2, further blocks would only sample rounding noise
    and the run stops ("exhausted").

Parity pinned by tests/test_oracle_randqb.py: orthonormality of Qbar
(Proposition 4.1(a)), residual identity A^(i) = A - Qbar Bbar and Bbar = Qbar^T A
(Proposition 4.1(b)), range identity (Proposition 4.1(c)), independence of the projector
from the block size for a fixed sketch (Section 4.1), Eckart-Young lower
bound and the expectation bound (Section 3.2), deterministic residuals of
sigma * orthonormal inputs, exact-rank inputs, brute force against LAPACK on
tiny inputs, and the rank of the 2000 x 1000 exp(-j/40) workload.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .gaussian import omega_block
from .cholqr import cholqr2, DROP_REL
from .intsplit import sample_exact

STOP = {
    "TOL_TRACKED": 0,
    "TOL_DIRECT": 1,
    "RANK_CAP": 2,
    "EXHAUSTED": 3,
    "KMAX": 4,
    "ZERO": 5,
}
STATUS = {"OK": 0, "KMAX": 1, "RANK_EXHAUSTED": 2}

DELTA_REL = 1e-13          # hybrid band half-width, relative to ||A||_F^2
FLOOR_REL = 2.0 ** -46     # rounding floor of the residual, relative to ||A||_F


def sumsq(X: np.ndarray) -> float:
    """||X||_F^2: per-column pairwise sums, then an exactly rounded sum."""
    X = np.asarray(X, dtype=np.float64)
    if X.size == 0:
        return 0.0
    cols = np.sum(X * X, axis=0)
    return math.fsum(cols.tolist())


@dataclass
class QBResult:
    Q: np.ndarray              # m x k, orthonormal columns
    B: np.ndarray              # k x n
    k: int
    R: np.ndarray              # final residual A - Q B (the overwritten A)
    status: int
    stop_reason: int
    normA2: float              # ||A||_F^2
    E: list = field(default_factory=list)      # tracked ||A||^2 - sum ||B_j||^2 per block
    D: list = field(default_factory=list)      # direct ||A^(i)||_F^2 per block
    widths: list = field(default_factory=list)  # kept columns per block
    blocks: int = 0


def _stop_decision(E: float, D: float, eps2: float, delta: float):
    if E <= eps2 - delta:
        return "TOL_TRACKED"
    if E > eps2 + delta:
        return None
    return "TOL_DIRECT" if D <= eps2 else None


def randqb_pb(A: np.ndarray, eps: float, b: int, power_iters: int = 0, seed: int = 0,
              kmax: int | None = None, omega_fn=None, drop_rel: float = DROP_REL,
              reorth: bool = True, power_orth: bool = True,
              max_blocks: int | None = None, sample: str = "f64") -> QBResult:
    """Blocked adaptive QB of A (m x n) to Frobenius tolerance eps.

    omega_fn(n, col0, w) -> n x w, if given, replaces the Philox sketch (used
    by tests that need a prescribed Omega).  reorth=False skips step (3')
    (Section 4.3).  power_orth=False skips the orthonormalisation between
    applications of A and A^T (the variant examined in Sections 5.4 and
    6.4): Y = (A A^T)^P A Omega_i, then Q_i = orth(Y).  max_blocks=1 with
    b = l is the unblocked scheme: randQB (Figure 3) for P = 0 and randQB_p
    (Figure 5) for P >= 1, one pass of width l with no continuation when
    orth drops columns; the run then ends with stop reason KMAX unless the
    tolerance was met.  sample="int8x8" forms the sample of step (3) as the
    exact-range product of intsplit.py (the residual on a fixed-point grid
    times the sketch on a 1/16 grid, exponent from the previous block's
    ||A^(i-1)||_F^2); the products of the power iterations stay float64.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    r = min(m, n)
    if not (np.isfinite(eps) and eps >= 0) or b < 1 or power_iters < 0:
        raise ValueError("invalid argument")
    if max_blocks is not None and max_blocks < 1:
        raise ValueError("invalid argument")
    if sample not in ("f64", "int8x8"):
        raise ValueError("invalid argument")
    if not np.all(np.isfinite(A)):
        raise FloatingPointError("non-finite entry in A")
    kcap = r if kmax is None else min(int(kmax), r)
    if omega_fn is None:
        def omega_fn(nn, col0, w):
            return omega_block(seed, nn, col0, w)

    sA = sumsq(A)
    eps2 = float(eps) * float(eps)
    delta = DELTA_REL * sA
    floor2 = (FLOOR_REL * math.sqrt(sA)) ** 2
    Qcols: list[np.ndarray] = []
    Brows: list[np.ndarray] = []
    res = QBResult(Q=np.zeros((m, 0)), B=np.zeros((0, n)), k=0, R=A.copy(order="F"),
                   status=STATUS["OK"], stop_reason=STOP["ZERO"], normA2=sA)
    if sA <= eps2:
        return res

    R = res.R
    k = 0
    sigB_parts: list[float] = []
    reason = None
    while True:
        w = min(b, kcap - k)
        if w == 0:
            reason = "KMAX" if kcap < r else "RANK_CAP"
            break
        # (2)-(3): sample the current residual and orthonormalise
        Om = omega_fn(n, k, w)
        if sample == "int8x8":
            Y = sample_exact(R, Om, res.D[-1] if res.D else sA)
        else:
            Y = R @ Om
        if power_orth:
            Qi, kept = cholqr2(Y, drop_rel)
            # (4)-(7): power iterations on the residual, orth after every product
            for _ in range(power_iters):
                if not kept:
                    break
                Z, kz = cholqr2(R.T @ Qi, drop_rel)
                if not kz:
                    kept = []
                    break
                Qi, kq = cholqr2(R @ Z, drop_rel)
                kept = kq
        else:
            for _ in range(power_iters):
                Y = R @ (R.T @ Y)
            Qi, kept = cholqr2(Y, drop_rel)
        # (3') / (8): re-project against the basis found so far, then orth
        if kept and reorth and k > 0:
            Qbar = np.hstack(Qcols)
            Qi = Qi - Qbar @ (Qbar.T @ Qi)
            Qi, kr = cholqr2(Qi, drop_rel)
            kept = kr
        wk = len(kept)
        if wk == 0:
            reason = "EXHAUSTED"
            break
        # (4) B_i = Q_i^T A^(i-1);  (5) downdate
        Bi = Qi.T @ R
        R -= Qi @ Bi
        Qcols.append(Qi)
        Brows.append(Bi)
        k += wk
        res.blocks += 1
        res.widths.append(wk)
        sigB_parts.append(sumsq(Bi))
        E = sA - math.fsum(sigB_parts)
        D = sumsq(R)
        res.E.append(E)
        res.D.append(D)
        # (6) stopping rule
        reason = _stop_decision(E, D, eps2, delta)
        if reason is not None:
            break
        if D <= floor2:
            reason = "EXHAUSTED"
            break
        if max_blocks is not None and res.blocks >= max_blocks:
            reason = "KMAX"
            break
        if k >= kcap:
            reason = "KMAX" if kcap < r else "RANK_CAP"
            break

    res.Q = np.asfortranarray(np.hstack(Qcols)) if Qcols else np.zeros((m, 0))
    res.B = np.asfortranarray(np.vstack(Brows)) if Brows else np.zeros((0, n))
    res.k = k
    res.stop_reason = STOP[reason]
    if reason in ("TOL_TRACKED", "TOL_DIRECT", "ZERO"):
        res.status = STATUS["OK"]
    elif reason == "KMAX":
        res.status = STATUS["KMAX"]
    else:
        res.status = STATUS["RANK_EXHAUSTED"]
    return res
