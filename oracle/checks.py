"""Quantities the paper fixes, used to pin the oracle and to check results.

  eckart_young(s, k)     optimal rank-k Frobenius error (eq. minerrors,
                         Section 2.2): sqrt(sum_{j>k} s_j^2)
  expectation_bound(s, k, p)  (1 + k/(p-1)) * EY(k) for a sketch with k + p
                         columns (Section 3.2, quoting Halko-Martinsson-Tropp
                         Thm. 10.5; the paper's factor has no square root,
                         a weaker but still valid bound, and is taken as
                         printed)
  eps_rank(s, eps)       smallest k with EY(k) <= eps
  orth_defect(Q)         ||Q^T Q - I||_F  (Proposition 4.1(a))
  unblocked_qb(A, Om)    Figure 3 (randQB): Q = orth(A Omega), B = Q^T A via
                         Householder QR (numpy), for the blocked-vs-unblocked
                         identity of Section 4.1

Parity pinned by tests/test_oracle_checks.py: EY(k) against the error of
the rank-k truncation rebuilt from numpy's SVD factors for every k, and no
orthonormal rank-k basis doing better; eps_rank as the smallest such k
(ties included); expectation_bound at hand-computed values and above the
Monte-Carlo mean error of randQB; planted off-by-one slips fail them.
"""
from __future__ import annotations

import math

import numpy as np


def eckart_young(s, k: int) -> float:
    s = np.sort(np.asarray(s, dtype=np.float64))[::-1]
    tail = s[k:]
    return math.sqrt(math.fsum((tail * tail).tolist()))


def expectation_bound(s, k: int, p: int) -> float:
    assert p >= 2
    return (1.0 + k / (p - 1.0)) * eckart_young(s, k)


def eps_rank(s, eps: float) -> int:
    s = np.sort(np.asarray(s, dtype=np.float64))[::-1]
    for k in range(len(s) + 1):
        if eckart_young(s, k) <= eps:
            return k
    return len(s)


def orth_defect(Q: np.ndarray) -> float:
    k = Q.shape[1]
    return float(np.linalg.norm(Q.T @ Q - np.eye(k)))


def unblocked_qb(A: np.ndarray, Om: np.ndarray):
    Q, _ = np.linalg.qr(A @ Om)
    return Q, Q.T @ A
