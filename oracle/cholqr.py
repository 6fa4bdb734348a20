"""orth(X): orthonormal basis of the column space of X (Section 2.4).

The paper computes orth with a packaged unpivoted QR.  The reading taken here
is Cholesky QR applied twice ("CholQR2"): with G = X^T X = T^T T
(T upper triangular with positive diagonal), Q = X T^{-1} is the Q factor of
the unique thin QR of X with positive diagonal R.  One pass loses
orthonormality in proportion to cond(X)^2 * u; the second pass, applied to
the output of the first, restores it to rounding level whenever
cond(X) < u^{-1/2}.

The paper assumes every sample block has full column rank (Proposition 4.1
assumes rank(A) >= s b).  For blocks that are numerically rank deficient the
reading taken is a Cholesky factorisation with column dropping, in natural
column order: column c is kept when its pivot, the part of G_cc left after
the kept earlier columns are projected out,

    d_c = G_cc - sum_{l kept, l < c} T_lc^2,

exceeds DROP_REL * max_j G_jj; otherwise column c is dropped (its row of T
is empty).  DROP_REL = 2^-40 keeps every column whose relative pivot norm is
above about 1e-6, well inside the range where CholQR2 is stable.  Kept
columns stay in their original order.

Parity pinned by: tests/test_oracle_cholqr.py (orthonormality, Q T = X,
agreement with numpy's Householder QR up to column signs, exact-rank inputs
dropping exactly the dependent columns, zero columns).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

DROP_REL = 2.0 ** -40


def chol_drop(G: np.ndarray, drop_rel: float = DROP_REL):
    """Upper Cholesky factor of the kept part of the Gram matrix G (w x w).

    Returns (T, kept): T is |kept| x |kept| upper triangular with positive
    diagonal and G[kept][:, kept] = T^T T up to rounding; kept is the list of
    kept column indices in increasing order.
    """
    G = np.asarray(G, dtype=np.float64)
    w = G.shape[0]
    if w == 0:
        return np.zeros((0, 0)), []
    gmax = float(np.max(np.diag(G)))
    thresh = drop_rel * gmax
    Tfull = np.zeros((w, w))
    kept: list[int] = []
    for c in range(w):
        # pivot: G_cc minus the squared entries of column c of the kept rows
        d = G[c, c] - float(np.dot(Tfull[kept, c], Tfull[kept, c])) if kept else G[c, c]
        if not (d > thresh) or gmax <= 0.0:
            continue
        tcc = np.sqrt(d)
        Tfull[c, c] = tcc
        if c + 1 < w:
            # row c of T right of the diagonal
            rest = G[c, c + 1:] - (Tfull[kept, c] @ Tfull[kept, c + 1:] if kept else 0.0)
            Tfull[c, c + 1:] = rest / tcc
        kept.append(c)
    T = Tfull[np.ix_(kept, kept)]
    return T, kept


def cholqr(X: np.ndarray, drop_rel: float = DROP_REL):
    """One Cholesky QR pass with dropping: returns (Q, kept) with
    Q = X[:, kept] T^{-1}."""
    X = np.asarray(X, dtype=np.float64)
    G = X.T @ X
    T, kept = chol_drop(G, drop_rel)
    if not kept:
        return np.zeros((X.shape[0], 0)), []
    Xk = X[:, kept]
    # Q T = X_k  <=>  T^T Q^T = X_k^T
    Q = scipy.linalg.solve_triangular(T, Xk.T, trans="T", lower=False).T
    return np.asfortranarray(Q), kept


def cholqr2(X: np.ndarray, drop_rel: float = DROP_REL):
    """orth(X) as two Cholesky QR passes.  Returns (Q, kept) where kept
    indexes the columns of X that survive both passes."""
    Q1, kept1 = cholqr(X, drop_rel)
    if not kept1:
        return Q1, []
    Q2, kept2 = cholqr(Q1, drop_rel)
    return Q2, [kept1[i] for i in kept2]
