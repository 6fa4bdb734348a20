"""Standard factorisations from a QB factorisation (Section 3.3): the low-rank
SVD (Section 3.3.1) and the partial column-pivoted QR (Section 3.3.2).
Plain float64 CPU reference; test infrastructure.

Low-rank SVD: with B = U_hat D V_hat^T the full SVD of the small k x n
matrix B, A ~ Q B = (Q U_hat) D V_hat^T.  The SVD of B is taken from LAPACK
(numpy), a library primitive; the singular values come out in
non-increasing order.

Partial pivoted QR: B P = Q_tilde R by Householder QR with column pivoting
(Businger and Golub): at step j the remaining column of largest 2-norm,
restricted to rows j.., is swapped to position j and a reflector
H_j = I - tau v v^T with v_0 = 1 zeroes it below the diagonal; then
A P ~ (Q Q_tilde) R.  Readings of points the paper leaves open:
  * column norms are recomputed from the current entries at every step
    (no downdating), each as a plain sum of squares;
  * a tie in the largest norm goes to the smallest column index;
  * the reflector maps x to beta e_1 with beta = -sign(x_0) ||x|| (sign(0)
    taken as +1), so R_jj has the opposite sign of the pivot entry; a zero
    column gets tau = 0 (H = I);
  * Q_tilde is formed as H_1 H_2 ... H_r applied to the leading k columns of
    the identity.
"""
from __future__ import annotations

import numpy as np


def qb_svd(Q: np.ndarray, B: np.ndarray):
    """Low-rank SVD factors of Q B: U (m x k), s (k), V (n x k), s sorted
    non-increasing, Q B = U diag(s) V^T."""
    Q = np.asarray(Q, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    Uh, s, Vt = np.linalg.svd(B, full_matrices=False)
    return Q @ Uh, s, Vt.T


def householder(x: np.ndarray):
    """(v, tau, beta) with (I - tau v v^T) x = beta e_1 and v[0] = 1."""
    x = np.asarray(x, dtype=np.float64)
    nrm = float(np.sqrt(np.sum(x * x)))
    v = np.zeros_like(x)
    if x.size == 0 or nrm == 0.0:
        if x.size:
            v[0] = 1.0
        return v, 0.0, 0.0
    beta = -nrm if x[0] >= 0.0 else nrm
    v0 = x[0] - beta
    v[0] = 1.0
    v[1:] = x[1:] / v0
    tau = (beta - x[0]) / beta
    return v, tau, beta


def pivoted_qr(B: np.ndarray):
    """Householder QR with column pivoting of the k x n matrix B.

    Returns (Qt, R, perm): Qt (k x k) orthogonal, R (k x n) upper
    trapezoidal, perm (n) with B[:, perm] = Qt @ R."""
    W = np.array(B, dtype=np.float64, copy=True)
    k, n = W.shape
    perm = np.arange(n)
    steps = min(k, n)
    vs, taus = [], []
    for j in range(steps):
        norms = np.sum(W[j:, j:] * W[j:, j:], axis=0)
        p = j + int(np.argmax(norms))          # first index of the maximum
        if p != j:
            W[:, [j, p]] = W[:, [p, j]]
            perm[[j, p]] = perm[[p, j]]
        v, tau, beta = householder(W[j:, j])
        if tau != 0.0:
            W[j:, j + 1:] -= tau * np.outer(v, v @ W[j:, j + 1:])
            W[j, j] = beta
            W[j + 1:, j] = 0.0
        vs.append(v)
        taus.append(tau)
    Qt = np.eye(k)
    for j in reversed(range(steps)):
        if taus[j] != 0.0:
            v = vs[j]
            Qt[j:, :] -= taus[j] * np.outer(v, v @ Qt[j:, :])
    R = np.triu(W)
    return Qt, R, perm


def qb_pivoted_qr(Q: np.ndarray, B: np.ndarray):
    """A P ~ Q_hat R from A ~ Q B: Q_hat = Q Q_tilde (m x k)."""
    Qt, R, perm = pivoted_qr(B)
    return np.asarray(Q, dtype=np.float64) @ Qt, R, perm
