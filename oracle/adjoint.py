"""Gradient of the fixed-sketch QB map A -> (Q, B).  Plain float64 CPU
reference; test infrastructure.

The map.  With the sketch fixed (the Gaussian columns of `seed`, Section
2.2 and Figure 4), the block width b, the number of blocks s and the number
of power iterations P fixed, the blocked scheme of Figures 4 and 6 is a
smooth function of A wherever every orthonormalisation sees a matrix of
full column rank (then orth(X) is the Q factor of the unique thin QR of X
with positive diagonal, Section 2.4):

    R = A
    for i = 1 .. s:
        Q_i = orth(R Omega_i)
        P times:  Z = orth(R^T Q_i);  Q_i = orth(R Z)          (Figure 6)
        i > 1:    Q_i = orth(Q_i - Qbar Qbar^T Q_i)           (Section 4.3)
        B_i = Q_i^T R;  R = R - Q_i B_i                       (Figure 4)
    Q = [Q_1 .. Q_s],  B = [B_1; .. ; B_s]

It is the forward of randqb_pb with eps = 0 and kmax = s b when no column is
dropped, which tests/test_oracle_adjoint.py checks.

The reference gradient.  For upstream gradients (dQ, dB) the vector-Jacobian
product dA = (dQ . dQ/dA + dB . dB/dA) is taken by reverse-mode automatic
differentiation of the forward above, written with torch CPU float64 matrix
products, Cholesky factorisation and triangular solves (library primitives;
orth is two Cholesky QR passes, as in cholqr.py, without dropping).

Parity pinned by tests/test_oracle_adjoint.py: central finite differences
of the numpy forward (randqb_pb) in random directions, the closed form
dA = G for L = <G, Q B> when s b = n and A has full column rank (then
Q B = A identically), and agreement of the forward with randqb_pb.
"""
from __future__ import annotations

import numpy as np
import torch

from .gaussian import omega_block


def orth_t(X: torch.Tensor) -> torch.Tensor:
    """Two Cholesky QR passes: X T1^{-1} T2^{-1} with G = T^T T (T upper).
    Raises when a Gram matrix is not positive definite (rank loss)."""
    for _ in range(2):
        L = torch.linalg.cholesky(X.T @ X)          # G = L L^T, T = L^T
        X = torch.linalg.solve_triangular(L, X.T, upper=False).T   # X L^{-T}
    return X


def qb_fixed(A: torch.Tensor, b: int, blocks: int, power_iters: int, seed: int):
    """The fixed-sketch QB map above on a float64 torch tensor (autograd-aware)."""
    m, n = A.shape
    if blocks * b > min(m, n):
        raise ValueError("s b must not exceed min(m, n)")
    R = A
    Qs, Bs = [], []
    for i in range(blocks):
        Om = torch.from_numpy(omega_block(seed, n, i * b, b)).to(A.dtype)
        Qi = orth_t(R @ Om)
        for _ in range(power_iters):
            Z = orth_t(R.T @ Qi)
            Qi = orth_t(R @ Z)
        if Qs:
            Qbar = torch.cat(Qs, dim=1)
            Qi = orth_t(Qi - Qbar @ (Qbar.T @ Qi))
        Bi = Qi.T @ R
        R = R - Qi @ Bi
        Qs.append(Qi)
        Bs.append(Bi)
    return torch.cat(Qs, dim=1), torch.cat(Bs, dim=0)


def qb_fixed_vjp(A: np.ndarray, dQ: np.ndarray, dB: np.ndarray, b: int, blocks: int,
                 power_iters: int, seed: int):
    """(Q, B, dA): the forward outputs and the gradient of
    <dQ, Q> + <dB, B> with respect to A, all float64 numpy."""
    At = torch.tensor(np.asarray(A, dtype=np.float64), requires_grad=True)
    Q, B = qb_fixed(At, b, blocks, power_iters, seed)
    L = (Q * torch.from_numpy(np.asarray(dQ, dtype=np.float64))).sum() + \
        (B * torch.from_numpy(np.asarray(dB, dtype=np.float64))).sum()
    (g,) = torch.autograd.grad(L, At)
    return Q.detach().numpy(), B.detach().numpy(), g.numpy()
