"""Pins for orth (oracle/cholqr.py): Cholesky QR applied twice with column
dropping.  Checked against LAPACK (numpy's Cholesky and Householder QR) and
against the defining properties of orth (Section 2.4): orthonormal columns
spanning the range of X."""
import numpy as np
import pytest

from oracle.cholqr import chol_drop, cholqr, cholqr2
from oracle.checks import orth_defect

U = 2.0 ** -53


def _with_cond(m, w, cond, seed):
    rng = np.random.default_rng(seed)
    u, _ = np.linalg.qr(rng.standard_normal((m, w)))
    v, _ = np.linalg.qr(rng.standard_normal((w, w)))
    s = np.logspace(0, -np.log10(cond), w)
    return (u * s) @ v.T


def test_chol_drop_matches_lapack_on_spd():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((50, 12))
    G = X.T @ X
    T, kept = chol_drop(G)
    assert kept == list(range(12))
    L = np.linalg.cholesky(G)
    assert np.allclose(T, L.T, rtol=1e-13, atol=1e-13 * np.abs(L).max())


def test_chol_drop_diagonal_with_zero():
    T, kept = chol_drop(np.diag([4.0, 0.0, 9.0]))
    assert kept == [0, 2]
    assert np.array_equal(T, np.diag([2.0, 3.0]))
    T, kept = chol_drop(np.zeros((3, 3)))
    assert kept == [] and T.shape == (0, 0)


@pytest.mark.parametrize("cond", [1.0, 1e3, 1e6])
def test_cholqr2_orthonormal_and_spanning(cond):
    X = _with_cond(400, 24, cond, seed=4)
    Q, kept = cholqr2(X)
    assert kept == list(range(24))
    assert orth_defect(Q) < 20 * U * 24
    # same range: X = Q Q^T X
    assert np.linalg.norm(X - Q @ (Q.T @ X)) < 50 * U * np.linalg.norm(X) * cond ** 0.5
    # equals the Householder Q up to column signs (unique thin QR, positive diag R)
    Qh, Rh = np.linalg.qr(X)
    Qh = Qh * np.sign(np.diag(Rh))[None, :]
    assert np.linalg.norm(Q - Qh) < 1e-14 * cond * 24


def test_single_pass_loses_orthonormality_on_ill_conditioned_input():
    X = _with_cond(400, 24, 1e6, seed=5)
    Q1, _ = cholqr(X)
    Q2, _ = cholqr2(X)
    assert orth_defect(Q1) > 1e3 * orth_defect(Q2)


def test_dependent_columns_are_dropped():
    rng = np.random.default_rng(6)
    x = rng.standard_normal((100, 4))
    X = np.column_stack([x[:, 0], x[:, 1], x[:, 0] + 2 * x[:, 1], x[:, 2], np.zeros(100), x[:, 3]])
    Q, kept = cholqr2(X)
    assert kept == [0, 1, 3, 5]
    assert orth_defect(Q) < 1e-14
    assert np.linalg.norm(X - Q @ (Q.T @ X)) < 1e-13 * np.linalg.norm(X)


def test_exact_rank_block_keeps_rank_columns():
    rng = np.random.default_rng(8)
    r, w = 7, 20
    X = rng.standard_normal((300, r)) @ rng.standard_normal((r, w))
    Q, kept = cholqr2(X)
    assert kept == list(range(r))
    assert orth_defect(Q) < 1e-14


def test_drop_threshold_is_relative():
    rng = np.random.default_rng(9)
    X = rng.standard_normal((200, 3))
    for scale in (1e-150, 1.0, 1e150):
        Q, kept = cholqr2(X * scale)
        assert kept == [0, 1, 2]
        assert orth_defect(Q) < 1e-14
    # a column 1e-7 outside the span of the others is dropped, 1e-5 is kept
    base = X[:, 0] + X[:, 1]
    perp = X[:, 2] - X[:, :2] @ np.linalg.lstsq(X[:, :2], X[:, 2], rcond=None)[0]
    perp /= np.linalg.norm(perp)
    for eta, want in ((1e-7, [0, 1]), (1e-5, [0, 1, 2])):
        Y = np.column_stack([X[:, 0], X[:, 1], base + eta * np.linalg.norm(base) * perp])
        assert cholqr2(Y)[1] == want
