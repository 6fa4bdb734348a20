"""Pins of oracle/postprocess.py (Section 3.3): the low-rank SVD from QB and
the partial column-pivoted QR (Householder with column pivoting).

Pivoted QR is pinned against LAPACK (scipy's dgeqp3) on generic inputs and
against the defining properties: B P = Q_tilde R, Q_tilde orthogonal, R
upper trapezoidal, and at every step the pivot column has the largest norm
of the remaining block (|R_jj|^2 >= sum_{i>=j} R_il^2 for l > j); the
reflector's sign convention by a 2 x 2 closed form.  The SVD step is
LAPACK's; the pins check the assembly U = Q U_hat against the SVD of the
product Q B.
"""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import randqb_pb
from oracle.postprocess import householder, pivoted_qr, qb_pivoted_qr, qb_svd


def test_householder_closed_forms():
    r = np.random.default_rng(1)
    for n in (1, 2, 7):
        x = r.standard_normal(n)
        v, tau, beta = householder(x)
        Hx = x - tau * v * (v @ x)
        e = np.zeros(n)
        e[0] = beta
        assert np.allclose(Hx, e, atol=1e-14) and v[0] == 1.0
        assert abs(abs(beta) - np.linalg.norm(x)) < 1e-14
        assert np.sign(beta) == -np.sign(x[0])
    v, tau, beta = householder(np.zeros(4))
    assert tau == 0.0 and beta == 0.0


def test_pivoted_qr_2x2_closed_form():
    Qt, R, perm = pivoted_qr(np.array([[3.0, 1.0], [4.0, 2.0]]))
    assert list(perm) == [0, 1]
    assert R[0, 0] == pytest.approx(-5.0, abs=1e-15)
    assert R[0, 1] == pytest.approx(-(3 * 1 + 4 * 2) / 5.0, abs=1e-15)
    assert abs(R[1, 1]) == pytest.approx(abs(3 * 2 - 4 * 1) / 5.0, abs=1e-15)
    # the larger column moves first
    Qt, R, perm = pivoted_qr(np.array([[1.0, 3.0], [2.0, 4.0]]))
    assert list(perm) == [1, 0] and R[0, 0] == pytest.approx(-5.0, abs=1e-15)


def _check_cpqr(B, Qt, R, perm):
    k, n = B.shape
    nB = np.linalg.norm(B)
    assert sorted(perm) == list(range(n))
    assert np.linalg.norm(B[:, perm] - Qt @ R) < 1e-13 * nB
    assert np.linalg.norm(Qt.T @ Qt - np.eye(k)) < 1e-13
    assert np.all(np.tril(R, -1) == 0.0)
    for j in range(min(k, n)):
        trail = np.sum(R[j:, j + 1:] ** 2, axis=0)
        assert np.all(R[j, j] ** 2 >= trail * (1 - 1e-12) - 1e-28)


@pytest.mark.parametrize("k,n", [(40, 70), (70, 40), (33, 33), (1, 9), (9, 1)])
def test_pivoted_qr_properties_and_lapack(k, n):
    B = np.random.default_rng(k * n).standard_normal((k, n))
    Qt, R, perm = pivoted_qr(B)
    _check_cpqr(B, Qt, R, perm)
    R2, P2 = scipy.linalg.qr(B, mode="r", pivoting=True)
    r = min(k, n)
    assert list(perm[:r]) == list(P2[:r])
    assert np.allclose(np.abs(np.diag(R)[:r]), np.abs(np.diag(R2)[:r]), rtol=1e-12)


def test_pivoted_qr_rank_deficient():
    r = np.random.default_rng(5)
    B = r.standard_normal((30, 7)) @ r.standard_normal((7, 50))
    Qt, R, perm = pivoted_qr(B)
    _check_cpqr(B, Qt, R, perm)
    d = np.abs(np.diag(R))
    assert np.all(d[:7] > 1e-3 * d[0]) and np.all(d[7:] < 1e-13 * d[0])


def test_qb_svd_and_qr_from_a_qb_run():
    w = synth.workload("exp40_2000x1000")
    A = synth.workload_matrix(w.name)
    nA = np.linalg.norm(A)
    res = randqb_pb(A, 1e-6 * nA, w.b, 0, w.seed_omega)
    U, s, V = qb_svd(res.Q, res.B)
    QB = res.Q @ res.B
    assert np.linalg.norm(U * s @ V.T - QB) < 1e-13 * nA
    assert np.linalg.norm(U.T @ U - np.eye(res.k)) < 1e-12
    assert np.all(np.diff(s) <= 0)
    assert np.allclose(s, np.linalg.svd(QB, compute_uv=False)[:res.k], rtol=0, atol=1e-13 * s[0])
    # the leading singular values are those of A (exp(-j/40) spectrum)
    sA = synth.spectrum("exp", 1000, scale=40.0)
    assert np.allclose(s[:200], sA[:200], rtol=1e-8)
    Qh, R, perm = qb_pivoted_qr(res.Q, res.B)
    assert np.linalg.norm(Qh @ R - QB[:, perm]) < 1e-13 * nA
    assert np.linalg.norm(Qh.T @ Qh - np.eye(res.k)) < 1e-12
