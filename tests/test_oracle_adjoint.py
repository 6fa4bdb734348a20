"""Pins of the gradient oracle (oracle/adjoint.py) against what does not
depend on it: central finite differences of the numpy forward (randqb_pb),
the closed form of a full-rank case, and the forward itself."""
import numpy as np
import pytest

import synth
from oracle import randqb_pb
from oracle.adjoint import qb_fixed_vjp


def forward_np(A, b, blocks, P, seed):
    r = randqb_pb(A, 0.0, b, P, seed, kmax=blocks * b)
    assert r.k == blocks * b and r.blocks == blocks
    return r.Q, r.B


def loss_np(A, dQ, dB, b, blocks, P, seed):
    Q, B = forward_np(A, b, blocks, P, seed)
    return float(np.sum(Q * dQ) + np.sum(B * dB))


def case(m, n, seed=3):
    s = np.exp(-np.arange(1, min(m, n) + 1) / 10.0)
    A = synth.prescribed_svd(m, n, s, seed, seed + 1)
    g = np.random.default_rng(seed + 7)
    return A, g


@pytest.mark.parametrize("P", [0, 1])
def test_forward_matches_randqb(P):
    A, g = case(70, 50)
    Q, B, _ = qb_fixed_vjp(A, np.zeros((70, 24)), np.zeros((24, 50)), 8, 3, P, 11)
    Qr, Br = forward_np(A, 8, 3, P, 11)
    assert np.linalg.norm(Q @ B - Qr @ Br) <= 1e-12 * np.linalg.norm(A)
    assert np.linalg.norm(Q - Qr) <= 1e-11


@pytest.mark.parametrize("P", [0, 1])
@pytest.mark.parametrize("upstream", ["QB", "Q", "B"])
def test_gradient_matches_central_differences(P, upstream):
    m, n, b, s = 60, 40, 8, 3
    A, g = case(m, n)
    dQ = g.standard_normal((m, b * s)) if upstream in ("QB", "Q") else np.zeros((m, b * s))
    dB = g.standard_normal((b * s, n)) if upstream in ("QB", "B") else np.zeros((b * s, n))
    _, _, dA = qb_fixed_vjp(A, dQ, dB, b, s, P, 5)
    h = 1e-5 * np.linalg.norm(A)
    for t in range(3):
        E = g.standard_normal((m, n))
        E /= np.linalg.norm(E)
        fd = (loss_np(A + h * E, dQ, dB, b, s, P, 5) - loss_np(A - h * E, dQ, dB, b, s, P, 5)) / (2 * h)
        ad = float(np.sum(dA * E))
        assert abs(fd - ad) <= 1e-7 * np.linalg.norm(dA), (t, fd, ad)


def test_closed_form_full_rank():
    """s b = n and rank(A) = n: Q B = Q Q^T A = A for every A nearby, so
    the gradient of <G, Q B> is G itself."""
    m, n, b = 50, 32, 8
    A, g = case(m, n, seed=9)
    G = g.standard_normal((m, n))
    for P in (0, 1):
        Q, B = forward_np(A, b, n // b, P, 2)
        _, _, dA = qb_fixed_vjp(A, G @ B.T, Q.T @ G, b, n // b, P, 2)
        assert np.linalg.norm(dA - G) <= 1e-9 * np.linalg.norm(G)


def test_loss_gradient_is_not_the_trivial_one():
    """With s b < n the projector moves with A: the gradient of <G, Q B>
    differs from the fixed-projector term Q Q^T G by O(1)."""
    m, n, b, s = 60, 40, 8, 2
    A, g = case(m, n)
    G = g.standard_normal((m, n))
    Q, B = forward_np(A, b, s, 0, 4)
    _, _, dA = qb_fixed_vjp(A, G @ B.T, Q.T @ G, b, s, 0, 4)
    assert np.linalg.norm(dA - Q @ (Q.T @ G)) > 1e-3 * np.linalg.norm(G)
