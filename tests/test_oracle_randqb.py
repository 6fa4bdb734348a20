"""Pins for the oracle's blocked QB driver (oracle/randqb.py).

Each test checks a fact the paper or the mathematics fixes, independent of
the oracle's own arithmetic:
  Proposition 4.1(a)   Qbar orthonormal
  Proposition 4.1(b)   A^(i) = A - Qbar Bbar  and  Bbar = Qbar^T A
  Proposition 4.1(c)   R(Qbar) = R(A [Omega_1 ... Omega_i])          (P = 0)
  Section 4.1    for a fixed Omega the projector does not depend on b
                 (b = k is Figure 3, b = 1 is Algorithm 1 with (4a)-(4c))
  eq. minerrors  error >= Eckart-Young optimum
  Section 3.2    error <= (1 + k/(p-1)) EY(k) (expectation; slack for one draw)
  Pythagoras     ||A - QB||^2 = ||A||^2 - ||B||^2
  closed forms   sigma * orthonormal input: residual sigma^2 (n - k) exactly
  brute force    tiny inputs reconstructed exactly, compared with LAPACK
"""
import math

import numpy as np
import pytest

import synth
from oracle import randqb_pb, STOP, STATUS
from oracle.randqb import sumsq, _stop_decision
from oracle.gaussian import omega_block
from oracle.checks import eckart_young, expectation_bound, orth_defect, unblocked_qb, eps_rank

U = 2.0 ** -53


def _fro(x):
    return float(np.linalg.norm(x))


@pytest.mark.parametrize("P", [0, 1])
def test_prop31_invariants(P):
    s = synth.spectrum("power", 200, p=2.0)
    A = synth.prescribed_svd(300, 200, s, 1, 2)
    nA = math.sqrt(sumsq(A))
    res = randqb_pb(A, 1e-3 * nA, 16, P, seed=4)
    k = res.k
    assert res.status == STATUS["OK"] and k % 16 == 0 and k > 0
    # (a) orthonormal
    assert orth_defect(res.Q) < 10 * U * math.sqrt(k) * 16
    # (b) residual and B identities
    assert _fro(res.R - (A - res.Q @ res.B)) < 20 * U * math.sqrt(res.blocks) * nA
    assert _fro(res.B - res.Q.T @ A) < 20 * U * nA
    # Pythagoras
    err2 = _fro(A - res.Q @ res.B) ** 2
    assert abs(err2 - (nA ** 2 - _fro(res.B) ** 2)) < (50 * U + orth_defect(res.Q)) * nA ** 2
    # tracked and direct indicators agree, and the stop happened at <= eps
    assert abs(res.E[-1] - res.D[-1]) < 1e-13 * nA ** 2
    assert res.D[-1] <= (1e-3 * nA) ** 2 < res.D[-2]
    # near-optimality: hard lower bound, soft expectation bound
    err = math.sqrt(err2)
    assert err >= eckart_young(s, k) * (1 - 1e-10)
    best = min(expectation_bound(s, k - p, p) for p in range(2, k - 1))
    assert err <= 10 * best


def test_prop31c_range_of_samples():
    s = synth.spectrum("exp", 120, scale=10.0)
    A = synth.prescribed_svd(160, 120, s, 3, 4)
    res = randqb_pb(A, 0.0, 8, 0, seed=11, kmax=40)
    Om = omega_block(11, 120, 0, 40)
    Y = A @ Om
    assert res.k == 40
    assert _fro(Y - res.Q @ (res.Q.T @ Y)) < 1e-10 * _fro(Y)


def test_blocked_equals_unblocked_projector():
    # Section 4.1: for a fixed Omega, Q Q^T (hence Q B) does not depend on b
    s = synth.spectrum("exp", 40, scale=4.0)
    A = synth.prescribed_svd(60, 40, s, 5, 6)
    k = 20
    Om = omega_block(21, 40, 0, k)
    Qu, Bu = unblocked_qb(A, Om)                  # Figure 3 with LAPACK QR
    nA = _fro(A)
    for b in (k, 10, 7, 1):
        res = randqb_pb(A, 0.0, b, 0, seed=21, kmax=k)
        assert res.k == k
        assert _fro(res.Q @ res.B - Qu @ Bu) < 1e-9 * nA, b
        P_blk = res.Q @ res.Q.T
        P_unb = Qu @ Qu.T
        assert _fro(P_blk - P_unb) < 1e-7, b


def test_sigma_orthonormal_input_has_closed_form_residual():
    m, n, sigma, b = 150, 100, 3.0, 16
    A = synth.orthonormal_scaled(m, n, sigma, seed=12)
    k0 = 40
    eps = sigma * math.sqrt(n - k0 + 0.5)
    res = randqb_pb(A, eps, b, 0, seed=1)
    # first block-granular k with sigma^2 (n - k) <= eps^2 is k = 48
    assert res.k == 48 and res.blocks == 3
    for i, (E, D) in enumerate(zip(res.E, res.D)):
        kk = b * (i + 1)
        assert abs(D - sigma ** 2 * (n - kk)) < 1e-12 * sigma ** 2 * n
        assert abs(E - sigma ** 2 * (n - kk)) < 1e-12 * sigma ** 2 * n


@pytest.mark.parametrize("r", [16, 48, 55])
@pytest.mark.parametrize("eps_rel", [0.0, 1e-10])
def test_exact_rank_stops_at_rank(r, eps_rel):
    A = synth.exact_rank(200, 120, r, seed=30 + r, cond=1e3)
    nA = _fro(A)
    res = randqb_pb(A, eps_rel * nA, 16, 0, seed=2)
    assert res.k == r
    assert _fro(A - res.Q @ res.B) < 1e-13 * nA
    if eps_rel == 0.0:
        assert res.status == STATUS["RANK_EXHAUSTED"] and res.stop_reason == STOP["EXHAUSTED"]
    else:
        assert res.status == STATUS["OK"]


def test_exact_rank_with_power_iterations():
    A = synth.exact_rank(200, 120, 37, seed=77, cond=1e2)
    res = randqb_pb(A, 0.0, 16, 1, seed=3)
    assert res.k == 37
    assert orth_defect(res.Q) < 1e-13


def test_zero_and_tolerance_above_norm():
    Z = np.zeros((10, 7), order="F")
    res = randqb_pb(Z, 0.0, 4, 0, seed=0)
    assert res.k == 0 and res.stop_reason == STOP["ZERO"] and res.status == STATUS["OK"]
    A = synth.exact_rank(30, 20, 5, seed=1)
    res = randqb_pb(A, _fro(A) * (1 + 1e-12), 4, 0, seed=0)
    assert res.k == 0 and res.stop_reason == STOP["ZERO"]


@pytest.mark.parametrize("m,n", [(1, 1), (3, 5), (8, 8), (8, 3), (2, 7)])
@pytest.mark.parametrize("b", [1, 2, 3, 8])
def test_brute_force_tiny(m, n, b):
    rng = np.random.default_rng(m * 100 + n * 10 + b)
    A = np.asfortranarray(rng.standard_normal((m, n)))
    r = min(m, n)
    res = randqb_pb(A, 0.0, b, 0, seed=b)
    assert res.k == r
    assert _fro(A - res.Q @ res.B) < 1e-13 * _fro(A)
    # the projector equals the one of Figure 3 with LAPACK's QR of A Omega
    Om = omega_block(b, n, 0, r)
    Qu, _ = np.linalg.qr(A @ Om)
    assert _fro(res.Q @ res.Q.T - Qu @ Qu.T) < 1e-10
    sv = np.linalg.svd(A, compute_uv=False)
    for kk in range(r + 1):
        assert eckart_young(sv, kk) <= _fro(A) + 1e-15


def test_kmax_and_rank_cap():
    s = synth.spectrum("power", 60, p=0.5)
    A = synth.prescribed_svd(80, 60, s, 7, 8)
    res = randqb_pb(A, 1e-12 * _fro(A), 16, 0, seed=1, kmax=40)
    assert res.k == 40 and res.status == STATUS["KMAX"] and res.widths == [16, 16, 8]
    res = randqb_pb(A, 0.0, 16, 0, seed=1)
    assert res.k == 60 and res.widths[-1] == 12


def test_power_iteration_improves_slow_decay():
    A = synth.paper_matrix2(200, 150, seed=21)
    errs = []
    for P in (0, 1, 2):
        res = randqb_pb(A, 0.0, 10, P, seed=5, kmax=50)
        errs.append(_fro(A - res.Q @ res.B))
    sv = np.linalg.svd(A, compute_uv=False)
    assert errs[1] < errs[0] and errs[2] <= errs[1] * 1.01
    assert errs[1] < 1.15 * eckart_young(sv, 50)


def test_kahan_close_to_optimal():
    A = synth.kahan(300, 0.99)
    sv = np.linalg.svd(A, compute_uv=False)
    res = randqb_pb(A, 0.0, 20, 1, seed=3, kmax=100)
    assert _fro(A - res.Q @ res.B) < 1.1 * eckart_young(sv, 100)


def test_stop_decision_bands():
    eps2, delta = 1.0, 0.1
    assert _stop_decision(0.85, 5.0, eps2, delta) == "TOL_TRACKED"
    assert _stop_decision(1.2, 0.0, eps2, delta) is None
    assert _stop_decision(1.05, 0.99, eps2, delta) == "TOL_DIRECT"
    assert _stop_decision(1.05, 1.0, eps2, delta) == "TOL_DIRECT"     # "at most eps"
    assert _stop_decision(0.95, 1.01, eps2, delta) is None


def test_invalid_arguments():
    A = np.ones((3, 3))
    for kw in ({"eps": -1.0, "b": 2}, {"eps": float("nan"), "b": 2}, {"eps": 0.1, "b": 0}):
        with pytest.raises(ValueError):
            randqb_pb(A, kw["eps"], kw["b"])
    with pytest.raises(ValueError):
        randqb_pb(A, 0.1, 2, power_iters=-1)
    bad = A.copy()
    bad[1, 1] = np.inf
    with pytest.raises(FloatingPointError):
        randqb_pb(bad, 0.1, 2)


def test_small_workload_rank_is_block_granular_above_ey_rank():
    w = synth.workload("exp40_2000x1000")
    A = synth.workload_matrix(w.name)
    s = w.singular_values()
    nA = math.sqrt(sumsq(A))
    eps = w.eps_rel * nA
    res = randqb_pb(A, eps, w.b, 0, seed=w.seed_omega)
    assert res.k % w.b == 0
    assert res.k >= eps_rank(s, eps)                  # cannot beat Eckart-Young
    assert math.sqrt(res.D[-1]) <= eps < math.sqrt(res.D[-2])
    assert orth_defect(res.Q) < 1e-13
    assert _fro(A - res.Q @ res.B) <= eps * (1 + 1e-10)
