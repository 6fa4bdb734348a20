"""Pins of the bound helpers in oracle/checks.py, each against something
other than its own formula:

  eckart_young(s, k)  ||A - A_k||_F with A_k the rank-k truncation rebuilt
                      from numpy's SVD factors (eq. minerrors, Section 2.2),
                      for every k of small random matrices; no rank-k
                      projection of A does better (brute force over random
                      and perturbed-optimal bases)
  eps_rank(s, eps)    the smallest k whose truncation error, rebuilt from
                      the SVD factors, is at most eps (ties included)
  expectation_bound   hand-computed values of (1 + k/(p-1)) EY(k)
                      (Section 3.2), and a Monte-Carlo mean of the error of
                      randQB with k + p Gaussian columns below it

Planted off-by-one and formula slips in copies of checks.py fail them.
"""
import math

import numpy as np
import pytest

from oracle import checks
from tests.test_oracle_mutations import mutant


def _svd_truncation_errors(A):
    """||A - A_k||_F for k = 0..r, each from the explicit rank-k matrix."""
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    out = []
    for k in range(len(s) + 1):
        Ak = (U[:, :k] * s[:k]) @ Vt[:k, :]
        out.append(float(np.linalg.norm(A - Ak)))
    return s, out


def _cases():
    rng = np.random.default_rng(1503)
    yield rng.standard_normal((12, 9))
    yield rng.standard_normal((7, 11))
    g = rng.standard_normal((10, 10))
    yield g @ np.diag(np.logspace(0, -5, 10)) @ rng.standard_normal((10, 10))


def _ey_pins_hold(ck) -> bool:
    for A in _cases():
        s, errs = _svd_truncation_errors(A)
        shuffled = np.random.default_rng(3).permutation(s)   # unsorted input is sorted
        for k, e in enumerate(errs):
            if abs(ck.eckart_young(shuffled, k) - e) > 1e-12 * (1.0 + errs[0]):
                return False
    return True


def test_eckart_young_matches_svd_truncation():
    assert _ey_pins_hold(checks)


def test_eckart_young_special_values():
    s = np.array([3.0, 2.0, 1.0, 0.5])
    assert checks.eckart_young(s, 0) == pytest.approx(math.sqrt(9 + 4 + 1 + 0.25), rel=1e-15)
    assert checks.eckart_young(s, 1) == pytest.approx(math.sqrt(4 + 1 + 0.25), rel=1e-15)
    assert checks.eckart_young(s, 3) == pytest.approx(0.5, rel=1e-15)
    assert checks.eckart_young(s, 4) == 0.0


def test_no_rank_k_projection_beats_eckart_young():
    """eq. minerrors: for every orthonormal Q with k columns,
    ||A - Q Q^T A|| >= EY(k); random bases and small perturbations of the
    optimal one (which reaches EY(k) exactly)."""
    rng = np.random.default_rng(77)
    A = rng.standard_normal((15, 10)) @ np.diag(np.logspace(0, -3, 10))
    U, s, _ = np.linalg.svd(A, full_matrices=False)
    for k in range(1, 10):
        ey = checks.eckart_young(s, k)
        best = float(np.linalg.norm(A - U[:, :k] @ (U[:, :k].T @ A)))
        assert best == pytest.approx(ey, rel=1e-10, abs=1e-14)
        for t in range(20):
            X = U[:, :k] + (0.3 if t < 10 else 1e-3) * rng.standard_normal((15, k))
            Q, _ = np.linalg.qr(X)
            assert float(np.linalg.norm(A - Q @ (Q.T @ A))) >= ey * (1 - 1e-12)


def _eps_rank_pins_hold(ck) -> bool:
    for A in _cases():
        s, errs = _svd_truncation_errors(A)
        for k in range(len(s)):
            e = ck.eckart_young(s, k)       # a tie: the truncation error itself
            want = min(j for j, ej in enumerate(errs) if ej <= e * (1 + 1e-12))
            if ck.eps_rank(s, e) != want:
                return False
            below = 0.5 * (errs[k] + errs[k + 1])
            want = min(j for j, ej in enumerate(errs) if ej <= below)
            if ck.eps_rank(s, below) != want:
                return False
        if ck.eps_rank(s, 0.0) != len(s) or ck.eps_rank(s, 2 * errs[0]) != 0:
            return False
    return True


def test_eps_rank_is_smallest_sufficient_truncation():
    assert _eps_rank_pins_hold(checks)


def _expectation_pins_hold(ck) -> bool:
    s = np.array([3.0, 2.0, 1.0, 0.5, 0.25])
    ey1 = math.sqrt(4 + 1 + 0.25 + 0.0625)
    ey2 = math.sqrt(1 + 0.25 + 0.0625)
    pairs = [((1, 2), 2.0 * ey1), ((1, 3), 1.5 * ey1), ((2, 3), 2.0 * ey2), ((2, 5), 1.5 * ey2)]
    return all(abs(ck.expectation_bound(s, k, p) - want) < 1e-14 * want
               for (k, p), want in pairs)


def test_expectation_bound_hand_values():
    assert _expectation_pins_hold(checks)


def test_expectation_bound_holds_for_randqb_on_average():
    """Section 3.2: the mean error of randQB with l = k + p Gaussian columns
    stays below (1 + k/(p-1)) EY(k); 400 draws, slow decay."""
    rng = np.random.default_rng(9)
    m, n = 60, 40
    s = 1.0 / np.arange(1, n + 1)
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (U * s) @ V.T
    for k, p in ((5, 2), (8, 4)):
        errs = []
        for _ in range(400):
            Q, _ = np.linalg.qr(A @ rng.standard_normal((n, k + p)))
            errs.append(np.linalg.norm(A - Q @ (Q.T @ A)))
        assert np.mean(errs) <= checks.expectation_bound(s, k, p)
        assert np.mean(errs) >= checks.eckart_young(s, k + p)


@pytest.mark.parametrize("old,new", [
    ("tail = s[k:]", "tail = s[k + 1:]"),                   # tail starts one late
    ("tail = s[k:]", "tail = s[max(k - 1, 0):]"),           # tail starts one early
    ("s = np.sort(np.asarray(s, dtype=np.float64))[::-1]\n    tail",
     "s = np.asarray(s, dtype=np.float64)\n    tail"),       # unsorted input taken as is
])
def test_eckart_young_mutations_are_caught(old, new):
    assert not _ey_pins_hold(mutant("checks", old, new))


@pytest.mark.parametrize("old,new", [
    ("if eckart_young(s, k) <= eps:", "if eckart_young(s, k) < eps:"),   # strict test
    ("            return k\n", "            return k + 1\n"),             # one past
    ("for k in range(len(s) + 1):", "for k in range(1, len(s) + 1):"),  # k = 0 never tried
])
def test_eps_rank_mutations_are_caught(old, new):
    assert not _eps_rank_pins_hold(mutant("checks", old, new))


@pytest.mark.parametrize("old,new", [
    ("(1.0 + k / (p - 1.0))", "(1.0 + k / (p + 1.0))"),
    ("(1.0 + k / (p - 1.0))", "math.sqrt(1.0 + k / (p - 1.0))"),
    ("* eckart_young(s, k)", "* eckart_young(s, k + p)"),
])
def test_expectation_bound_mutations_are_caught(old, new):
    assert not _expectation_pins_hold(mutant("checks", old, new))
