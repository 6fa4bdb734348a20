"""Pins of the oracle's unblocked and skip-re-orthonormalisation paths
(Section 5.4, Section 6.3 and Figure 8; randQB_p of Figure 5).

* single pass with orth between applications = subspace iteration started
  from A Omega with a Householder QR (numpy) at each step: same projector;
* single pass without it = the range of (A A^T)^P A Omega, orthonormalised
  by numpy's Householder QR: same projector (inputs conditioned well enough
  for both orths to be exact to rounding);
* blocked, with or without it, on a well-conditioned input: same rank and
  the same Q B;
* the behaviour Section 5.4 predicts: without re-orthonormalisation a single
  pass resolves nothing below sigma_1 tau^(1/(2P+1)), with tau the relative
  column size the orth can still separate (2^-20 for CholQR with the 2^-40
  pivot test on the Gram matrix; the unit roundoff for the Householder QR of
  the paper); with it, a single pass stops at sigma_1 tau (the first
  orth(A Omega) already drops what lies below); the blocked scheme samples
  the rest in later blocks and still reaches a tight tolerance.
"""
import numpy as np
import pytest

import synth
from oracle import randqb_pb
from oracle.checks import eckart_young
from oracle.gaussian import omega_block


def _proj(Q):
    return Q @ Q.T


def _mild(m=300, n=200, seed=3):
    s = 1.0 / (1.0 + np.arange(n)) ** 0.5       # cond of A^3 Omega stays < 1e4
    return synth.prescribed_svd(m, n, s, seed, seed + 1), s


@pytest.mark.parametrize("P", [1, 2])
def test_single_pass_with_orth_is_subspace_iteration(P):
    A, _ = _mild()
    l, seed = 30, 5
    r = randqb_pb(A, 0.0, l, P, seed, kmax=l, max_blocks=1)
    assert r.k == l and r.blocks == 1 and r.stop_reason == 4  # KMAX
    Q = np.linalg.qr(A @ omega_block(seed, A.shape[1], 0, l))[0]
    for _ in range(P):
        Z = np.linalg.qr(A.T @ Q)[0]
        Q = np.linalg.qr(A @ Z)[0]
    assert np.linalg.norm(_proj(r.Q) - _proj(Q)) < 1e-10
    assert np.linalg.norm(r.B - r.Q.T @ A) < 1e-13 * np.linalg.norm(A)


@pytest.mark.parametrize("P", [1, 2])
def test_single_pass_without_orth_is_range_of_power(P):
    A, _ = _mild()
    l, seed = 30, 6
    r = randqb_pb(A, 0.0, l, P, seed, kmax=l, max_blocks=1, power_orth=False)
    Y = A @ omega_block(seed, A.shape[1], 0, l)
    for _ in range(P):
        Y = A @ (A.T @ Y)
    Q = np.linalg.qr(Y)[0]
    assert r.k == l
    assert np.linalg.norm(_proj(r.Q) - _proj(Q)) < 1e-9


def test_blocked_with_and_without_orth_agree_when_well_conditioned():
    A, _ = _mild(400, 300, 9)
    nA = np.linalg.norm(A)
    a = randqb_pb(A, 0.3 * nA, 16, 1, 11)
    b = randqb_pb(A, 0.3 * nA, 16, 1, 11, power_orth=False)
    assert a.k == b.k and a.widths == b.widths
    assert np.linalg.norm(a.Q @ a.B - b.Q @ b.B) < 1e-9 * nA


def test_max_blocks_validation():
    A, _ = _mild(40, 30)
    with pytest.raises(ValueError):
        randqb_pb(A, 0.0, 8, 0, 1, max_blocks=0)
    # one block of an adaptive run equals the first block of the full run
    full = randqb_pb(A, 1e-6, 8, 0, 1)
    one = randqb_pb(A, 1e-6, 8, 0, 1, max_blocks=1)
    assert one.k == full.widths[0]
    assert np.allclose(one.Q, full.Q[:, :one.k], atol=1e-14)


TAU = 2.0 ** -20   # relative column size CholQR with the 2^-40 Gram test resolves


@pytest.mark.parametrize("P", [1, 2])
def test_floor_without_reorth_single_pass_but_not_blocked(P):
    """Matrix 1 of Section 6.2 (800 x 600, singular values down to 1e-18).

    A single pass resolves nothing below sigma_1 tau^(1/(2P+1)) without
    re-orthonormalisation (Section 5.4 with the orth's resolution tau in
    place of the unit roundoff); with it, the first orth(A Omega) already
    limits the pass to sigma_1 tau.  The blocked scheme samples what a block
    could not resolve in the next block and reaches a tight tolerance."""
    A = synth.paper_matrix1(800, 600, seed=1)
    s = np.linalg.svd(A, compute_uv=False)
    nA = np.linalg.norm(A)
    floor_no = s[0] * TAU ** (1.0 / (2 * P + 1))
    floor_yes = s[0] * TAU
    for l in (40, 60, 80):
        no = randqb_pb(A, 0.0, l, P, 7, kmax=l, max_blocks=1, power_orth=False)
        yes = randqb_pb(A, 0.0, l, P, 7, kmax=l, max_blocks=1)
        e_no = np.linalg.norm(A - no.Q @ no.B)
        e_yes = np.linalg.norm(A - yes.Q @ yes.B)
        assert 0.1 * floor_no <= e_no <= 3.0 * floor_no and no.k < l
        assert 0.1 * floor_yes <= e_yes <= 3.0 * floor_yes and yes.k < l
        assert e_yes < 1e-3 * e_no
    # above the floors a single pass is near-optimal
    l = 20
    yes = randqb_pb(A, 0.0, l, P, 7, kmax=l, max_blocks=1)
    assert yes.k == l
    assert np.linalg.norm(A - yes.Q @ yes.B) <= 3 * eckart_young(s, l)
    # blocked without re-orthonormalisation still reaches a tight tolerance
    eps = 1e-13 * nA
    blk = randqb_pb(A, eps, 10, P, 7, power_orth=False)
    assert blk.stop_reason in (0, 1) and np.linalg.norm(A - blk.Q @ blk.B) <= eps * (1 + 1e-9)
