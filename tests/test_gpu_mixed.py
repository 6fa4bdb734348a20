"""GPU checks of the mixed-precision sampling forms (FP32 and bf16x3 MFMA).

The sampling products only choose the subspace (Figure 4 step (3), Figure 6
steps (5)-(6)); orth, B = Q^T A, the downdate and the stopping rule stay in
float64.  A sample with relative error delta (2^-24 for f32, about 2^-16 for
bf16x3) leaves a first-order leftover of relative size ~delta of the captured
directions in the residual, which later blocks must pick up.  So:
  * the error bound ||A - QB|| <= eps always holds (float64 downdate and
    stopping quantity);
  * the rank equals the float64 oracle's when eps_rel >> delta, and may
    exceed it by whole blocks when eps_rel is below delta.
Bars:
  products   |Y - X W| <= 4 u_p K |X||W| elementwise, u_p = delta; and
             norm-wise, row i and column j: f32 within 1e-6 ||x_i|| ||w_j||
             of the float64 product of the float32-rounded inputs, bf16x3
             within max(2e-6, 4 2^-15 / sqrt(K)) ||x_i|| ||w_j|| of X W
             (both below the size of one wrong term), also at the full
             20000 x 16000 x 256 launch configuration on sampled rows
  factor     rank and widths equal to the oracle's when eps_rel >= 30 delta;
             otherwise k >= oracle k; always Q orthonormal to float64
             rounding and ||A - QB|| <= eps checked directly; Q B within
             2 eps of the oracle's (triangle inequality)
"""
import math

import numpy as np
import pytest
import torch

import paper_1503_07157_amd as qbmi
import synth
from oracle import randqb_pb
from oracle.randqb import sumsq

pytestmark = pytest.mark.gpu
UNIT = {"f32": 2.0 ** -24, "bf16x3": 2.0 ** -16}


def dev(x):
    return qbmi.colmajor(torch.from_numpy(np.ascontiguousarray(x)).cuda())


def _check_normwise(got, A, Bm, prec, not_f64):
    """got ~ A @ Bm: the elementwise bound 4 u_p K |A||B|, and the sharper
    norm-wise bars of the full-size test below: f32 against the float64
    product of the float32-rounded inputs, bar 1e-6 ||a_i|| ||b_j||; bf16x3
    against the float64 product, bar max(2e-6, 4 2^-15 / sqrt(K))
    ||a_i|| ||b_j|| (each term carries a split error below 2^-15 |a_k b_k|;
    with random signs, on Gaussian data, they add to about
    2^-15 ||a_i|| ||b_j|| / sqrt(K))."""
    ref = A @ Bm
    K = A.shape[1]
    assert np.all(np.abs(got - ref) <= 4 * UNIT[prec] * K * (np.abs(A) @ np.abs(Bm)))
    norms = np.outer(np.linalg.norm(A, axis=1), np.linalg.norm(Bm, axis=0))
    norms[norms == 0] = 1.0
    if prec == "f32":
        A32 = A.astype(np.float32).astype(np.float64)
        B32 = Bm.astype(np.float32).astype(np.float64)
        assert np.max(np.abs(got - A32 @ B32) / norms) <= 1e-6
    else:
        assert np.max(np.abs(got - ref) / norms) <= max(2e-6, 4 * 2.0 ** -15 / np.sqrt(K))
    if not_f64:  # and it is not silently the float64 product
        assert np.max(np.abs(got - ref)) > 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
@pytest.mark.parametrize("m,K,w", [(300, 500, 50), (129, 1000, 128), (1000, 4100, 256), (1, 3, 1),
                                   # 256 x 128 tiles up to 128 columns, 128 x 256 above;
                                   # ragged rows and depth, odd ld (pairwise loads off),
                                   # several depth chunks
                                   (1025, 777, 127), (2600, 2050, 129), (5003, 3001, 200),
                                   (4096, 6000, 256)])
def test_lowp_sample_product(cuda, prec, m, K, w):
    r = np.random.default_rng(m + K + w)
    X = np.asfortranarray(r.standard_normal((m, K)))
    W = np.asfortranarray(r.standard_normal((K, w)))
    Y = qbmi.sample_product(dev(X), dev(W), prec).cpu().numpy()
    _check_normwise(Y, X, W, prec, K > 100)


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
@pytest.mark.parametrize("K,w,N", [(500, 50, 300), (4100, 256, 257), (33, 7, 2000),
                                   (3001, 200, 1111), (6000, 129, 4000)])
def test_lowp_project(cuda, prec, K, w, N):
    r = np.random.default_rng(K + w + N)
    Qm = np.asfortranarray(r.standard_normal((K, w)))
    X = np.asfortranarray(r.standard_normal((K, N)))
    C = qbmi.project(dev(Qm), dev(X), prec).cpu().numpy()
    _check_normwise(C.T, X.T, Qm, prec, False)


# Full size, in the launch configuration of the 20000 x 16000, b = 256
# factorisation (the depth split, the packed 256-wide panel, 128 x 256 and
# 256 x 128 tiles): sampled rows of Y = X W and sampled columns of
# C = Q^T X against float64 host products of the same rows and columns.
# Sampled: the first and last rows and columns, both sides of tile edges,
# the ragged tail, and random ones.  At K = 16000 the elementwise bound above
# is far looser than the actual error, so two sharper checks are added:
#   * f32: the reference is the float64 product of the float32-rounded
#     inputs, leaving only the float32 accumulation (a random walk of about
#     u sqrt(sum of squared partial sums), measured 9e-8 ||x_i|| ||w_j||
#     for this Gaussian data); the bar 1e-6 ||x_i|| ||w_j|| still catches a
#     single wrong term of size |x_ik w_kj| (about 6e-5 ||x_i|| ||w_j||);
#   * bf16x3: against the float64 product; the split's residual (x - hi -
#     lo about 2^-17 |x| after the float rounding, the dropped lo*lo terms)
#     and the float32 accumulation add up with random signs (measured
#     1.4e-7 ||x_i|| ||w_j|| on MI355X); bar 2e-6, which a single wrong
#     term (about 6e-5 ||x_i|| ||w_j|| here) exceeds.
def _sampled(n, edges, count, seed):
    r = np.random.default_rng(seed)
    idx = set(i for i in edges if 0 <= i < n)
    idx.update(int(i) for i in r.integers(0, n, count))
    return np.array(sorted(idx))


def _check_sampled(got, A, Bm, prec, what):
    # got ~ A @ Bm (A: the sampled rows)
    norms = np.outer(np.linalg.norm(A, axis=1), np.linalg.norm(Bm, axis=0))
    ref = (A.astype(np.float32).astype(np.float64) @ Bm.astype(np.float32).astype(np.float64)
           if prec == "f32" else A @ Bm)
    print(f"[case] full-size {what} {prec}: max err / (|x_i| |w_j|) "
          f"{np.max(np.abs(got - ref) / norms):.2e}", flush=True)
    _check_normwise(got, A, Bm, prec, True)


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_lowp_full_size_sampled(cuda, prec):
    m, n, w = 20000, 16000, 256
    g = torch.Generator(device="cuda").manual_seed(1503)
    X = torch.randn((n, m), dtype=torch.float64, device="cuda", generator=g).t()
    W = torch.randn((w, n), dtype=torch.float64, device="cuda", generator=g).t()
    Qm = torch.randn((w, m), dtype=torch.float64, device="cuda", generator=g).t()
    Y = qbmi.sample_product(X, W, prec)
    C = qbmi.project(Qm, X, prec)
    torch.cuda.synchronize()
    rows = torch.from_numpy(_sampled(m, [0, 1, 127, 128, 255, 256, 19967, 19968, m - 1], 40, 7))
    cols = torch.from_numpy(_sampled(n, [0, 1, 127, 128, 255, 256, 15871, 15872, n - 1], 40, 8))
    _check_sampled(Y[rows.cuda()].cpu().numpy(), X[rows.cuda()].cpu().numpy(),
                   W.cpu().numpy(), prec, "sample rows")
    # C[:, j] = Q^T X[:, j]: rows of C^T = X^T Q
    _check_sampled(C[:, cols.cuda()].t().cpu().numpy(), X[:, cols.cuda()].t().cpu().numpy(),
                   Qm.cpu().numpy(), prec, "projection columns")


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
@pytest.mark.parametrize("P", [0, 1])
@pytest.mark.parametrize("eps_rel", [1e-6, 1e-3])
def test_mixed_factor_small_workload(cuda, prec, P, eps_rel):
    w = synth.workload("exp40_2000x1000")
    A = synth.workload_matrix(w.name)
    nA = math.sqrt(sumsq(A))
    eps = eps_rel * nA
    g = qbmi.qb_factor(dev(A), eps, w.b, P, w.seed_omega, sample=prec)
    o = randqb_pb(A, eps, w.b, P, w.seed_omega)
    print(f"[case] prec={prec} P={P} eps_rel={eps_rel} k_gpu={g.k} k_oracle={o.k}", flush=True)
    if eps_rel >= 30 * UNIT[prec]:
        assert g.k == o.k and g.widths == o.widths
    else:
        assert g.k >= o.k
    Q, B = g.Q.cpu().numpy(), g.B.cpu().numpy()
    assert np.linalg.norm(Q.T @ Q - np.eye(g.k)) < 1e-12
    assert np.linalg.norm(A - Q @ B) <= eps * (1 + 1e-9)
    assert np.linalg.norm(Q @ B - o.Q @ o.B) <= 2 * eps


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_mixed_exact_rank(cuda, prec):
    A = synth.exact_rank(300, 200, 37, seed=4, cond=1e3)
    nA = np.linalg.norm(A)
    # tolerance far above the sampling precision: stops at the true rank
    g = qbmi.qb_factor(dev(A), 1e-2 * nA, 16, 0, 3, sample=prec)
    o = randqb_pb(A, 1e-2 * nA, 16, 0, 3)
    assert g.k == o.k
    # tolerance below it: accurate, at the cost of extra blocks
    g = qbmi.qb_factor(dev(A), 1e-10 * nA, 16, 0, 3, sample=prec)
    Q, B = g.Q.cpu().numpy(), g.B.cpu().numpy()
    assert g.k >= 37
    assert np.linalg.norm(A - Q @ B) <= 1e-10 * nA


# ---- B_i = Q_i^T A in reduced precision (sweep variants) -------------------
# The downdate, residual norm and stopping rule stay float64, so the returned
# factorisation satisfies ||A - QB|| <= eps whenever the call reports QB_OK.
# The leftover Q_i (B~_i - Q_i^T A) lies in the span of Qbar and is never
# sampled again, so the attainable error floors near the product's rounding:
# below that the run goes to full rank and reports the floor.
FLOOR = {"f32": 1e-5, "bf16x3": 1e-2}


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_bgemm_variant_matches_oracle_above_floor(cuda, prec):
    w = synth.workload("exp40_2000x1000")
    A = synth.workload_matrix(w.name)
    nA = math.sqrt(sumsq(A))
    eps = 1e-2 * nA
    g = qbmi.qb_factor(dev(A), eps, w.b, 0, w.seed_omega, bgemm=prec)
    o = randqb_pb(A, eps, w.b, 0, w.seed_omega)
    print(f"[case] bgemm={prec} k_gpu={g.k} k_oracle={o.k}", flush=True)
    assert g.k == o.k and g.widths == o.widths and g.stop_reason in ("TOL_TRACKED", "TOL_DIRECT")
    Q, B = g.Q.cpu().numpy(), g.B.cpu().numpy()
    assert np.linalg.norm(Q.T @ Q - np.eye(g.k)) < 1e-12
    assert np.linalg.norm(A - Q @ B) <= eps * (1 + 1e-9)
    # B differs from Q^T A by the product's rounding only (elementwise bound)
    Qd = g.Q.cpu().numpy()
    bound = 4 * UNIT[prec] * w.m * (np.abs(Qd).T @ np.abs(A))
    assert np.all(np.abs(B - Qd.T @ A) <= bound)


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_bgemm_variant_reports_its_floor(cuda, prec):
    w = synth.workload("exp40_2000x1000")
    A = synth.workload_matrix(w.name)
    nA = math.sqrt(sumsq(A))
    g = qbmi.qb_factor(dev(A), 1e-12 * nA, w.b, 0, w.seed_omega, bgemm=prec)
    Q, B = g.Q.cpu().numpy(), g.B.cpu().numpy()
    err = np.linalg.norm(A - Q @ B) / nA
    print(f"[case] bgemm={prec} k={g.k} stop={g.stop_reason} floor={err:.3e}", flush=True)
    # the tolerance is out of reach: full rank, no false success
    assert g.k == min(A.shape) and g.stop_reason == "RANK_CAP"
    assert 1e-12 < err <= FLOOR[prec]
    # the reported direct residual is the true one
    assert abs(math.sqrt(g.resid2) / nA - err) <= 1e-3 * err
