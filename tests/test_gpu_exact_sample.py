"""GPU parity of the exact-range sample (QB_SAMPLE_INT8X8) against the
oracle's definition (oracle/intsplit.py), through the C ABI.

Component bar: the GPU forms the grid product exactly in integers and
rounds it once (a Horner sum of eight int32 digit sums), the oracle forms
it with a float64 matmul; both are within (K + 16) u |X~||W~| of the exact
value, elementwise.  On small inputs the GPU result is also compared with
the exact rational product (Python integers): within 16 u of its magnitude
sum.  Driver bar: the factorisation with this sample has the oracle's rank,
kept widths and stop reason, and Q B within 1e-10 ||A||_F.  At full size
(20000 x 16000, s_j = 1/j and the spectral-gap matrix, b = 256) the run
reaches eps = 1e-8 ||A||_F with k = 16000, measured directly as
||A - Q B||_F, and its first blocks match the oracle within 1e-10.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import torch

import paper_1503_07157_amd as qbmi
import synth
from oracle import randqb_pb, STOP
from oracle.intsplit import sample_exact, quantize_sketch, fixed_point, split_exponent
from oracle.randqb import sumsq

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
STATUS_NAMES = {v: k for k, v in STOP.items()}


def dev(x):
    return qbmi.colmajor(torch.from_numpy(np.ascontiguousarray(x)).cuda())


@pytest.mark.parametrize("m,K,w", [(300, 1000, 16), (257, 130, 64), (1000, 3000, 128),
                                   (513, 777, 256), (33, 64, 1), (40, 140000, 8),
                                   (2048, 4096, 200)])
def test_component_matches_oracle(cuda, m, K, w):
    rng = np.random.default_rng(m + K + w)
    X = rng.standard_normal((m, K)) * np.exp2(rng.integers(-8, 3, size=(m, K)))
    W = rng.standard_normal((K, w))
    Y = qbmi.sample_product(dev(X), dev(W), "int8x8").cpu().numpy()
    D = sumsq(X)
    Yo = sample_exact(X, W, D)
    mag = np.abs(fixed_point(X, split_exponent(D))) @ np.abs(quantize_sketch(W))
    print(f"[case] exact sample {m}x{K}x{w}: max |Y - Yo| / mag = "
          f"{np.max(np.abs(Y - Yo) / (mag + 1e-300)):.2e}", flush=True)
    assert np.all(np.abs(Y - Yo) <= (K + 16) * U * mag + 1e-300)


def test_component_is_exact_on_small_inputs(cuda):
    rng = np.random.default_rng(5)
    m, K, w = 5, 300, 3
    X = rng.standard_normal((m, K)) * np.exp2(rng.integers(-20, 2, size=(m, K)))
    W = rng.standard_normal((K, w)) * 3.0
    Y = qbmi.sample_product(dev(X), dev(W), "int8x8").cpu().numpy()
    E = split_exponent(sumsq(X))
    a = [[round(Fraction(float(x)) * Fraction(2) ** (55 - E)) for x in row] for row in X]
    q = [[max(-127, min(127, round(Fraction(float(x)) * 16))) for x in row] for row in W]
    for i in range(m):
        for j in range(w):
            ex = sum(a[i][k] * q[k][j] for k in range(K)) * Fraction(2) ** (E - 59)
            mag = sum(abs(a[i][k] * q[k][j]) for k in range(K)) * Fraction(2) ** (E - 59)
            assert abs(Fraction(float(Y[i, j])) - ex) <= 16 * Fraction(U) * mag


@pytest.mark.parametrize("m,n,b,P,rel", [(300, 200, 16, 0, 1e-6), (600, 250, 32, 1, 1e-7),
                                         (257, 129, 64, 0, 1e-9), (1000, 300, 64, 0, 1e-12),
                                         (129, 257, 32, 0, 1e-8)])
def test_factorisation_matches_oracle(cuda, m, n, b, P, rel):
    s = 1.0 / np.arange(1, min(m, n) + 1)
    A = synth.prescribed_svd(m, n, s, 30 + m, 40 + n)
    nA = math.sqrt(sumsq(A))
    eps = rel * nA
    g = qbmi.qb_factor(dev(A), eps, b, P, 77, sample="int8x8")
    o = randqb_pb(A, eps, b, P, 77, sample="int8x8")
    print(f"[case] int8x8 {m}x{n} b={b} P={P} eps_rel={rel}: k {g.k}/{o.k} "
          f"stop {g.stop_reason}/{STATUS_NAMES[o.stop_reason]}", flush=True)
    assert g.k == o.k and g.widths == o.widths
    assert g.stop_reason == STATUS_NAMES[o.stop_reason] and g.status == o.status
    Q, B = g.Q.cpu().numpy(), g.B.cpu().numpy()
    assert np.linalg.norm(Q @ B - o.Q @ o.B) <= 1e-10 * nA
    if g.status == 0:
        assert np.linalg.norm(A - Q @ B) <= eps


@pytest.mark.parametrize("name", ["inv1_20000x16000", "gap_20000x16000"])
def test_full_size_reaches_tolerance_at_full_rank(cuda, name):
    wl = synth.workload(name)
    A = synth.workload_matrix_gpu(wl.name)
    nA = float(torch.linalg.norm(A))
    eps = wl.eps_rel * nA
    g = qbmi.qb_factor(A, eps, wl.b, 0, wl.seed_omega, sample="int8x8")
    err = float(torch.linalg.norm(A - g.Q @ g.B))
    print(f"[case] {name} int8x8 full: k={g.k} stop={g.stop_reason} err/|A|={err / nA:.3e}",
          flush=True)
    assert g.status == 0 and g.k == wl.n
    assert err <= eps
    # the first blocks against the oracle's exact-range run
    Ah = A.cpu().numpy()
    kmax = 2 * wl.b
    g2 = qbmi.qb_factor(A, eps, wl.b, 0, wl.seed_omega, kmax=kmax, sample="int8x8")
    o = randqb_pb(Ah, eps, wl.b, 0, wl.seed_omega, kmax=kmax, sample="int8x8")
    rel = np.linalg.norm(g2.Q.cpu().numpy() @ g2.B.cpu().numpy() - o.Q @ o.B) / nA
    print(f"[case] {name} int8x8 first 2 blocks: |QB - QB_oracle|/|A| = {rel:.3e}", flush=True)
    assert g2.k == o.k == kmax and rel <= 1e-10
    del A, g, g2
    torch.cuda.empty_cache()
