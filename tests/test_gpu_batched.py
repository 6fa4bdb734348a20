"""GPU parity of the batched QB (qb_factor_batched) with the float64 oracle,
problem by problem, through the C ABI.

The batch mixes sizes, spectra and block sizes (s_j = r^j, uneven m and n,
b in {16, 32, 64}) at eps = 1e-5 ||A||_F, the tolerance of the batched
workload.  The inputs are float32; the batched path computes in float64,
so each problem must match the oracle run on the same float32 values
widened to float64: the same rank, widths, stop reason and Q B within
1e-10 ||A||.  Plus the per-problem edge cases: a zero matrix, a NaN, kmax.
"""
import math

import numpy as np
import pytest
import torch

import paper_1503_07157_amd as qbmi
import synth
from oracle import STOP, randqb_pb
from paper_1503_07157_amd._lib import QB_ENONFINITE, QB_KMAX

STOP_NAMES = {v: k for k, v in STOP.items()}

pytestmark = pytest.mark.gpu


def dev32(x):
    """Column-major float32 device copy."""
    x = np.asarray(x, dtype=np.float32)
    out = torch.empty((x.shape[1], x.shape[0]), dtype=torch.float32, device="cuda").t()
    out.copy_(torch.from_numpy(np.ascontiguousarray(x)))
    return out


def test_batch_matches_oracle(cuda):
    specs = synth.batch_specs(count=24, seed=77, m_range=(64, 700), n_max=400)
    mats = [synth.batch_matrix(sp) for sp in specs]
    eps = [1e-5 * float(np.linalg.norm(A.astype(np.float64))) for A in mats]
    res = qbmi.qb_factor_batched([dev32(A) for A in mats], eps, [sp.b for sp in specs],
                                 [sp.seed_omega for sp in specs])
    for sp, A, e, g in zip(specs, mats, eps, res):
        A64 = A.astype(np.float64)
        o = randqb_pb(A64, e, sp.b, 0, sp.seed_omega)
        nA = math.sqrt(g.normA2)
        print(f"[case] {sp.m}x{sp.n} r={sp.r:.4f} b={sp.b}: k={g.k}/{o.k} "
              f"stop={g.stop_reason}/{STOP_NAMES[o.stop_reason]}", flush=True)
        assert g.status >= 0
        assert g.k == o.k and g.blocks == o.blocks
        assert g.stop_reason == STOP_NAMES[o.stop_reason]
        Q, B = g.Q.cpu().numpy(), g.B.cpu().numpy()
        assert np.linalg.norm(Q @ B - o.Q @ o.B) <= 1e-10 * nA
        assert np.linalg.norm(A64 - Q @ B) <= e * (1 + 1e-9)
        assert abs(g.normA2 - o.normA2) <= 1e-14 * o.normA2


def test_batch_edge_cases(cuda):
    r = np.random.default_rng(3)
    good = synth.batch_matrix(synth.BatchSpec(300, 200, 0.95, 32, 5, 6, 7))
    zero = np.zeros((100, 50), dtype=np.float32)
    bad = r.standard_normal((80, 60)).astype(np.float32)
    bad[3, 7] = np.nan
    nA = float(np.linalg.norm(good.astype(np.float64)))
    res = qbmi.qb_factor_batched([dev32(good), dev32(zero), dev32(bad), dev32(good)],
                                 [1e-5 * nA, 0.0, 1.0, 1e-5 * nA], [32, 16, 16, 16],
                                 [7, 1, 1, 7], kmax=[200, 50, 60, 40])
    g, z, b, c = res
    o = randqb_pb(good.astype(np.float64), 1e-5 * nA, 32, 0, 7)
    assert g.k == o.k and g.status == 0
    assert z.k == 0 and z.stop_reason == "ZERO" and z.status == 0
    assert b.status == QB_ENONFINITE and b.k == 0
    oc = randqb_pb(good.astype(np.float64), 1e-5 * nA, 16, 0, 7, kmax=40)
    assert c.k == 40 == oc.k and c.status == QB_KMAX and c.stop_reason == "KMAX"
    Q, B = c.Q.cpu().numpy(), c.B.cpu().numpy()
    assert np.linalg.norm(Q @ B - oc.Q @ oc.B) <= 1e-10 * nA


def test_batch_full_distribution(cuda):
    """48 problems drawn from the full size range (m up to 4096, n up to
    2048), built on the GPU, in one call: every problem meets its tolerance
    with orthonormal Q and the exact residual identity; the two cheapest
    match the oracle problem by problem."""
    specs = synth.batch_specs(count=48, seed=9090)
    As = [synth.batch_matrix_gpu(sp) for sp in specs]
    nA = [float(torch.linalg.norm(A, dtype=torch.float64)) for A in As]
    eps = [1e-5 * v for v in nA]
    res = qbmi.qb_factor_batched(As, eps, [sp.b for sp in specs], [sp.seed_omega for sp in specs])
    for sp, A, e, g in zip(specs, As, eps, res):
        print(f"[case] {sp.m}x{sp.n} r={sp.r:.4f} b={sp.b}: k={g.k} stop={g.stop_reason}", flush=True)
        assert g.status == 0 and g.stop_reason in ("TOL_TRACKED", "TOL_DIRECT", "RANK_CAP")
        A64 = A.to(torch.float64)
        R = A64 - g.Q @ g.B
        assert float(torch.linalg.norm(R)) <= e * (1 + 1e-9)
        I = g.Q.t() @ g.Q
        assert float(torch.linalg.norm(I - torch.eye(g.k, dtype=torch.float64, device=cuda))) <= 1e-12 * g.k
        # ||A - Q B||^2 = ||A||^2 - ||B||^2 for orthonormal Q and B = Q^T A
        lhs = float(torch.linalg.norm(R)) ** 2
        rhs = float(torch.linalg.norm(A64)) ** 2 - float(torch.linalg.norm(g.B)) ** 2
        assert abs(lhs - rhs) <= 1e-12 * float(torch.linalg.norm(A64)) ** 2
    order = sorted(range(len(specs)), key=lambda i: specs[i].m * specs[i].n * max(res[i].k, 1))
    for i in order[:2]:
        sp = specs[i]
        o = randqb_pb(As[i].cpu().numpy().astype(np.float64), eps[i], sp.b, 0, sp.seed_omega)
        assert res[i].k == o.k
        Qg, Bg = res[i].Q.cpu().numpy(), res[i].B.cpu().numpy()
        assert np.linalg.norm(Qg @ Bg - o.Q @ o.B) <= 1e-10 * nA[i]


def test_batch_result_independent_of_batch_mates(cuda):
    """The depth split of a problem's products depends only on its own
    sizes, so a problem factorised inside a batch gives bitwise the same Q
    and B as the same problem alone, and a repeated batch is bitwise
    reproducible."""
    specs = synth.batch_specs(count=10, seed=515, m_range=(300, 1500), n_max=800)
    mats = [dev32(synth.batch_matrix(sp)) for sp in specs]
    eps = [1e-5 * float(torch.linalg.norm(A, dtype=torch.float64)) for A in mats]
    bs = [sp.b for sp in specs]
    seeds = [sp.seed_omega for sp in specs]
    full = qbmi.qb_factor_batched(mats, eps, bs, seeds)
    again = qbmi.qb_factor_batched(mats, eps, bs, seeds)
    for i in (0, 3, 7):
        alone = qbmi.qb_factor_batched([mats[i]], [eps[i]], [bs[i]], [seeds[i]])[0]
        print(f"[case] problem {i}: k batch {full[i].k} alone {alone.k}", flush=True)
        assert alone.k == full[i].k
        assert torch.equal(alone.Q, full[i].Q) and torch.equal(alone.B, full[i].B)
    for r1, r2 in zip(full, again):
        assert r1.k == r2.k and torch.equal(r1.Q, r2.Q) and torch.equal(r1.B, r2.B)


def test_other_tile_classes_match_oracle(cuda):
    """Every allowed tile class computes the same products: a batch run with
    a non-default table (the one the tuner may pick) still matches the
    oracle problem by problem."""
    specs = synth.batch_specs(count=8, seed=31, m_range=(200, 900), n_max=500)
    mats = [synth.batch_matrix(sp) for sp in specs]
    eps = [1e-5 * float(np.linalg.norm(A.astype(np.float64))) for A in mats]
    saved = qbmi.batched_tiles()
    try:
        qbmi.set_batched_tiles({"sample": ["16x16", "32x32", "64x32"],
                                "gram": ["64x64", "64x64", "32x32"],
                                "apply": ["64x64", "32x64", "16x16"],
                                "reproj_c": ["32x32", "64x64", "64x32"],
                                "reproj_q": ["64x64", "16x16", "32x64"],
                                "b": ["32x32", "64x32", "64x64"],
                                "downdate": ["32x32", "64x32", "32x64"]})
        res = qbmi.qb_factor_batched([dev32(A) for A in mats], eps, [sp.b for sp in specs],
                                     [sp.seed_omega for sp in specs])
    finally:
        qbmi.set_batched_tiles(saved)
    for sp, A, e, g in zip(specs, mats, eps, res):
        o = randqb_pb(A.astype(np.float64), e, sp.b, 0, sp.seed_omega)
        assert g.k == o.k and g.stop_reason == STOP_NAMES[o.stop_reason]
        Q, B = g.Q.cpu().numpy(), g.B.cpu().numpy()
        assert np.linalg.norm(Q @ B - o.Q @ o.B) <= 1e-10 * math.sqrt(g.normA2)


def test_graph_replays_match_eager(cuda, monkeypatch):
    """The block loop runs as replays of a captured HIP graph (eight
    iterations per replay, the host reading one flag in between).  The same
    launches run eagerly, one iteration at a time, when QB_BATCHED_EAGER is
    set.  Both give bitwise the same factors, also when the batch needs
    many replays (b = 16 problems with k up to a few hundred) and when the
    call is repeated after eager work in between."""
    specs = synth.batch_specs(count=12, seed=4041, m_range=(200, 1200), n_max=600)
    mats = [dev32(synth.batch_matrix(sp)) for sp in specs]
    eps = [1e-6 * float(torch.linalg.norm(A, dtype=torch.float64)) for A in mats]
    bs = [16] * len(specs)
    seeds = [sp.seed_omega for sp in specs]
    g1 = qbmi.qb_factor_batched(mats, eps, bs, seeds)
    monkeypatch.setenv("QB_BATCHED_EAGER", "1")
    e1 = qbmi.qb_factor_batched(mats, eps, bs, seeds)
    monkeypatch.delenv("QB_BATCHED_EAGER")
    torch.cuda.synchronize()
    g2 = qbmi.qb_factor_batched(mats, eps, bs, seeds)
    print(f"[case] iterations {max(r.blocks for r in g1)}", flush=True)
    assert max(r.blocks for r in g1) > 16  # several graph replays
    for a, b_, c in zip(g1, e1, g2):
        assert a.k == b_.k == c.k and a.stop_reason == b_.stop_reason == c.stop_reason
        assert torch.equal(a.Q, b_.Q) and torch.equal(a.B, b_.B)
        assert torch.equal(a.Q, c.Q) and torch.equal(a.B, c.B)


def test_walking_launches_match(cuda, monkeypatch):
    """A launch whose unit bound exceeds 2^22 workgroups runs a fixed grid
    of 2048 that takes units from a per-launch counter instead of one
    workgroup per unit.  QB_BATCHED_WALK forces that form for every launch:
    the factors are bitwise those of the one-workgroup-per-unit launches,
    replayed as graphs and eagerly."""
    specs = synth.batch_specs(count=10, seed=4043, m_range=(200, 1500), n_max=800)
    mats = [dev32(synth.batch_matrix(sp)) for sp in specs]
    eps = [1e-6 * float(torch.linalg.norm(A, dtype=torch.float64)) for A in mats]
    bs = [sp.b for sp in specs]
    seeds = [sp.seed_omega for sp in specs]
    ref = qbmi.qb_factor_batched(mats, eps, bs, seeds)
    monkeypatch.setenv("QB_BATCHED_WALK", "1")
    walked = qbmi.qb_factor_batched(mats, eps, bs, seeds)
    monkeypatch.setenv("QB_BATCHED_EAGER", "1")
    walked_eager = qbmi.qb_factor_batched(mats, eps, bs, seeds)
    monkeypatch.delenv("QB_BATCHED_EAGER")
    monkeypatch.delenv("QB_BATCHED_WALK")
    print(f"[case] ranks {[r.k for r in ref]}", flush=True)
    for a, b_, c in zip(ref, walked, walked_eager):
        assert a.status == b_.status == c.status and a.status >= 0
        assert a.k == b_.k == c.k and a.stop_reason == b_.stop_reason == c.stop_reason
        assert torch.equal(a.Q, b_.Q) and torch.equal(a.B, b_.B)
        assert torch.equal(a.Q, c.Q) and torch.equal(a.B, c.B)
