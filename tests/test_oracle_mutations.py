"""Planted mistakes: each test builds a copy of one oracle module with a
plausible slip (a dropped term, a wrong sign, a skipped step, a wrong
operand) and checks that the pins used on the real oracle reject it.  This
shows the pins can see such mistakes; nothing here touches the GPU path."""
import math
import sys
import types

import numpy as np
import pytest

import oracle
import synth
from oracle.checks import orth_defect, eckart_young

U = 2.0 ** -53


def mutant(modname: str, old: str, new: str) -> types.ModuleType:
    """Load oracle.<modname> from source with one textual change applied."""
    real = sys.modules[f"oracle.{modname}"]
    src = open(real.__file__).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old!r}"
    name = f"oracle._mutant_{modname}"
    mod = types.ModuleType(name)
    mod.__package__ = "oracle"
    mod.__file__ = real.__file__
    sys.modules[name] = mod  # dataclasses look their module up by name
    try:
        exec(compile(src.replace(old, new), real.__file__, "exec"), mod.__dict__)
    finally:
        del sys.modules[name]
    return mod


def _invariants_hold(randqb_pb) -> bool:
    """The Proposition 4.1 / Pythagoras / Eckart-Young pins of test_oracle_randqb."""
    s = synth.spectrum("exp", 120, scale=6.0)
    A = synth.prescribed_svd(160, 120, s, 1, 2)
    nA = float(np.linalg.norm(A))
    try:
        res = randqb_pb(A, 1e-12 * nA, 10, 0, seed=4)
    except Exception:
        return False
    if res.k == 0:
        return False
    ok = orth_defect(res.Q) < 1e-13
    ok &= np.linalg.norm(res.R - (A - res.Q @ res.B)) < 1e-13 * nA
    ok &= np.linalg.norm(res.B - res.Q.T @ A) < 1e-13 * nA
    err = np.linalg.norm(A - res.Q @ res.B)
    ok &= err <= 1e-12 * nA * (1 + 1e-9)
    ok &= err >= eckart_young(s, res.k) * (1 - 1e-9)
    return bool(ok)


def _closed_form_holds(randqb_pb) -> bool:
    A = synth.orthonormal_scaled(150, 100, 3.0, seed=12)
    res = randqb_pb(A, 3.0 * math.sqrt(100 - 40 + 0.5), 16, 0, seed=1)
    return res.k == 48 and all(abs(D - 9.0 * (100 - 16 * (i + 1))) < 1e-9
                               for i, D in enumerate(res.D))


def test_real_oracle_passes_the_mutation_pins():
    assert _invariants_hold(oracle.randqb_pb)
    assert _closed_form_holds(oracle.randqb_pb)


@pytest.mark.parametrize("old,new", [
    ("R -= Qi @ Bi", "R += Qi @ Bi"),                                    # downdate sign
    ("R -= Qi @ Bi", "R -= Y @ Bi"),                                     # sample used for basis
    ("if kept and reorth and k > 0:", "if False:"),                      # skip re-projection (3')
    ("Qi = Qi - Qbar @ (Qbar.T @ Qi)", "Qi = Qi + Qbar @ (Qbar.T @ Qi)"),  # projection sign
    ("Y = R @ Om", "Y = R @ Om[:, :1].repeat(Om.shape[1], axis=1)"),     # one sketch column reused
])
def test_driver_mutations_are_caught(old, new):
    mod = mutant("randqb", old, new)
    assert not (_invariants_hold(mod.randqb_pb) and _closed_form_holds(mod.randqb_pb))


@pytest.mark.parametrize("old,new", [
    ("if E <= eps2 - delta:", "if E < eps2 - delta - 1e300:"),           # tracked branch dead
    ("E = sA - math.fsum(sigB_parts)", "E = sA + math.fsum(sigB_parts)"),  # indicator sign
    ("w = min(b, kcap - k)", "w = b"),                                  # no width cap
])
def test_stop_rule_mutations_are_caught(old, new):
    mod = mutant("randqb", old, new)
    ok = _closed_form_holds(mod.randqb_pb)
    # kmax / rank-cap behaviour of test_kmax_and_rank_cap
    A = synth.prescribed_svd(80, 60, synth.spectrum("power", 60, p=0.5), 7, 8)
    try:
        r1 = mod.randqb_pb(A, 1e-12 * np.linalg.norm(A), 16, 0, seed=1, kmax=40)
        r2 = mod.randqb_pb(A, 0.0, 16, 0, seed=1)
        ok &= r1.k == 40 and r2.k == 60
    except Exception:
        ok = False
    # tracked branch: sigma*orthonormal input with eps far above the band
    B = synth.orthonormal_scaled(150, 100, 3.0, seed=12)
    try:
        r3 = mod.randqb_pb(B, 3.0 * math.sqrt(100 - 40 + 0.5), 16, 0, seed=1)
        ok &= r3.stop_reason == oracle.STOP["TOL_TRACKED"]
    except Exception:
        ok = False
    assert not ok


@pytest.mark.parametrize("old,new", [
    ("d = G[c, c] - float(np.dot(Tfull[kept, c], Tfull[kept, c])) if kept else G[c, c]",
     "d = G[c, c]"),                                                     # dropped pivot term
    ("Tfull[c, c + 1:] = rest / tcc", "Tfull[c, c + 1:] = rest * tcc"),  # wrong scaling
    ("Q2, kept2 = cholqr(Q1, drop_rel)", "Q2, kept2 = Q1, list(range(Q1.shape[1]))"),  # one pass only
])
def test_orth_mutations_are_caught(old, new):
    mod = mutant("cholqr", old, new)
    rng = np.random.default_rng(4)
    u, _ = np.linalg.qr(rng.standard_normal((400, 24)))
    X = (u * np.logspace(0, -6, 24)) @ np.linalg.qr(rng.standard_normal((24, 24)))[0].T
    Q, kept = mod.cholqr2(X)
    good = kept == list(range(24)) and orth_defect(Q) < 20 * U * 24 \
        and np.linalg.norm(X - Q @ (Q.T @ X)) < 1e-10 * np.linalg.norm(X)
    assert not good


@pytest.mark.parametrize("old,new", [
    ("ATANH_C = [1.0 / float(2 * k + 1)", "ATANH_C = [1.0 / float(2 * k + 2)"),  # series index
    ("return e * LN2_HI + (logf + e * LN2_LO)", "return e * LN2_HI + logf"),  # ln2 low part dropped
    ("cos_out = np.select([qi == 0, qi == 1, qi == 2], [cs, -sn, -cs], sn)",
     "cos_out = np.select([qi == 0, qi == 1, qi == 2], [cs, sn, -cs], sn)"),  # quadrant sign
    ("ps = ps * z + SIN_C[k]", "ps = ps * z - SIN_C[k]"),                # sine series sign
])
def test_gaussian_mutations_are_caught(old, new):
    mod = mutant("gaussian", old, new)
    rng = np.random.default_rng(1)
    u = np.exp(-rng.uniform(0, 36.7, 20000))
    want = np.log(u.astype(np.longdouble))
    logok = np.max(np.abs((mod.log_own(u) - want) / want)) < 4 * U
    v = rng.uniform(0, 1, 20000)
    ang = np.longdouble("6.28318530717958647692528676655900576839") * v.astype(np.longdouble)
    c, s = mod.sincos_2pi(v)
    trigok = np.max(np.abs(c - np.cos(ang))) < 3e-16 and np.max(np.abs(s - np.sin(ang))) < 3e-16
    assert not (logok and trigok)


def test_philox_constant_mutation_is_caught():
    mod = mutant("philox", "M0 = np.uint64(0xD2511F53)", "M0 = np.uint64(0xD2511F55)")
    # known-answer rows produced by the real generator, re-checked against
    # rocRAND in test_oracle_philox; a changed multiplier changes them
    real = oracle.philox.philox4x32_10(12345, 678, 0, 0, 1503, 0)
    fake = mod.philox4x32_10(12345, 678, 0, 0, 1503, 0)
    assert tuple(int(x) for x in real) != tuple(int(x) for x in fake)


def _single_pass_pins_hold(randqb_pb) -> bool:
    """Pins of test_oracle_skip_reorth: one pass without re-orthonormalisation
    spans (A A^T) A Omega; max_blocks=1 stops after one block."""
    from oracle.gaussian import omega_block
    s = 1.0 / (1.0 + np.arange(200)) ** 0.5
    A = synth.prescribed_svd(300, 200, s, 3, 4)
    try:
        r = randqb_pb(A, 0.0, 30, 1, 6, kmax=60, max_blocks=1, power_orth=False)
    except Exception:
        return False
    Y = A @ omega_block(6, 200, 0, 30)
    Y = A @ (A.T @ Y)
    Q = np.linalg.qr(Y)[0]
    return (r.blocks == 1 and r.k == 30
            and np.linalg.norm(r.Q @ r.Q.T - Q @ Q.T) < 1e-9)


def test_real_oracle_passes_the_single_pass_pins():
    assert _single_pass_pins_hold(oracle.randqb_pb)


@pytest.mark.parametrize("old,new", [
    ("            for _ in range(power_iters):\n                Y = R @ (R.T @ Y)",
     "            for _ in range(power_iters - 1):\n                Y = R @ (R.T @ Y)"),  # one power too few
    ("if max_blocks is not None and res.blocks >= max_blocks:",
     "if max_blocks is not None and res.blocks > max_blocks:"),           # block cap off by one
])
def test_single_pass_mutations_are_caught(old, new):
    mod = mutant("randqb", old, new)
    assert not _single_pass_pins_hold(mod.randqb_pb)


def _cpqr_pins_hold(mod) -> bool:
    try:
        Qt, R, perm = mod.pivoted_qr(np.array([[3.0, 1.0], [4.0, 2.0]]))
        ok = list(perm) == [0, 1] and abs(R[0, 0] + 5.0) < 1e-14
        B = np.random.default_rng(2800).standard_normal((40, 70))
        Qt, R, perm = mod.pivoted_qr(B)
        ok &= np.linalg.norm(B[:, perm] - Qt @ R) < 1e-13 * np.linalg.norm(B)
        for j in range(40):
            trail = np.sum(R[j:, j + 1:] ** 2, axis=0)
            ok &= bool(np.all(R[j, j] ** 2 >= trail * (1 - 1e-12)))
        return bool(ok)
    except Exception:
        return False


def test_real_oracle_passes_the_cpqr_pins():
    import oracle.postprocess as pp
    assert _cpqr_pins_hold(pp)


@pytest.mark.parametrize("old,new", [
    ("norms = np.sum(W[j:, j:] * W[j:, j:], axis=0)",
     "norms = np.sum(W[:, j:] * W[:, j:], axis=0)"),                    # norms over all rows
    ("beta = -nrm if x[0] >= 0.0 else nrm", "beta = nrm if x[0] >= 0.0 else -nrm"),  # reflector sign
    ("for j in reversed(range(steps)):", "for j in range(steps):"),     # wrong accumulation order
])
def test_cpqr_mutations_are_caught(old, new):
    assert not _cpqr_pins_hold(mutant("postprocess", old, new))


def _adjoint_fd_holds(mod) -> bool:
    """The central-difference pin of test_oracle_adjoint on one case."""
    from tests.test_oracle_adjoint import case, loss_np
    m, n, b, s, P = 60, 40, 8, 3, 1
    A, g = case(m, n)
    dQ = g.standard_normal((m, b * s))
    dB = g.standard_normal((b * s, n))
    _, _, dA = mod.qb_fixed_vjp(A, dQ, dB, b, s, P, 5)
    h = 1e-5 * np.linalg.norm(A)
    for _ in range(3):
        E = g.standard_normal((m, n))
        E /= np.linalg.norm(E)
        fd = (loss_np(A + h * E, dQ, dB, b, s, P, 5) - loss_np(A - h * E, dQ, dB, b, s, P, 5)) / (2 * h)
        if abs(fd - float(np.sum(dA * E))) > 1e-7 * np.linalg.norm(dA):
            return False
    return True


def test_real_oracle_passes_the_adjoint_pin():
    import oracle.adjoint
    assert _adjoint_fd_holds(oracle.adjoint)


@pytest.mark.parametrize("old,new", [
    # re-projection treated as a constant projector in the backward
    ("Qi = orth_t(Qi - Qbar @ (Qbar.T @ Qi))", "Qi = orth_t(Qi - Qbar.detach() @ (Qbar.detach().T @ Qi))"),
    # B_i = Q_i^T R with Q_i held fixed
    ("Bi = Qi.T @ R", "Bi = Qi.detach().T @ R"),
    # one operand of the Gram matrix held fixed
    ("L = torch.linalg.cholesky(X.T @ X)", "L = torch.linalg.cholesky(X.detach().T @ X)"),
    # power iteration: the transposed product held fixed
    ("Z = orth_t(R.T @ Qi)", "Z = orth_t(R.detach().T @ Qi)"),
])
def test_adjoint_mutations_are_caught(old, new):
    assert not _adjoint_fd_holds(mutant("adjoint", old, new))
