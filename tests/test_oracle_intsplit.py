"""Pins for the exact-range sample of the mixed-precision form
(oracle/intsplit.py).

  exact arithmetic   the sample equals the exactly rounded rational product
                     of the two grid matrices, computed with Python integers
                     from the definitions (grid 2^(E-55) for the residual,
                     1/16 for the sketch, clip at 127)
  bounds             every entry below 2^(E-1); E no coarser than needed;
                     grid error at most 2^(E-56); sketch on its grid
  purpose            at k = n < m the run reaches 1e-12 ||A||, while a
                     sample carrying a relative 1e-7 component outside the
                     range floors above 1e-9 ||A||
  mutations          a planted change of the grid, the clip, the sketch
                     scale or the exponent margin fails one of these pins
"""
import math
import sys
import types
from fractions import Fraction

import numpy as np
import pytest

import synth
import oracle.intsplit as intsplit
from oracle import randqb_pb, STATUS
from oracle.randqb import sumsq


def _mutant(old, new):
    src = open(intsplit.__file__).read()
    assert old in src
    mod = types.ModuleType("oracle._mutant_intsplit")
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), intsplit.__file__, "exec"), mod.__dict__)
    return mod


def _inputs(seed, m=6, n=37, w=5):
    rng = np.random.default_rng(seed)
    R = rng.standard_normal((m, n)) * np.exp2(rng.integers(-30, 4, size=(m, n)))
    R[0, 0] = 0.0
    Om = rng.standard_normal((n, w)) * 2.5
    Om[3, 1] = 9.0      # beyond the clip
    Om[4, 2] = -8.2
    return R, Om


def _exact_product(R, Om, D):
    """Rational A~ Omega~ from the definitions, with Python integers."""
    _, e = math.frexp(D)
    E = -((-e) // 2) + 1
    a = [[round(Fraction(float(x)) * Fraction(2) ** (55 - E)) for x in row] for row in R]
    wq = [[max(-127, min(127, round(Fraction(float(x)) * 16))) for x in row] for row in Om]
    m, n = R.shape
    w = Om.shape[1]
    scale = Fraction(2) ** (E - 55) / 16
    return [[sum(a[i][k] * wq[k][j] for k in range(n)) * scale for j in range(w)]
            for i in range(m)], a, wq


def _agrees(mod, seed):
    R, Om = _inputs(seed)
    D = sumsq(R)
    Y = mod.sample_exact(R, Om, D)
    ex, a, wq = _exact_product(R, Om, D)
    m, n = R.shape
    _, e = math.frexp(D)
    E = -((-e) // 2) + 1
    for i in range(m):
        for j in range(Om.shape[1]):
            mag = sum(abs(a[i][k] * wq[k][j]) for k in range(n)) * Fraction(2) ** (E - 55) / 16
            if abs(Fraction(float(Y[i, j])) - ex[i][j]) > Fraction(2) ** -50 * (mag + 1e-300):
                return False
    return True


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_sample_is_the_exact_grid_product(seed):
    assert _agrees(intsplit, seed)


@pytest.mark.parametrize("scale", [1e-150, 1e-20, 1.0, 3.0, 1e150])
def test_exponent_bounds_every_entry(scale):
    rng = np.random.default_rng(7)
    for shape in ((1, 1), (5, 3), (40, 30)):
        R = rng.standard_normal(shape) * scale
        D = sumsq(R)
        E = intsplit.split_exponent(D)
        assert np.max(np.abs(R)) < 2.0 ** (E - 1)
        assert math.sqrt(D) >= 2.0 ** (E - 3)           # not coarser than needed
        Rt = intsplit.fixed_point(R, E)
        assert np.max(np.abs(Rt - R)) <= 2.0 ** (E - 56)
        q = np.ldexp(Rt, 55 - E)
        assert np.all(q == np.rint(q)) and np.max(np.abs(q)) < 2.0 ** 54
    assert intsplit.split_exponent(0.0) == 0


def test_exponent_at_powers_of_four():
    # D = 4^j: sqrt(D) = 2^j exactly, and an entry can equal it (a single
    # nonzero entry), so E - 1 must exceed j
    for j in (-600, -3, 0, 1, 5, 400):
        R = np.array([[2.0 ** j]])
        E = intsplit.split_exponent(sumsq(R))
        assert 2.0 ** j < 2.0 ** (E - 1)


def test_sketch_grid():
    Om = np.array([[0.0, 1.0 / 32, 3.0 / 32, -0.49, 7.9375, 7.97, 9.0, -100.0]]).T
    q = intsplit.quantize_sketch(Om)[:, 0] * 16
    assert list(q) == [0.0, 0.0, 2.0, -8.0, 127.0, 127.0, 127.0, -127.0]
    rng = np.random.default_rng(3)
    X = rng.standard_normal((500, 4))
    Xq = intsplit.quantize_sketch(X)
    assert np.max(np.abs(Xq - X)) <= 1.0 / 32 + 1e-15
    assert np.all(np.abs(Xq * 16) <= 127)


def _tall_problem():
    s = 1.0 / np.arange(1, 121)
    A = synth.prescribed_svd(300, 120, s, 5, 6)
    return A, math.sqrt(sumsq(A))


def test_exact_range_sample_reaches_full_precision_at_full_rank():
    A, nA = _tall_problem()
    res = randqb_pb(A, 1e-12 * nA, 16, 0, seed=9, sample="int8x8")
    assert res.status == STATUS["OK"] and res.k == 120
    assert np.linalg.norm(A - res.Q @ res.B) <= 1e-12 * nA
    # and its first block equals the float64 run's to the grid's size
    f = randqb_pb(A, 0.0, 16, 0, seed=9, kmax=16)
    g = randqb_pb(A, 0.0, 16, 0, seed=9, kmax=16, sample="int8x8")
    assert np.linalg.norm(f.Q @ f.B - g.Q @ g.B) < 0.05 * nA   # a different sketch, same quality
    assert abs(math.sqrt(g.D[0]) - math.sqrt(f.D[0])) < 0.2 * math.sqrt(f.D[0])


def test_a_sample_outside_the_range_floors(monkeypatch):
    """The contrast that motivates the exact form: a sample with a relative
    1e-7 part outside range(A) (the size of a float32 product's rounding)
    leaves the error far above 1e-12 once k reaches n < m."""
    import oracle.randqb as rq
    A, nA = _tall_problem()
    rng = np.random.default_rng(11)

    def noisy(R, Om, D):
        Y = intsplit.sample_exact(R, Om, D)
        return Y + 1e-7 * np.linalg.norm(Y) / math.sqrt(Y.size) * rng.standard_normal(Y.shape)

    monkeypatch.setattr(rq, "sample_exact", noisy)
    res = rq.randqb_pb(A, 1e-12 * nA, 16, 0, seed=9, sample="int8x8")
    assert res.k == 120 and res.status != STATUS["OK"]
    assert np.linalg.norm(A - res.Q @ res.B) > 1e-9 * nA


@pytest.mark.parametrize("old,new", [
    ("FRAC_BITS = 55", "FRAC_BITS = 54"),                 # grid one bit coarser
    ("SKETCH_SCALE = 16.0", "SKETCH_SCALE = 8.0"),       # sketch grid
    ("SKETCH_CLIP = 127", "SKETCH_CLIP = 128"),          # clip beyond int8
    ("return -((-e) // 2) + 1", "return -((-e) // 2)"),  # exponent without margin
    ("return -((-e) // 2) + 1", "return e // 2 + 1"),    # floor instead of ceil
])
def test_intsplit_mutations_are_caught(old, new):
    mod = _mutant(old, new)
    ok = all(_agrees(mod, s) for s in (1, 2, 3))
    try:
        for j in (-3, 0, 1, 5):
            R = np.array([[2.0 ** j]])
            ok &= 2.0 ** j < 2.0 ** (mod.split_exponent(sumsq(R)) - 1)
        for scale in (1e-20, 1.0, 3.0):
            R = np.random.default_rng(7).standard_normal((40, 30)) * scale
            E = mod.split_exponent(sumsq(R))
            ok &= bool(np.max(np.abs(R)) < 2.0 ** (E - 1))
    except Exception:
        ok = False
    assert not ok
