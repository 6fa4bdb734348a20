"""Pins for the oracle's Gaussian sketch (oracle/gaussian.py): its own log
and sine/cosine against extended-precision libm values, exact special
points, the Box-Muller output against N(0,1), and the column-slice property
that makes the sketch independent of the block size (Section 4.1, eq.
OmegaBlock)."""
import math

import numpy as np
import pytest
import scipy.stats

from oracle import gaussian as G

LD = np.longdouble
TWO_PI_LD = LD("6.28318530717958647692528676655900576839")


def test_constants_are_nearest_doubles():
    assert G.HALF_PI == math.pi / 2
    assert G.SQRT_HALF == math.sqrt(0.5)
    assert abs(float((LD(G.LN2_HI) + LD(G.LN2_LO)) - LD("0.693147180559945309417232121458")) ) < 1e-19
    assert G.SIN_C[1] == -1.0 / 6.0 and G.COS_C[1] == -0.5


def test_uniforms_exact_range():
    assert G.uniforms53(0, 0) == 2.0 ** -53
    assert G.uniforms53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0
    assert G.uniforms53(0x80000000, 0) == 0.5 + 2.0 ** -53
    u = G.uniforms53(np.uint64(0x12345678), np.uint64(0x9ABCDEF0))
    want = ((0x12345678 << 21) | (0x9ABCDEF0 >> 11)) + 1
    assert u == want / 2.0 ** 53


def test_log_against_libm():
    rng = np.random.default_rng(1)
    u = np.concatenate([
        np.exp(-rng.uniform(0, 36.7, 200000)),          # log-uniform over (2^-53, 1]
        1.0 - rng.integers(1, 2**20, 2000) * 2.0 ** -53,  # just below 1
        np.array([1.0, 0.5, 0.25, 2.0 ** -53, math.sqrt(0.5), math.nextafter(math.sqrt(0.5), 1)]),
    ])
    got = G.log_own(u)
    want = np.log(u.astype(LD))
    rel = np.abs((got.astype(LD) - want) / np.where(want == 0, 1, want)).astype(np.float64)
    assert rel.max() < 4 * 2.0 ** -53
    assert G.log_own(1.0) == 0.0
    assert G.log_own(0.5) == -math.log(2.0)


def test_sincos_against_libm():
    rng = np.random.default_rng(2)
    u = np.concatenate([rng.uniform(0, 1, 200000), np.arange(0, 1025) / 1024.0])
    c, s = G.sincos_2pi(u)
    ang = TWO_PI_LD * u.astype(LD)
    assert np.max(np.abs(c.astype(LD) - np.cos(ang))) < 3e-16
    assert np.max(np.abs(s.astype(LD) - np.sin(ang))) < 3e-16
    # exact quarter points
    c, s = G.sincos_2pi(np.array([0.0, 0.25, 0.5, 0.75, 1.0]))
    assert list(c) == [1.0, 0.0, -1.0, 0.0, 1.0]
    assert [abs(x) for x in s] == [0.0, 1.0, 0.0, 1.0, 0.0]
    assert list(np.sign(s[[1, 3]])) == [1.0, -1.0]


def test_box_muller_is_standard_normal():
    om = G.omega_block(seed=42, n=2000, col0=0, w=500)
    x = om.ravel()
    assert abs(x.mean()) < 5e-3
    assert abs(x.var() - 1.0) < 5e-3
    assert scipy.stats.kstest(x, "norm").pvalue > 1e-3
    # columns and the two rows of a pair are uncorrelated
    cc = np.corrcoef(om[:, :50].T)
    assert np.max(np.abs(cc - np.eye(50))) < 0.12
    assert abs(np.corrcoef(om[0::2].ravel(), om[1::2].ravel())[0, 1]) < 5e-3


def test_column_slices_independent_of_block():
    full = G.omega_block(seed=1503, n=37, col0=0, w=40)
    for col0, w in [(0, 5), (5, 13), (18, 22), (39, 1)]:
        part = G.omega_block(seed=1503, n=37, col0=col0, w=w)
        assert np.array_equal(part, full[:, col0:col0 + w])
    # odd n: rows are a prefix of the even-n sketch
    even = G.omega_block(seed=9, n=38, col0=3, w=4)
    odd = G.omega_block(seed=9, n=37, col0=3, w=4)
    assert np.array_equal(odd, even[:37])
    assert not np.array_equal(G.omega_block(seed=10, n=38, col0=3, w=4), even)
    assert G.omega_block(1, 0, 0, 3).shape == (0, 3)


@pytest.mark.parametrize("seed", [0, 2**32 + 5, 2**64 - 1])
def test_seed_word_split(seed):
    om = G.omega_block(seed=seed, n=4, col0=0, w=2)
    assert np.all(np.isfinite(om))
