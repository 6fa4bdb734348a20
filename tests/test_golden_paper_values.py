"""Values the paper prints (tests/golden/, each file citing its passage),
checked against the input generator and the oracle's rank helper.

Section 6.2 describes Matrix 1 (800 x 600, d_j about g_j^2 0.65^(j-1)) and
states that its rank to precision 1e-15 is about 75: the generator's
spectrum must give that rank (counted as singular values above 1e-15 s_1,
read as "about": within 10), whatever the seed of the g_j, and the
singular values of the assembled matrix must agree with the prescribed
ones, so the same count holds for the matrix the experiments factor."""
import os

import numpy as np

import synth
from oracle.checks import eps_rank

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_matrix1_rank_about_75():
    g = _read("matrix1_section6_2.txt")
    m, n, prec, rank = int(g["m"]), int(g["n"]), g["precision"], g["rank_about"]
    for seed in range(1, 9):
        d = synth.spectrum("m1", min(m, n), seed=seed)
        assert d[0] > 0 and np.all(np.diff(d) <= 0)
        r = int(np.sum(d > prec * d[0]))
        assert abs(r - rank) <= 10, (seed, r)
        # successive ratios follow beta^(j-1) up to the random g_j^2 factors:
        # on average the log-decay per index is log(beta)
        slope = np.polyfit(np.arange(r), np.log(d[:r]), 1)[0]
        assert abs(slope - np.log(g["beta"])) < 0.1, (seed, slope)
    A = synth.paper_matrix1(m, n, seed=1)
    s = np.linalg.svd(A, compute_uv=False)
    d = synth.spectrum("m1", min(m, n), seed=1)
    assert np.allclose(s[:60], d[:60], rtol=1e-10, atol=1e-14 * s[0])
    r = int(np.sum(s > prec * s[0]))
    assert abs(r - rank) <= 10, r


def test_matrix1_frobenius_eps_rank_near_75():
    # the same statement through the oracle's rank helper: the smallest k
    # whose Frobenius tail is below 1e-15 ||A||_F sits near the printed rank
    g = _read("matrix1_section6_2.txt")
    d = synth.spectrum("m1", 600, seed=1)
    k = eps_rank(d, g["precision"] * np.linalg.norm(d))
    assert abs(k - g["rank_about"]) <= 10, k
