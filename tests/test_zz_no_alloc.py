"""qb_factor_noalloc (the entry point that runs in the library's fixed
device scratch) against qb_factor (caller workspace), through the C ABI.

Two calls in a row, the second on a smaller problem, so the second runs in
scratch that still holds the first call's contents.  Both calls must give
what qb_factor gives on the same input: the same rank, kept widths and stop
reason, and the same Q and B bit for bit (the same kernels run in the same
order; only the workspace address differs), which is stricter than the
float64 parity bar of 1e-10 ||A||_F.  A problem whose workspace exceeds the
scratch is rejected with QB_ETOOBIG before any device work."""
import math

import numpy as np
import pytest
import torch

import paper_1503_07157_amd as qbmi
from paper_1503_07157_amd import _lib
import synth

pytestmark = pytest.mark.gpu


def _dev(x):
    return qbmi.colmajor(torch.from_numpy(np.ascontiguousarray(x)).cuda())


def _check_same(A, eps, b, P, seed):
    ref = qbmi.qb_factor(A, eps, b, P, seed)
    got = qbmi.qb_factor(A, eps, b, P, seed, noalloc=True)
    print(f"[case] {A.shape[0]}x{A.shape[1]} b={b} P={P} k={ref.k}/{got.k} "
          f"stop={ref.stop_reason}/{got.stop_reason}", flush=True)
    assert got.k == ref.k and got.k > 0
    assert got.widths == ref.widths
    assert got.stop_reason == ref.stop_reason and got.status == ref.status
    assert got.E == ref.E and got.D == ref.D
    assert torch.equal(got.Q, ref.Q)
    assert torch.equal(got.B, ref.B)
    nA = float(torch.linalg.norm(A))
    assert float(torch.linalg.norm(got.Q @ got.B - ref.Q @ ref.B)) <= 1e-10 * nA


def test_noalloc_matches_qb_factor_twice(cuda):
    lib = _lib.load()
    big = (2000, 1000, 50, 0)
    small = (700, 400, 32, 1)
    for m, n, b, _ in (big, small):
        assert 0 < lib.qb_workspace_bytes(m, n, b, -1, 0) <= _lib.QB_NOALLOC_SCRATCH_BYTES
    s = np.exp(-np.arange(1, 1001) / 40.0)
    A1 = _dev(synth.prescribed_svd(2000, 1000, s, 1001, 1002))
    _check_same(A1, 1e-6 * float(torch.linalg.norm(A1)), 50, 0, 1503)
    s2 = synth.spectrum("exp", 400, scale=12.0)
    A2 = _dev(synth.prescribed_svd(700, 400, s2, 71, 72))
    _check_same(A2, 1e-7 * float(torch.linalg.norm(A2)), 32, 1, 77)


def test_noalloc_rejects_problems_beyond_the_scratch(cuda):
    m, n = 4000, 4000  # 128 MB residual copy alone exceeds the 128 MiB scratch
    A = torch.zeros((n, m), dtype=torch.float64, device="cuda").t()
    with pytest.raises(qbmi.QBError) as e:
        qbmi.qb_factor(A, 0.1, 64, 0, 1, noalloc=True)
    assert e.value.code == _lib.QB_ETOOBIG
