"""Seeded synthetic matrices with prescribed singular values.

The construction follows the paper's accuracy test matrices (Section 6.2,
"Matrix 1", "Matrix 2", "Matrix 5"): A = U diag(d) V^T where U and V are
random matrices with orthonormal columns obtained from the QR factorisation
of Gaussian matrices.  The speed experiments of Section 6.1 note that the
choice of matrix does not matter for run time, so the timed workloads use the
same family with the singular-value profiles of the benchmark configurations.

All matrices are returned in column-major (Fortran) order, float64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# ---------------------------------------------------------------------------
# singular-value profiles
# ---------------------------------------------------------------------------
def spectrum(kind: str, r: int, **kw) -> np.ndarray:
    """Return r singular values s_1 >= s_2 >= ... (index j is 1-based).

    kind:
      "exp"    s_j = exp(-j / scale)                    (scale=40)
      "power"  s_j = j^(-p)                             (p=2)
      "gap"    s_j = 1 for j <= g, `low` after          (g=500, low=1e-6)
      "geom"   s_j = ratio^j                            (ratio)
      "m1"     Matrix 1 of the paper: g_j^2 * 0.65^(j-1), g_j ~ U[0,1], sorted
      "m2"     Matrix 2 of the paper: (1 + 200 (j-1))^(-1/2)
    """
    j = np.arange(1, r + 1, dtype=np.float64)
    if kind == "exp":
        return np.exp(-j / float(kw.get("scale", 40.0)))
    if kind == "power":
        return j ** (-float(kw.get("p", 2.0)))
    if kind == "gap":
        g = int(kw.get("g", 500))
        low = float(kw.get("low", 1e-6))
        return np.where(j <= g, 1.0, low)
    if kind == "geom":
        return float(kw["ratio"]) ** j
    if kind == "m1":
        rng = np.random.default_rng(int(kw.get("seed", 11)))
        g = rng.uniform(0.0, 1.0, size=r)
        d = g * g * 0.65 ** (j - 1)
        return np.sort(d)[::-1].copy()
    if kind == "m2":
        return (1.0 + 200.0 * (j - 1)) ** -0.5
    raise ValueError(f"unknown spectrum kind {kind!r}")


def random_orthonormal(rows: int, cols: int, seed: int) -> np.ndarray:
    """rows x cols matrix with orthonormal columns: Q factor of a seeded
    N(0,1) matrix (numpy PCG64)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((rows, cols))
    q, _ = np.linalg.qr(g)
    return q


def prescribed_svd(m: int, n: int, s: np.ndarray, seed_u: int, seed_v: int) -> np.ndarray:
    """A = U diag(s) V^T with len(s) <= min(m, n); column-major float64."""
    r = len(s)
    assert r <= min(m, n)
    u = random_orthonormal(m, r, seed_u)
    v = random_orthonormal(n, r, seed_v)
    a = (u * np.asarray(s, dtype=np.float64)[None, :]) @ v.T
    return np.asfortranarray(a)


def exact_rank(m: int, n: int, r: int, seed: int, cond: float = 1e3) -> np.ndarray:
    """Rank-r matrix, singular values log-spaced from 1 down to 1/cond."""
    s = np.logspace(0.0, -math.log10(cond), r) if r > 1 else np.ones(1)
    return prescribed_svd(m, n, s, seed, seed + 1)


def orthonormal_scaled(m: int, n: int, sigma: float, seed: int) -> np.ndarray:
    """sigma * U with U (m x n, m >= n) orthonormal: every singular value is
    sigma, so after k orthonormal directions taken from its range the
    residual is exactly sigma * sqrt(n - k)."""
    assert m >= n
    return np.asfortranarray(sigma * random_orthonormal(m, n, seed))


def kahan(n: int, zeta: float) -> np.ndarray:
    """Matrix 4 of the paper: S K with S = diag(1, zeta, zeta^2, ...) and K
    unit upper triangular with -phi above the diagonal, zeta^2 + phi^2 = 1."""
    phi = math.sqrt(1.0 - zeta * zeta)
    k = np.triu(np.full((n, n), -phi), 1) + np.eye(n)
    s = zeta ** np.arange(n, dtype=np.float64)
    return np.asfortranarray(s[:, None] * k)


def paper_matrix1(m: int = 800, n: int = 600, seed: int = 11) -> np.ndarray:
    return prescribed_svd(m, n, spectrum("m1", min(m, n), seed=seed), seed + 1, seed + 2)


def paper_matrix2(m: int = 800, n: int = 600, seed: int = 21) -> np.ndarray:
    return prescribed_svd(m, n, spectrum("m2", min(m, n)), seed + 1, seed + 2)


# ---------------------------------------------------------------------------
# benchmark / parity workloads
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    m: int
    n: int
    kind: str
    params: dict = field(default_factory=dict)
    b: int = 50
    power_iters: tuple = (0,)
    eps_rel: float = 1e-8
    seed_u: int = 0
    seed_v: int = 0
    seed_omega: int = 0
    note: str = ""

    def singular_values(self) -> np.ndarray:
        return spectrum(self.kind, min(self.m, self.n), **self.params)


WORKLOADS = {
    w.name: w
    for w in [
        Workload("exp40_2000x1000", 2000, 1000, "exp", {"scale": 40.0}, b=50,
                 power_iters=(0,), eps_rel=1e-6, seed_u=1001, seed_v=1002, seed_omega=1503,
                 note="plain FP64 QB, the small case the oracle finishes in seconds"),
        Workload("pow2_10000x10000", 10000, 10000, "power", {"p": 2.0}, b=128,
                 power_iters=(0, 1), eps_rel=1e-8, seed_u=2001, seed_v=2002, seed_omega=1504,
                 note="square FP64 QB with s_j = j^-2"),
        Workload("inv1_20000x16000", 20000, 16000, "power", {"p": 1.0}, b=256,
                 power_iters=(0,), eps_rel=1e-8, seed_u=3001, seed_v=3002, seed_omega=1505,
                 note="precision sweep, slow decay s_j = 1/j"),
        Workload("gap_20000x16000", 20000, 16000, "gap", {"g": 500, "low": 1e-6}, b=256,
                 power_iters=(0,), eps_rel=1e-8, seed_u=3003, seed_v=3004, seed_omega=1506,
                 note="precision sweep, spectral gap after 500"),
    ]
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def workload_matrix(name: str) -> np.ndarray:
    """CPU (numpy) construction; practical for the small workloads."""
    w = WORKLOADS[name]
    return prescribed_svd(w.m, w.n, w.singular_values(), w.seed_u, w.seed_v)


def workload_matrix_gpu(name: str, device="cuda"):
    """GPU construction with torch (device memory plumbing only): U and V are
    Q factors of seeded N(0,1) matrices drawn by torch's device generator.

    Returns a torch float64 tensor of shape (m, n) with column-major strides
    (1, m).  The values differ from `workload_matrix` (another RNG) but come
    from the same recipe; the same bytes are handed to both the GPU path and
    the oracle.
    """
    import torch

    w = WORKLOADS[name]
    m, n = w.m, w.n
    r = min(m, n)
    s = torch.as_tensor(w.singular_values(), dtype=torch.float64, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(w.seed_u)
    u = torch.linalg.qr(torch.randn((m, r), generator=gen, dtype=torch.float64, device=device))[0]
    gen.manual_seed(w.seed_v)
    v = torch.linalg.qr(torch.randn((n, r), generator=gen, dtype=torch.float64, device=device))[0]
    u.mul_(s[None, :])
    # (V (U s)^T) is A^T stored row-major, i.e. A stored column-major.
    at = v @ u.t()
    del u, v
    return at.t()


# ---- batched workload: many matrices of uneven sizes ------------------------
@dataclass(frozen=True)
class BatchSpec:
    m: int
    n: int
    r: float          # singular values s_j = r^j, j = 1 .. min(m, n)
    b: int
    seed_u: int
    seed_v: int
    seed_omega: int


def batch_specs(count: int = 512, seed: int = 4242, m_range=(256, 4096), n_max: int = 2048,
                r_range=(0.9, 0.995), blocks=(16, 32, 64)):
    """Sizes and spectra of a batch: m uniform in m_range, n uniform in
    [128, min(m, n_max)] (or [m/2, m] when m < 128), s_j = r^j with r
    uniform in r_range, b drawn from `blocks`."""
    g = np.random.default_rng(seed)
    out = []
    for i in range(count):
        m = int(g.integers(m_range[0], m_range[1] + 1))
        lo = min(128, m)
        n = int(g.integers(lo, min(m, n_max) + 1))
        r = float(g.uniform(*r_range))
        b = int(g.choice(blocks))
        out.append(BatchSpec(m, n, r, b, seed + 3 * i + 1, seed + 3 * i + 2, seed + 3 * i + 3))
    return out


def batch_singular_values(sp: BatchSpec) -> np.ndarray:
    return sp.r ** np.arange(1, min(sp.m, sp.n) + 1, dtype=np.float64)


def batch_matrix(sp: BatchSpec) -> np.ndarray:
    """float32 m x n (column-major) U diag(r^j) V^T, U and V from numpy QR."""
    A = prescribed_svd(sp.m, sp.n, batch_singular_values(sp), sp.seed_u, sp.seed_v)
    return np.asfortranarray(A.astype(np.float32))


def batch_matrix_gpu(sp: BatchSpec, device="cuda"):
    """GPU construction of the batch matrix (torch, device memory plumbing
    only): U diag(r^j) V^T with U and V the Q factors of seeded N(0,1)
    matrices from torch's device generator, built in float64 and rounded to
    float32.  Column-major (strides (1, m)).  The values differ from
    `batch_matrix` (another RNG); the same bytes go to both the GPU path and
    the oracle."""
    import torch

    m, n = sp.m, sp.n
    r = min(m, n)
    s = torch.as_tensor(batch_singular_values(sp), dtype=torch.float64, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(sp.seed_u)
    u = torch.linalg.qr(torch.randn((m, r), generator=gen, dtype=torch.float64, device=device))[0]
    gen.manual_seed(sp.seed_v)
    v = torch.linalg.qr(torch.randn((n, r), generator=gen, dtype=torch.float64, device=device))[0]
    u.mul_(s[None, :])
    at = (v @ u.t()).to(torch.float32)
    del u, v
    return at.t()
