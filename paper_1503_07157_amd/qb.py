"""Python face of the C ABI: torch tensors in, torch tensors out.

Only argument marshalling happens here: device pointers, sizes, strides and
the current HIP stream of torch are passed to libqbmi.so, which runs every
step on the GPU.  Matrices are column-major float64 device tensors, i.e.
tensors of shape (m, n) with strides (1, ld), ld >= m (use
`colmajor(x)` to obtain one).
"""
from __future__ import annotations

import ctypes
import json
import os
from dataclasses import dataclass, field

import torch

from . import _lib
from ._lib import (QBError, QBInfo, QBProblem, QB_BGEMM, QB_SAMPLE, QB_OVERWRITE_A, QB_POWER_NO_ORTH,
                   QB_SINGLE_BLOCK, QB_NO_SPECULATE, QB_STOP)


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def colmajor(x: torch.Tensor) -> torch.Tensor:
    """Column-major (Fortran-order) float64 copy of a 2-D tensor on its device."""
    if x.dim() != 2:
        raise ValueError("expected a matrix")
    m, n = x.shape
    out = torch.empty((n, m), dtype=torch.float64, device=x.device).t()
    out.copy_(x)
    return out


def _ld(x: torch.Tensor, name: str, dtype=torch.float64) -> int:
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {str(dtype).replace('torch.', '')}")
    if not x.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if x.dim() != 2:
        raise ValueError(f"{name} must be a matrix")
    m, n = x.shape
    if x.stride(0) != 1 and m > 1:
        raise ValueError(f"{name} must be column-major (stride(0) == 1)")
    ld = x.stride(1) if n > 1 else max(m, 1)
    return max(ld, m, 1)


def _check(code: int, where: str) -> int:
    if code < 0:
        raise QBError(code, where)
    return code


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)


def _aligned_ptr(ws: torch.Tensor) -> int:
    p = ws.data_ptr()
    return (p + 255) & ~255


@dataclass
class QBResult:
    Q: torch.Tensor
    B: torch.Tensor
    k: int
    status: int
    stop_reason: str
    normA2: float
    indicator: float
    resid2: float
    blocks: int
    widths: list = field(default_factory=list)
    E: list = field(default_factory=list)
    D: list = field(default_factory=list)
    R: torch.Tensor | None = None


def _trace_record(rec: dict) -> None:
    """QB_TRACE=1: one JSON line per qb_factor call (sizes, rank, stop
    reason and the per-block kept widths, tracked E_i and direct D_i) appended
    to QB_TRACE_FILE (default qb_trace.jsonl)."""
    with open(os.environ.get("QB_TRACE_FILE", "qb_trace.jsonl"), "a") as f:
        f.write(json.dumps(rec) + "\n")


def workspace_bytes(m, n, b, kmax=-1, sample="f64", overwrite=False) -> int:
    flags = QB_SAMPLE[sample] | (QB_OVERWRITE_A if overwrite else 0)
    return int(_lib.load().qb_workspace_bytes(m, n, b, kmax, flags))


def qb_factor(A: torch.Tensor, eps: float, b: int, power_iters: int = 0, seed: int = 0,
              kmax: int | None = None, sample: str = "f64", overwrite: bool = False,
              trace_cap: int = 4096, workspace: torch.Tensor | None = None,
              Q: torch.Tensor | None = None, B: torch.Tensor | None = None,
              bgemm: str = "f64", power_orth: bool = True,
              single_block: bool = False, speculate: bool = True,
              noalloc: bool = False) -> QBResult:
    """Blocked adaptive randomized QB (randQB_pb) of the column-major float64
    device matrix A to Frobenius tolerance eps.  Returns Q[:, :k], B[:k, :].
    sample / bgemm: precision of the sampling products and of B_i = Q_i^T A
    ("f64", "f32", "bf16x3").  power_orth=False skips the orthonormalisation
    between applications of A and A^T; single_block=True stops after the
    first block (the unblocked scheme with l = b).  speculate=False queues no
    work past the stop decision (QB_NO_SPECULATE).  noalloc=True calls
    qb_factor_noalloc, which runs in the library's fixed device scratch
    (`workspace` is then ignored; Q and B are still allocated here unless
    passed)."""
    lib = _lib.load()
    lda = _ld(A, "A")
    m, n = A.shape
    r = min(m, n)
    kcap = r if kmax is None else int(kmax)
    dev = A.device
    if Q is None:
        Q = torch.empty((max(kcap, 1), m), dtype=torch.float64, device=dev).t()
    if B is None:
        B = torch.empty((n, max(kcap, 1)), dtype=torch.float64, device=dev).t()
    ldq, ldb = _ld(Q, "Q"), _ld(B, "B")
    flags = (QB_SAMPLE[sample] | QB_BGEMM[bgemm] | (QB_OVERWRITE_A if overwrite else 0)
             | (0 if power_orth else QB_POWER_NO_ORTH) | (QB_SINGLE_BLOCK if single_block else 0)
             | (0 if speculate else QB_NO_SPECULATE))
    if not noalloc:
        need = int(lib.qb_workspace_bytes(m, n, b, kcap, flags))
        if need == 0:
            raise QBError(_lib.QB_EINVAL, "qb_workspace_bytes")
        if workspace is None or workspace.numel() < need + 256:
            workspace = _workspace(need, dev)
    info = QBInfo()
    tw = (ctypes.c_int32 * trace_cap)()
    tE = (ctypes.c_double * trace_cap)()
    tD = (ctypes.c_double * trace_cap)()
    info.trace_cap = trace_cap
    info.trace_w = ctypes.cast(tw, ctypes.POINTER(ctypes.c_int32))
    info.trace_E = ctypes.cast(tE, ctypes.POINTER(ctypes.c_double))
    info.trace_D = ctypes.cast(tD, ctypes.POINTER(ctypes.c_double))
    k = ctypes.c_int64(0)
    if noalloc:
        code = lib.qb_factor_noalloc(A.data_ptr(), m, n, lda, float(eps), int(b),
                                     int(power_iters), int(seed) & 0xFFFFFFFFFFFFFFFF,
                                     Q.data_ptr(), ldq, B.data_ptr(), ldb, kcap, ctypes.byref(k),
                                     ctypes.byref(info), _stream(dev), flags)
        _check(code, "qb_factor_noalloc")
    else:
        code = lib.qb_factor(A.data_ptr(), m, n, lda, float(eps), int(b), int(power_iters),
                             int(seed) & 0xFFFFFFFFFFFFFFFF, Q.data_ptr(), ldq, B.data_ptr(), ldb,
                             kcap, ctypes.byref(k), ctypes.byref(info), _aligned_ptr(workspace),
                             need, _stream(dev), flags)
        _check(code, "qb_factor")
    kk = int(k.value)
    L = info.trace_len
    if os.environ.get("QB_TRACE") == "1":
        _trace_record({"m": m, "n": n, "b": int(b), "power_iters": int(power_iters),
                       "seed": int(seed), "sample": sample, "bgemm": bgemm, "eps": float(eps),
                       "k": kk, "blocks": int(info.blocks), "status": int(code),
                       "stop": QB_STOP.get(info.stop_reason, str(info.stop_reason)),
                       "normA2": info.normA2, "widths": list(tw[:L]), "E": list(tE[:L]),
                       "D": list(tD[:L])})
    return QBResult(Q=Q[:, :kk], B=B[:kk, :], k=kk, status=code,
                    stop_reason=QB_STOP.get(info.stop_reason, str(info.stop_reason)),
                    normA2=info.normA2, indicator=info.indicator, resid2=info.resid2,
                    blocks=info.blocks, widths=list(tw[:L]), E=list(tE[:L]), D=list(tD[:L]),
                    R=A if overwrite else None)


def sketch(seed: int, n: int, col0: int, w: int, device="cuda") -> torch.Tensor:
    """Columns [col0, col0 + w) of the n x inf Gaussian sketch (column-major)."""
    out = torch.empty((w, n), dtype=torch.float64, device=device).t()
    _check(_lib.load().qb_sketch(int(seed) & 0xFFFFFFFFFFFFFFFF, n, col0, w, out.data_ptr(),
                                 max(n, 1), _stream(out.device)), "qb_sketch")
    return out


def orth(X: torch.Tensor):
    """CholQR2 with dropping.  Returns (Q, kept): Q has the kept columns first."""
    lib = _lib.load()
    ldx = _ld(X, "X")
    m, w = X.shape
    Qo = torch.empty((w, m), dtype=torch.float64, device=X.device).t()
    need = int(lib.qb_orth_workspace_bytes(m, w))
    ws = _workspace(need, X.device)
    kept = ctypes.c_int32(0)
    _check(lib.qb_orth(X.data_ptr(), m, w, ldx, Qo.data_ptr(), max(m, 1), ctypes.byref(kept),
                       _aligned_ptr(ws), need, _stream(X.device)), "qb_orth")
    return Qo, int(kept.value)


def sample_product(X: torch.Tensor, W: torch.Tensor, precision: str = "f64") -> torch.Tensor:
    """Y = X W with the sampling kernel."""
    lib = _lib.load()
    ldx, ldw = _ld(X, "X"), _ld(W, "W")
    m, K = X.shape
    K2, w = W.shape
    assert K == K2
    Y = torch.empty((w, m), dtype=torch.float64, device=X.device).t()
    need = int(lib.qb_gemm_workspace_bytes(m, K, w))
    ws = _workspace(need, X.device)
    _check(lib.qb_sample(X.data_ptr(), m, K, ldx, W.data_ptr(), w, ldw, Y.data_ptr(), max(m, 1),
                         QB_SAMPLE[precision], _aligned_ptr(ws), need, _stream(X.device)),
           "qb_sample")
    return Y


def project(Qm: torch.Tensor, X: torch.Tensor, precision: str = "f64") -> torch.Tensor:
    """C = Q^T X with the projection kernel."""
    lib = _lib.load()
    ldq, ldx = _ld(Qm, "Q"), _ld(X, "X")
    K, w = Qm.shape
    K2, N = X.shape
    assert K == K2
    C = torch.empty((N, w), dtype=torch.float64, device=X.device).t()
    need = int(lib.qb_gemm_workspace_bytes(N, K, w))
    ws = _workspace(need, X.device)
    _check(lib.qb_project(Qm.data_ptr(), K, w, ldq, X.data_ptr(), N, ldx, C.data_ptr(), max(w, 1),
                          QB_SAMPLE[precision], _aligned_ptr(ws), need, _stream(X.device)),
           "qb_project")
    return C


def downdate(R: torch.Tensor, Qm: torch.Tensor, B: torch.Tensor) -> float:
    """R -= Q B in place; returns ||R||_F^2 after the update."""
    lib = _lib.load()
    ldr, ldq, ldb = _ld(R, "R"), _ld(Qm, "Q"), _ld(B, "B")
    m, n = R.shape
    w = Qm.shape[1]
    need = int(lib.qb_downdate_workspace_bytes(m, n))
    ws = _workspace(need, R.device)
    out = ctypes.c_double(0.0)
    _check(lib.qb_downdate(R.data_ptr(), m, n, ldr, Qm.data_ptr(), w, ldq, B.data_ptr(), ldb,
                           ctypes.byref(out), _aligned_ptr(ws), need, _stream(R.device)),
           "qb_downdate")
    return float(out.value)


def frob2(X: torch.Tensor):
    """(||X||_F^2, has_nonfinite)."""
    lib = _lib.load()
    ldx = _ld(X, "X")
    m, n = X.shape
    need = int(lib.qb_downdate_workspace_bytes(m, n))
    ws = _workspace(need, X.device)
    out = ctypes.c_double(0.0)
    bad = ctypes.c_int32(0)
    _check(lib.qb_frob2(X.data_ptr(), m, n, ldx, ctypes.byref(out), ctypes.byref(bad),
                        _aligned_ptr(ws), need, _stream(X.device)), "qb_frob2")
    return float(out.value), bool(bad.value)


def svd(Q: torch.Tensor, B: torch.Tensor):
    """Low-rank SVD of Q B (Section 3.3.1): returns (U, S, V, sweeps) with
    Q B = U diag(S) V^T, S non-increasing."""
    lib = _lib.load()
    ldq, ldb = _ld(Q, "Q"), _ld(B, "B")
    m, k = Q.shape
    k2, n = B.shape
    if k2 != k:
        raise ValueError("Q and B do not conform")
    dev = Q.device
    U = torch.empty((k, m), dtype=torch.float64, device=dev).t()
    V = torch.empty((k, n), dtype=torch.float64, device=dev).t()
    S = torch.empty(k, dtype=torch.float64, device=dev)
    need = int(lib.qb_svd_workspace_bytes(m, n, k))
    if need == 0:
        raise QBError(_lib.QB_EINVAL, "qb_svd_workspace_bytes")
    ws = _workspace(need, dev)
    sweeps = ctypes.c_int32(0)
    _check(lib.qb_svd(Q.data_ptr(), m, k, ldq, B.data_ptr(), n, ldb, U.data_ptr(), m,
                      S.data_ptr(), V.data_ptr(), n, ctypes.byref(sweeps), _aligned_ptr(ws),
                      need, _stream(dev)), "qb_svd")
    return U, S, V, int(sweeps.value)


def pivoted_qr(Q: torch.Tensor, B: torch.Tensor):
    """Partial column-pivoted QR from Q B (Section 3.3.2): returns
    (Qhat, R, perm) with (Q B)[:, perm] = Qhat R."""
    lib = _lib.load()
    ldq, ldb = _ld(Q, "Q"), _ld(B, "B")
    m, k = Q.shape
    k2, n = B.shape
    if k2 != k:
        raise ValueError("Q and B do not conform")
    dev = Q.device
    Qh = torch.empty((k, m), dtype=torch.float64, device=dev).t()
    R = torch.empty((n, k), dtype=torch.float64, device=dev).t()
    perm = torch.empty(n, dtype=torch.int64, device=dev)
    need = int(lib.qb_pivoted_qr_workspace_bytes(m, n, k))
    if need == 0:
        raise QBError(_lib.QB_EINVAL, "qb_pivoted_qr_workspace_bytes")
    ws = _workspace(need, dev)
    _check(lib.qb_pivoted_qr(Q.data_ptr(), m, k, ldq, B.data_ptr(), n, ldb, Qh.data_ptr(), m,
                             R.data_ptr(), k, perm.data_ptr(), _aligned_ptr(ws), need,
                             _stream(dev)), "qb_pivoted_qr")
    return Qh, R, perm


def qb_factor_batched(As, eps, bs, seeds, kmax=None):
    """Batched QB of the float32 column-major device matrices As (list):
    eps, bs, seeds per problem (lists).  Returns a list of QBResult (no
    trace), each with its own status.  The outputs of all problems share two
    device buffers (problem i's Q is m x kcap with ld m, its B kcap x n with
    ld kcap, each at an offset 16-byte aligned); each result holds views of
    its own part."""
    lib = _lib.load()
    count = len(As)
    if count == 0:
        return []
    dev = As[0].device
    probs = (QBProblem * count)()
    shapes = []
    offq = offb = 0
    for i, A in enumerate(As):
        if A.dtype != torch.float32:
            raise ValueError("qb_factor_batched takes float32 matrices")
        if A.device != dev:
            raise ValueError("qb_factor_batched takes matrices on one device")
        lda = _ld(A, "A", torch.float32)
        m, n = A.shape
        r = min(m, n)
        kc = r if kmax is None or int(kmax[i]) < 0 else int(kmax[i])
        kq = max(kc, 1)
        shapes.append((m, n, kq, offq, offb))
        offq += (kq * m + 1) & ~1
        offb += (kq * n + 1) & ~1
        p = probs[i]
        p.A, p.m, p.n, p.lda = A.data_ptr(), m, n, lda
        p.eps, p.seed, p.kmax = float(eps[i]), int(seeds[i]) & 0xFFFFFFFFFFFFFFFF, kc
        p.ldq, p.ldb = max(m, 1), kq
        p.b = int(bs[i])
    qbuf = torch.empty(max(offq, 1), dtype=torch.float64, device=dev)
    bbuf = torch.empty(max(offb, 1), dtype=torch.float64, device=dev)
    q0, b0 = qbuf.data_ptr(), bbuf.data_ptr()
    for i, (m, n, kq, oq, ob) in enumerate(shapes):
        probs[i].Q = q0 + 8 * oq
        probs[i].B = b0 + 8 * ob
    need = int(lib.qb_factor_batched_workspace_bytes(probs, count))
    if need == 0:
        raise QBError(_lib.QB_EINVAL, "qb_factor_batched_workspace_bytes")
    ws = _workspace(need, dev)
    _check(lib.qb_factor_batched(probs, count, _aligned_ptr(ws), need, _stream(dev)),
           "qb_factor_batched")
    out = []
    for i, (m, n, kq, oq, ob) in enumerate(shapes):
        p = probs[i]
        kk = int(p.k) if p.status >= 0 else 0
        Q = torch.as_strided(qbuf, (m, kk), (1, m), oq)
        B = torch.as_strided(bbuf, (kk, n), (1, kq), ob)
        out.append(QBResult(Q=Q, B=B, k=kk, status=int(p.status),
                            stop_reason=QB_STOP.get(p.stop_reason, str(p.stop_reason)),
                            normA2=p.normA2, indicator=float("nan"), resid2=p.resid2,
                            blocks=int(p.blocks), widths=[], E=[], D=[], R=None))
    return out


def qb_adjoint(A, Q, B, dQ, dB, b: int, blocks: int, power_iters: int, seed: int):
    """dA = J^T (dQ, dB) for the fixed-sketch map A -> (Q, B) (qb_factor with
    eps = 0, kmax = blocks * b, no dropped column); float64 column-major
    device tensors, dQ or dB may be None.  Raises QBError with
    QB_RANK_EXHAUSTED when a recomputed orthonormalisation loses rank."""
    lib = _lib.load()
    lda = _ld(A, "A")
    m, n = A.shape
    kt = int(b) * int(blocks)
    if Q.shape != (m, kt) or B.shape != (kt, n):
        raise ValueError("Q and B must be m x (blocks b) and (blocks b) x n")
    ldq, ldb = _ld(Q, "Q"), _ld(B, "B")
    pdq, lddq = (0, m) if dQ is None else (dQ.data_ptr(), _ld(dQ, "dQ"))
    pdb, lddb = (0, kt) if dB is None else (dB.data_ptr(), _ld(dB, "dB"))
    if dQ is not None and dQ.shape != Q.shape:
        raise ValueError("dQ must have the shape of Q")
    if dB is not None and dB.shape != B.shape:
        raise ValueError("dB must have the shape of B")
    dA = torch.empty((n, m), dtype=torch.float64, device=A.device).t()
    need = int(lib.qb_adjoint_workspace_bytes(m, n, int(b), int(blocks), int(power_iters)))
    if need == 0:
        raise QBError(_lib.QB_EINVAL, "qb_adjoint_workspace_bytes")
    ws = _workspace(need, A.device)
    code = lib.qb_adjoint(A.data_ptr(), m, n, lda, int(b), int(blocks), int(power_iters),
                          int(seed) & 0xFFFFFFFFFFFFFFFF, Q.data_ptr(), ldq, B.data_ptr(), ldb,
                          pdq, lddq, pdb, lddb, dA.data_ptr(), _ld(dA, "dA"), _aligned_ptr(ws),
                          need, _stream(A.device))
    if code != _lib.QB_OK:
        raise QBError(code, "qb_adjoint")
    return dA


def qb_fixed(A, b: int, blocks: int, power_iters: int, seed: int):
    """The fixed-sketch map A -> (Q, B): qb_factor with eps = 0 and kmax =
    blocks * b; raises unless it ran exactly `blocks` full blocks."""
    res = qb_factor(A, 0.0, b, power_iters, seed, kmax=int(b) * int(blocks))
    if res.k != int(b) * int(blocks) or res.blocks != int(blocks):
        raise QBError(_lib.QB_RANK_EXHAUSTED, "qb_fixed: a block lost rank")
    return res.Q, res.B


class QBFunction(torch.autograd.Function):
    """(Q, B) = QBFunction.apply(A, b, blocks, power_iters, seed): the
    fixed-sketch QB map with its hand-written adjoint (qb_adjoint) as the
    backward.  A may be float32 or float64 (column-major or not); it is
    widened to a column-major float64 copy, Q and B are float64 and the
    gradient is returned in A's dtype."""

    @staticmethod
    def forward(ctx, A, b, blocks, power_iters, seed):
        A64 = colmajor(A.detach())
        Q, B = qb_fixed(A64, b, blocks, power_iters, seed)
        ctx.save_for_backward(A64, Q, B)
        ctx.cfg = (int(b), int(blocks), int(power_iters), int(seed), A.dtype)
        return Q, B

    @staticmethod
    def backward(ctx, gQ, gB):
        A64, Q, B = ctx.saved_tensors
        b, blocks, P, seed, dtype = ctx.cfg
        dQ = None if gQ is None else colmajor(gQ)
        dB = None if gB is None else colmajor(gB)
        dA = qb_adjoint(A64, Q, B, dQ, dB, b, blocks, P, seed)
        return dA.to(dtype), None, None, None, None


def batched_tiles():
    """The batched products' tile classes: {role: [class for w <= 16, <= 32,
    <= 64]}, class names as in _lib.BATCH_TILES."""
    lib = _lib.load()
    names = {v: k for k, v in _lib.BATCH_TILES.items()}
    out = {}
    for role, r in _lib.BATCH_ROLES.items():
        out[role] = [names[_check(lib.qb_batched_get_tile(r, wc), "qb_batched_get_tile")]
                     for wc in range(3)]
    return out


def set_batched_tiles(table):
    """Set tile classes: table {role: [class per width class]} (partial
    tables allowed; None keeps an entry).  Raises QBError for a class not
    allowed for its role."""
    lib = _lib.load()
    for role, classes in table.items():
        for wc, name in enumerate(classes):
            if name is None:
                continue
            _check(lib.qb_batched_set_tile(_lib.BATCH_ROLES[role], wc, _lib.BATCH_TILES[name]),
                   f"qb_batched_set_tile({role}, {wc}, {name})")
