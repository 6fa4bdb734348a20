"""CPU checks of the C-ABI boundary: the library builds and loads, exports
every function include/qb.h declares, and rejects invalid arguments on the
host before touching a device (no compute call is made here)."""
import ctypes
import os
import re

import pytest

from paper_1503_07157_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qb.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(qb_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("qb_factor", "qb_workspace_bytes", "qb_status_string", "qb_sketch", "qb_orth"):
        assert required in names
    assert set(names) == set(_lib.SIGNATURES)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_status_strings():
    lib = _lib.load()
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6):
        assert lib.qb_status_string(code).startswith(b"QB_")
    assert lib.qb_status_string(12345) == b"QB_UNKNOWN"


def test_workspace_sizes():
    lib = _lib.load()
    small = lib.qb_workspace_bytes(2000, 1000, 50, -1, 0)
    big = lib.qb_workspace_bytes(10000, 10000, 128, -1, 0)
    assert 2000 * 1000 * 8 < small < 64 * 2**20
    assert 10000 * 10000 * 8 < big < 2 * 10000 * 10000 * 8
    # overwriting A removes the residual copy
    assert lib.qb_workspace_bytes(10000, 10000, 128, -1, 1) < big - 7e8
    assert lib.qb_workspace_bytes(0, 10, 4, -1, 0) == 0
    assert lib.qb_workspace_bytes(10, 10, 0, -1, 0) == 0
    assert lib.qb_workspace_bytes(10, 10, 257, -1, 0) == 0
    assert lib.qb_orth_workspace_bytes(1000, 64) > 0
    assert lib.qb_orth_workspace_bytes(1000, 300) == 0


def test_invalid_arguments_rejected_on_host():
    lib = _lib.load()
    k = ctypes.c_int64(7)
    fake = ctypes.c_void_p(4096)
    args = dict(A=fake, m=10, n=8, lda=10, eps=0.1, b=4, P=0, seed=1, Q=fake, ldq=10, B=fake,
                ldb=8, kmax=-1)

    def call(**over):
        a = dict(args, **over)
        return lib.qb_factor(a["A"], a["m"], a["n"], a["lda"], a["eps"], a["b"], a["P"],
                             a["seed"], a["Q"], a["ldq"], a["B"], a["ldb"], a["kmax"],
                             ctypes.byref(k), None, None, 0, None, 0)

    assert call(A=None) == _lib.QB_EINVAL
    assert call(lda=9) == _lib.QB_EINVAL
    assert call(eps=-1.0) == _lib.QB_EINVAL
    assert call(eps=float("nan")) == _lib.QB_EINVAL
    assert call(eps=float("inf")) == _lib.QB_EINVAL
    assert call(b=0) == _lib.QB_EINVAL
    assert call(P=-1) == _lib.QB_EINVAL
    assert call(kmax=9) == _lib.QB_EINVAL
    assert call(ldb=3, kmax=4) == _lib.QB_EINVAL
    assert call(m=0) == _lib.QB_EINVAL
    assert call() == _lib.QB_EWORKSPACE          # NULL workspace
    assert k.value == 0
    assert lib.qb_sketch(1, 0, 0, 4, fake, 1, None) == _lib.QB_EINVAL
    assert lib.qb_sketch(1, 10, 0, 4, fake, 9, None) == _lib.QB_EINVAL


def test_adjoint_arguments_checked_on_host():
    lib = _lib.load()
    assert lib.qb_adjoint_workspace_bytes(4096, 2048, 64, 4, 1) > 0
    assert lib.qb_adjoint_workspace_bytes(100, 50, 16, 4, 0) == 0     # s b > min(m, n)
    assert lib.qb_adjoint_workspace_bytes(1000, 500, 300, 1, 0) == 0  # b > 256
    assert lib.qb_adjoint_workspace_bytes(1000, 500, 16, 2, 9) == 0   # P > 8
    assert lib.qb_adjoint_workspace_bytes(1000, 500, 16, 0, 0) == 0
    fake = ctypes.c_void_p(4096)
    base = [fake, 100, 80, 100, 8, 2, 0, 1, fake, 100, fake, 16, None, 100, None, 16,
            fake, 100, fake, 1 << 20, None]
    bad = list(base)
    bad[16] = None                                  # no dA
    assert lib.qb_adjoint(*bad) == _lib.QB_EINVAL
    bad = list(base)
    bad[9] = 50                                     # ldq < m
    assert lib.qb_adjoint(*bad) == _lib.QB_EINVAL
    bad = list(base)
    bad[11] = 8                                     # ldb < s b
    assert lib.qb_adjoint(*bad) == _lib.QB_EINVAL
    bad = list(base)
    bad[18] = None                                  # no workspace
    assert lib.qb_adjoint(*bad) == _lib.QB_EWORKSPACE


def test_batched_arguments_checked_on_host():
    lib = _lib.load()
    fake = 4096

    def prob(**kw):
        p = _lib.QBProblem()
        d = dict(A=fake, m=300, n=200, lda=300, eps=1.0, seed=1, kmax=-1, Q=fake, ldq=300,
                 B=fake, ldb=200, b=32)
        d.update(kw)
        for k, v in d.items():
            setattr(p, k, v)
        return p

    def ws(*ps):
        arr = (_lib.QBProblem * len(ps))(*ps)
        return lib.qb_factor_batched_workspace_bytes(arr, len(ps))

    assert ws(prob(), prob(m=4096, n=2048, lda=4096, ldq=4096, ldb=2048, b=64)) > 0
    assert ws(prob(b=65)) == 0          # panels up to 64 wide
    assert ws(prob(kmax=201)) == 0      # kmax > min(m, n)
    assert ws(prob(ldq=299)) == 0
    assert ws(prob(ldb=100)) == 0       # ldb < kmax
    assert ws(prob(eps=-1.0)) == 0
    assert ws(prob(A=None)) == 0
    arr = (_lib.QBProblem * 1)(prob(b=0))
    assert lib.qb_factor_batched(arr, 1, ctypes.c_void_p(256), 1 << 20, None) == _lib.QB_EINVAL


def test_batched_tile_table_checked_on_host():
    lib = _lib.load()
    R, T = _lib.BATCH_ROLES, _lib.BATCH_TILES
    saved = [[lib.qb_batched_get_tile(r, wc) for wc in range(3)] for r in range(len(R))]
    try:
        assert lib.qb_batched_get_tile(R["gram"], 0) == T["32x32"]
        assert lib.qb_batched_set_tile(R["b"], 2, T["16x16"]) == _lib.QB_EINVAL
        assert lib.qb_batched_set_tile(R["b"], 1, T["32x64"]) == _lib.QB_OK
        assert lib.qb_batched_set_tile(R["downdate"], 2, T["64x32"]) == _lib.QB_OK
        assert lib.qb_batched_set_tile(R["downdate"], 0, T["16x16"]) == _lib.QB_EINVAL
        assert lib.qb_batched_set_tile(R["downdate"], 0, T["32x32"]) == _lib.QB_OK
        assert lib.qb_batched_set_tile(7, 0, 0) == _lib.QB_EINVAL
        assert lib.qb_batched_set_tile(0, 3, 0) == _lib.QB_EINVAL
        assert lib.qb_batched_set_tile(0, 0, 5) == _lib.QB_EINVAL
        assert lib.qb_batched_get_tile(R["downdate"], 0) == T["32x32"]
    finally:
        for r in range(len(R)):
            for wc in range(3):
                assert lib.qb_batched_set_tile(r, wc, saved[r][wc]) == _lib.QB_OK


def test_size_limits_rejected_up_front():
    """Sizes the kernels cannot launch (32-bit tile offsets, the downdate
    grid) are refused before any device work, not midway through a run."""
    lib = _lib.load()
    assert lib.qb_workspace_bytes((1 << 24) - 1, 64, 64, -1, 0) == 0   # even_up(m) = 2^24
    assert lib.qb_workspace_bytes((1 << 24) - 2, 64, 64, -1, 0) > 0
    assert lib.qb_workspace_bytes(64, 65535 * 64 + 1, 64, -1, 0) == 0  # downdate grid
    assert lib.qb_workspace_bytes(64, 65535 * 64, 64, -1, 0) > 0
    assert lib.qb_workspace_bytes(100, 80, 16, 81, 0) == 0              # kmax > min(m, n)
    assert lib.qb_workspace_bytes(100, 80, 16, 0, 0) > 0                # capacity 0 is valid
    k = ctypes.c_int64(7)
    fake = ctypes.c_void_p(4096)
    ws = ctypes.c_void_p(1 << 20)
    for lda, ldq, ldb in ((1 << 24, 100, 80), (100, 1 << 24, 80), (100, 100, 1 << 24)):
        assert lib.qb_factor(fake, 100, 80, lda, 0.1, 16, 0, 1, fake, ldq, fake, ldb, -1,
                             ctypes.byref(k), None, ws, 1 << 30, None, 0) == _lib.QB_EINVAL
    assert lib.qb_factor(fake, 64, 65535 * 64 + 1, 64, 0.1, 16, 0, 1, fake, 64, fake, 64, -1,
                         ctypes.byref(k), None, ws, 1 << 30, None, 0) == _lib.QB_EINVAL


def _no_gpu_here() -> bool:
    import torch
    return torch.cuda.device_count() == 0


@pytest.mark.skipif(not _no_gpu_here(), reason="checks the answer on a machine without a GPU")
def test_no_device_is_reported():
    """With valid arguments and no usable device, every entry point that
    would launch work returns QB_ENODEVICE before touching a pointer."""
    lib = _lib.load()
    k = ctypes.c_int64(7)
    fake = ctypes.c_void_p(4096)
    ws = ctypes.c_void_p(1 << 20)
    assert lib.qb_factor(fake, 100, 80, 100, 0.1, 16, 0, 1, fake, 100, fake, 80, -1,
                         ctypes.byref(k), None, ws, 1 << 30, None, 0) == _lib.QB_ENODEVICE
    assert k.value == 0
    assert lib.qb_sketch(1, 10, 0, 4, fake, 10, None) == _lib.QB_ENODEVICE
    kept = ctypes.c_int32(3)
    assert lib.qb_orth(fake, 100, 8, 100, fake, 100, ctypes.byref(kept), ws, 1 << 30,
                       None) == _lib.QB_ENODEVICE
    assert lib.qb_frob2(fake, 10, 10, 10, ctypes.byref(ctypes.c_double()), None, ws, 1 << 30,
                        None) == _lib.QB_ENODEVICE
    assert lib.qb_status_string(_lib.QB_ENODEVICE).startswith(b"QB_ENODEVICE")


def test_noalloc_limits_checked_on_host():
    """qb_factor_noalloc rejects invalid sizes (QB_EINVAL) and problems whose
    workspace exceeds its fixed scratch (QB_ETOOBIG) before touching a
    device or a pointer."""
    lib = _lib.load()
    k = ctypes.c_int64(7)
    fake = ctypes.c_void_p(4096)
    # 4000 x 4000: the residual copy alone is 128 MB
    assert lib.qb_workspace_bytes(4000, 4000, 64, -1, 0) > _lib.QB_NOALLOC_SCRATCH_BYTES
    assert lib.qb_factor_noalloc(fake, 4000, 4000, 4000, 0.1, 64, 0, 1, fake, 4000, fake, 4000,
                                 -1, ctypes.byref(k), None, None, 0) == _lib.QB_ETOOBIG
    assert k.value == 0
    assert lib.qb_factor_noalloc(fake, 0, 10, 1, 0.1, 4, 0, 1, fake, 1, fake, 10, -1,
                                 ctypes.byref(k), None, None, 0) == _lib.QB_EINVAL
    assert lib.qb_status_string(_lib.QB_ETOOBIG).startswith(b"QB_ETOOBIG")
    if _no_gpu_here():
        assert lib.qb_factor_noalloc(fake, 100, 80, 100, 0.1, 16, 0, 1, fake, 100, fake, 80, -1,
                                     ctypes.byref(k), None, None, 0) == _lib.QB_ENODEVICE
