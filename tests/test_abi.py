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
    for code in (0, 1, 2, -1, -2, -3, -4, -5):
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
