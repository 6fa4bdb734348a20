"""ctypes loader for the in-tree HIP library libqbmi.so (C ABI in include/qb.h).

The library is built by `paper_1503_07157_amd.build` (or
`__graft_entry__.build()`).  Loading fails loudly when it is missing: there
is no other implementation of these entry points.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqbmi.so")
# The host-AddressSanitizer build of the same sources (build.py --asan), for
# the CPU checks of the argument paths; QB_LIBRARY selects it.
ASAN_LIB_PATH = os.path.join(HERE, "libqbmi_asan.so")

c_i64 = ctypes.c_int64
c_i32 = ctypes.c_int32
c_u32 = ctypes.c_uint32
c_u64 = ctypes.c_uint64
c_dbl = ctypes.c_double
c_vp = ctypes.c_void_p
c_size = ctypes.c_size_t

QB_OK = 0
QB_KMAX = 1
QB_RANK_EXHAUSTED = 2
QB_NOT_CONVERGED = 3
QB_EINVAL = -1
QB_ENONFINITE = -2
QB_EWORKSPACE = -3
QB_EHIP = -4
QB_ENODEVICE = -5
QB_ETOOBIG = -6
QB_NOALLOC_SCRATCH_BYTES = 128 << 20

BATCH_ROLES = {"sample": 0, "gram": 1, "apply": 2, "reproj_c": 3, "reproj_q": 4, "b": 5,
               "downdate": 6}
BATCH_TILES = {"64x64": 0, "16x16": 1, "32x32": 2, "64x32": 3, "32x64": 4}
QB_STOP = {0: "TOL_TRACKED", 1: "TOL_DIRECT", 2: "RANK_CAP", 3: "EXHAUSTED", 4: "KMAX", 5: "ZERO"}

QB_OVERWRITE_A = 1 << 0
QB_SAMPLE = {"f64": 0 << 4, "f32": 1 << 4, "bf16x3": 2 << 4, "int8x8": 3 << 4}
QB_BGEMM = {"f64": 0 << 6, "f32": 1 << 6, "bf16x3": 2 << 6}
QB_POWER_NO_ORTH = 1 << 8
QB_SINGLE_BLOCK = 1 << 9
QB_NO_SPECULATE = 1 << 10


class QBInfo(ctypes.Structure):
    _fields_ = [
        ("k", c_i64),
        ("blocks", c_i32),
        ("stop_reason", c_i32),
        ("normA2", c_dbl),
        ("indicator", c_dbl),
        ("resid2", c_dbl),
        ("trace_cap", c_i32),
        ("trace_len", c_i32),
        ("trace_w", ctypes.POINTER(c_i32)),
        ("trace_E", ctypes.POINTER(c_dbl)),
        ("trace_D", ctypes.POINTER(c_dbl)),
    ]


class QBProblem(ctypes.Structure):
    _fields_ = [
        ("A", c_vp),
        ("m", c_i64),
        ("n", c_i64),
        ("lda", c_i64),
        ("eps", c_dbl),
        ("seed", ctypes.c_uint64),
        ("kmax", c_i64),
        ("Q", c_vp),
        ("ldq", c_i64),
        ("B", c_vp),
        ("ldb", c_i64),
        ("b", c_i32),
        ("status", c_i32),
        ("stop_reason", c_i32),
        ("blocks", c_i32),
        ("k", c_i64),
        ("normA2", c_dbl),
        ("resid2", c_dbl),
    ]


# name -> (restype, argtypes)
SIGNATURES = {
    "qb_workspace_bytes": (c_size, [c_i64, c_i64, c_i32, c_i64, c_u32]),
    "qb_factor": (ctypes.c_int, [c_vp, c_i64, c_i64, c_i64, c_dbl, c_i32, c_i32, c_u64,
                                 c_vp, c_i64, c_vp, c_i64, c_i64,
                                 ctypes.POINTER(c_i64), ctypes.POINTER(QBInfo), c_vp, c_size,
                                 c_vp, c_u32]),
    "qb_factor_noalloc": (ctypes.c_int, [c_vp, c_i64, c_i64, c_i64, c_dbl, c_i32, c_i32, c_u64,
                                         c_vp, c_i64, c_vp, c_i64, c_i64,
                                         ctypes.POINTER(c_i64), ctypes.POINTER(QBInfo), c_vp,
                                         c_u32]),
    "qb_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "qb_sketch": (ctypes.c_int, [c_u64, c_i64, c_i64, c_i32, c_vp, c_i64, c_vp]),
    "qb_orth_workspace_bytes": (c_size, [c_i64, c_i32]),
    "qb_orth": (ctypes.c_int, [c_vp, c_i64, c_i32, c_i64, c_vp, c_i64, ctypes.POINTER(c_i32),
                               c_vp, c_size, c_vp]),
    "qb_gemm_workspace_bytes": (c_size, [c_i64, c_i64, c_i32]),
    "qb_sample": (ctypes.c_int, [c_vp, c_i64, c_i64, c_i64, c_vp, c_i32, c_i64, c_vp, c_i64,
                                 c_u32, c_vp, c_size, c_vp]),
    "qb_project": (ctypes.c_int, [c_vp, c_i64, c_i32, c_i64, c_vp, c_i64, c_i64, c_vp, c_i64,
                                  c_u32, c_vp, c_size, c_vp]),
    "qb_downdate_workspace_bytes": (c_size, [c_i64, c_i64]),
    "qb_downdate": (ctypes.c_int, [c_vp, c_i64, c_i64, c_i64, c_vp, c_i32, c_i64, c_vp, c_i64,
                                   ctypes.POINTER(c_dbl), c_vp, c_size, c_vp]),
    "qb_frob2": (ctypes.c_int, [c_vp, c_i64, c_i64, c_i64, ctypes.POINTER(c_dbl),
                                ctypes.POINTER(c_i32), c_vp, c_size, c_vp]),
    "qb_svd_workspace_bytes": (c_size, [c_i64, c_i64, c_i64]),
    "qb_svd": (ctypes.c_int, [c_vp, c_i64, c_i64, c_i64, c_vp, c_i64, c_i64, c_vp, c_i64, c_vp,
                              c_vp, c_i64, ctypes.POINTER(c_i32), c_vp, c_size, c_vp]),
    "qb_pivoted_qr_workspace_bytes": (c_size, [c_i64, c_i64, c_i64]),
    "qb_pivoted_qr": (ctypes.c_int, [c_vp, c_i64, c_i64, c_i64, c_vp, c_i64, c_i64, c_vp, c_i64,
                                     c_vp, c_i64, c_vp, c_vp, c_size, c_vp]),
    "qb_factor_batched_workspace_bytes": (c_size, [ctypes.POINTER(QBProblem), c_i32]),
    "qb_factor_batched": (ctypes.c_int, [ctypes.POINTER(QBProblem), c_i32, c_vp, c_size, c_vp]),
    "qb_batched_set_tile": (ctypes.c_int, [c_i32, c_i32, c_i32]),
    "qb_batched_get_tile": (ctypes.c_int, [c_i32, c_i32]),
    "qb_adjoint_workspace_bytes": (c_size, [c_i64, c_i64, c_i32, c_i32, c_i32]),
    "qb_adjoint": (ctypes.c_int, [c_vp, c_i64, c_i64, c_i64, c_i32, c_i32, c_i32, c_u64,
                                  c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64,
                                  c_vp, c_i64, c_vp, c_size, c_vp]),
    "qb_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "qb_profile_count": (c_i32, []),
    "qb_profile_name": (ctypes.c_char_p, [c_i32]),
    "qb_profile_read": (ctypes.c_int, [c_i32, ctypes.POINTER(c_dbl), ctypes.POINTER(c_i64),
                                       ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl)]),
}

_lock = threading.Lock()
_lib = None


def load(path: str | None = None) -> ctypes.CDLL:
    """Load libqbmi.so (or the library QB_LIBRARY names) and attach
    signatures; raises if it is not built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if path is None:
            path = os.environ.get("QB_LIBRARY") or LIB_PATH
        if not os.path.exists(path):
            raise RuntimeError(
                f"{path} is not built; run `python -m paper_1503_07157_amd.build` "
                "(the HIP library is the only implementation)")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def status_string(code: int) -> str:
    return load().qb_status_string(code).decode()


class QBError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {status_string(code)} ({code})")
        self.code = code
