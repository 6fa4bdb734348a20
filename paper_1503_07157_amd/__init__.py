"""Blocked randomized QB factorisation (randQB_b / randQB_pb) on AMD MI355X.

The computation lives in the HIP library libqbmi.so (C ABI: include/qb.h);
this package only loads it and marshals torch tensors into its calls.
"""
from ._lib import QBError, load  # noqa: F401
from .qb import (  # noqa: F401
    QBFunction,
    QBResult,
    batched_tiles,
    colmajor,
    downdate,
    frob2,
    orth,
    pivoted_qr,
    project,
    qb_adjoint,
    qb_factor,
    qb_factor_batched,
    qb_fixed,
    sample_product,
    set_batched_tiles,
    sketch,
    svd,
    workspace_bytes,
)
