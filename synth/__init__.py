"""Seeded synthetic test matrices shared by the tests, the benchmark and the
smoke check.

This package builds inputs only.  It holds none of the arithmetic of the
blocked randomized QB method: no random sketch, no orthonormalisation of a
sample, no downdate, no stopping rule.  Both the CPU oracle and the GPU path
consume the bytes it produces.
"""
from .matrices import (  # noqa: F401
    spectrum,
    random_orthonormal,
    prescribed_svd,
    exact_rank,
    orthonormal_scaled,
    kahan,
    paper_matrix1,
    paper_matrix2,
    WORKLOADS,
    workload,
    workload_matrix,
    workload_matrix_gpu,
    BatchSpec,
    batch_specs,
    batch_singular_values,
    batch_matrix,
    batch_matrix_gpu,
)
