"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and
the benchmark.

This package only *generates* matrices and index patterns.  It holds none of
the permanent arithmetic, so that the oracle (``oracle/``) and the HIP path
(``paper_1606_05836_amd``) can both consume the same bytes without sharing any
code of the method itself.
"""
from .gen import (  # noqa: F401
    haar,
    int_matrix,
    all_r,
    diag_matrix,
    submatrix,
    sha256_of,
    haar400_block20,
    int12_matrix,
    mixed_batch_16_26,
    haar1600_block,
    grad_batch_20,
    boson_workload,
    collision_pattern,
)
