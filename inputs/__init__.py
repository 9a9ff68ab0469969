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
    config1_haar20,
    config1_int12,
    config2_batch,
    config3_matrix,
    config4_batch,
    config5_workload,
    collision_pattern,
)
