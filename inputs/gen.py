"""Seeded input generators (no permanent arithmetic lives here).

Workload recipes follow the paper's inputs where they are described: the
boson-sampling matrices are n x n submatrices of an m x m Haar-random unitary
(main text, Eq. (1) and the definition of U_{S,T} beside it); the precision
study uses all-r matrices and random unitaries (Supplementary tables on errors
of BB/FG and Ryser); the 45 x 45 production run used diag(1+i)
(Supplementary figure with the 13,000-node screenshot).  The paper's own
matrices are not published, so every matrix here is synthetic and seeded.

Haar(m, seed):
  1. rng = numpy.random.default_rng(seed)
  2. Z = (N(0,1) + i N(0,1)) / sqrt(2), an m x m complex Gaussian matrix
  3. Q, R = numpy.linalg.qr(Z)
  4. U = Q * diag(R_kk / |R_kk|)            (phase-fixed, Haar distributed)
"""
from __future__ import annotations

import functools
import hashlib

import numpy as np


@functools.lru_cache(maxsize=16)
def _haar_cached(m: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    z = (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    u = q * (d / np.abs(d))[None, :]
    u = np.ascontiguousarray(u, dtype=np.complex128)
    u.setflags(write=False)
    return u


def haar(m: int, seed: int) -> np.ndarray:
    """Seeded m x m Haar-random unitary, complex128, C-contiguous (read-only view)."""
    return _haar_cached(int(m), int(seed))


def submatrix(u: np.ndarray, rows, cols) -> np.ndarray:
    """Contiguous copy of u[rows][:, cols] (rows/cols may repeat)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    return np.ascontiguousarray(u[rows][:, cols], dtype=np.complex128)


def int_matrix(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """n x n integers uniform in [lo, hi] (inclusive), returned as complex128."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, (n, n)).astype(np.complex128)


def all_r(n: int, r: complex) -> np.ndarray:
    """The n x n matrix with every entry equal to r."""
    return np.full((n, n), complex(r), dtype=np.complex128)


def diag_matrix(n: int, d: complex) -> np.ndarray:
    """d on the diagonal, zero elsewhere (the paper's ``e`` input has d = 1+i)."""
    a = np.zeros((n, n), dtype=np.complex128)
    a[np.arange(n), np.arange(n)] = d
    return a


def sha256_of(a: np.ndarray) -> str:
    """SHA-256 of the C-contiguous bytes of an array (used to pin stored values)."""
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


# ---------------------------------------------------------------- workloads

def haar400_block20() -> np.ndarray:
    """Top-left 20 x 20 block of Haar(400, seed 11)."""
    return submatrix(haar(400, 11), range(20), range(20))


def int12_matrix() -> np.ndarray:
    """12 x 12 integer matrix, entries uniform in {-3..3}, seed 12."""
    return int_matrix(12, -3, 3, 12)


def mixed_batch_16_26(batch: int = 4096, seed_ns: int = 21, seed_rows: int = 22):
    """Batch of n x n submatrices with n ~ U{16..26}.

    For each n the parent is Haar(n^2, 2000+n); matrix b takes n distinct random
    rows (sorted) and the first n columns.  Returns (ns, list of matrices).
    """
    ns = np.random.default_rng(seed_ns).integers(16, 27, batch)
    rng = np.random.default_rng(seed_rows)
    mats = []
    for n in ns:
        n = int(n)
        u = haar(n * n, 2000 + n)
        rows = np.sort(rng.choice(n * n, n, replace=False))
        mats.append(submatrix(u, rows, range(n)))
    return ns.astype(np.int32), mats


def haar1600_block(n: int) -> np.ndarray:
    """n x n submatrix of Haar(1600, 31): sorted random rows (seed 32+n), first n columns."""
    u = haar(1600, 31)
    rows = np.sort(np.random.default_rng(32 + n).choice(1600, n, replace=False))
    return submatrix(u, rows, range(n))


def grad_batch_20(batch: int = 1024, n: int = 20):
    """batch x n x n submatrices of Haar(400, 41), rows drawn with seed 42."""
    u = haar(400, 41)
    rng = np.random.default_rng(42)
    out = np.empty((batch, n, n), dtype=np.complex128)
    for b in range(batch):
        rows = np.sort(rng.choice(400, n, replace=False))
        out[b] = submatrix(u, rows, range(n))
    return out


def collision_pattern(rng: np.random.Generator, m: int, n: int) -> np.ndarray:
    """One output pattern of n photons over m modes with collisions.

    c3 in {0,1,2} modes hold 3 photons, c2 in {1..5} modes hold 2, the rest hold
    one; the modes are distinct and uniform over [0, m).  Returned as the sorted
    list of n output-mode indices (a mode with t photons appears t times).
    """
    c3 = int(rng.integers(0, 3))
    c2 = int(rng.integers(1, 6))
    c1 = n - 3 * c3 - 2 * c2
    assert c1 >= 0
    modes = rng.choice(m, c3 + c2 + c1, replace=False)
    out = list(np.repeat(modes[:c3], 3)) + list(np.repeat(modes[c3:c3 + c2], 2)) + list(modes[c3 + c2:])
    return np.sort(np.asarray(out, dtype=np.int64))


def boson_workload(m: int = 900, n: int = 30, patterns: int = 256, seed_u: int = 51, seed_p: int = 52):
    """Boson-sampling workload: U = Haar(m, 51), inputs in modes 0..n-1 (one photon
    each), ``patterns`` collision output patterns drawn with seed 52.

    Returns (U, in_modes (n,), out_patterns (patterns, n) int64).
    """
    u = haar(m, seed_u)
    rng = np.random.default_rng(seed_p)
    pats = np.stack([collision_pattern(rng, m, n) for _ in range(patterns)])
    return u, np.arange(n, dtype=np.int64), pats

