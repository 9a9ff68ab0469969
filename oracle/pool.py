"""Multi-process runner for the exact Glynn oracle.

TEST INFRASTRUCTURE ONLY (tests/, __graft_entry__.smoke(), bench.py's
cpu_baseline leg).

The Gray-index range [0, 2^(n-1)) is cut into contiguous pieces, one per
worker, and each worker seeds its row sums at the start of its piece -- the
contiguous per-process split of the parallel BB/FG listing in the
Supplementary section "Utilizing Multiple CPUs".  The partial sums are exact
integers, so the result does not depend on the split.
"""
from __future__ import annotations

import multiprocessing as mp
import os
from fractions import Fraction

from .exact import glynn_gray_raw, to_gaussian_integers


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def _work(args):
    g, k0, k1 = args
    return glynn_gray_raw(g, k0, k1)


def split_range(total: int, pieces: int):
    """Contiguous, near-equal pieces [k0, k1) covering [0, total)."""
    pieces = max(1, min(pieces, total))
    bounds = [total * p // pieces for p in range(pieces + 1)]
    return [(bounds[p], bounds[p + 1]) for p in range(pieces) if bounds[p] < bounds[p + 1]]


def glynn_raw_parallel(g, k_begin: int, k_end: int, workers: int | None = None):
    """Exact Glynn numerator over [k_begin, k_end) of a Gaussian-integer matrix,
    spread over ``workers`` processes."""
    workers = workers or host_cores()
    pieces = [(k_begin + a, k_begin + b) for a, b in split_range(k_end - k_begin, workers * 4)]
    if workers == 1 or len(pieces) == 1:
        parts = [_work((g, a, b)) for a, b in pieces]
    else:
        ctx = mp.get_context("fork")
        with ctx.Pool(workers) as pool:
            parts = pool.map(_work, [(g, a, b) for a, b in pieces])
    return sum(p[0] for p in parts), sum(p[1] for p in parts)


def perm_exact_parallel(a, workers: int | None = None):
    """Exact permanent (Fraction pair) by Eq. (S2) using several processes."""
    g, d = to_gaussian_integers(a)
    n = len(g)
    if n == 0:
        return Fraction(1), Fraction(0)
    re, im = glynn_raw_parallel(g, 0, 1 << (n - 1), workers)
    div = 1 << (n - 1)
    if re % div or im % div:
        raise ArithmeticError("Glynn numerator not divisible by 2^(n-1)")
    den = d ** n
    return Fraction(re // div, den), Fraction(im // div, den)
