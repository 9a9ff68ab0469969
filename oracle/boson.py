"""Exact boson-sampling output probabilities (main text, Eq. (1)).

TEST INFRASTRUCTURE ONLY (tests/, __graft_entry__.smoke(), bench.py's
cpu_baseline leg).

Pr[S -> T] = |Per(U_{S,T})|^2 / (s_1! ... s_m! t_1! ... t_m!), where U is the
m x m unitary of the network indexed [output mode, input mode] and U_{S,T} is
the n x n submatrix whose rows are the output modes of T, each repeated t_j
times, and whose columns are the input modes of S, each repeated s_i times.
(The paper states only that the submatrix comes from U; this is the standard
reading and the one the tests fix with the completeness sum below.)

Two independent exact routes to Per(U_{S,T}):
* ``prob_exact``: gather the matrix and run the exact Glynn oracle;
* ``perm_multiplicity``: Ryser's Eq. (S1) with the subsets grouped by how many
  copies of each repeated column they take.  With distinct columns c_l of
  multiplicity mu_l, a subset holding k_l copies of column l occurs
  C(mu_l, k_l) times and has row sums sum_l k_l c_il, so
  Per = (-1)^n sum_{0<=k_l<=mu_l} (-1)^{sum k} prod_l C(mu_l, k_l)
        prod_i sum_l k_l c_il.
  Repeated rows are turned into repeated columns by transposing
  (Per(A) = Per(A^T)).
"""
from __future__ import annotations

import itertools
import math
from collections import Counter
from fractions import Fraction

import numpy as np

from .exact import _as_rational_parts, perm_exact
from .pool import perm_exact_parallel


def gather_u_st(u: np.ndarray, in_modes, out_modes) -> np.ndarray:
    """U_{S,T}: rows = output modes (with repeats), columns = input modes
    (with repeats), both in the given order."""
    if isinstance(u, list):
        # exact entries (e.g. (re, im) Fraction pairs) stay Python objects
        return [[u[int(i)][int(j)] for j in in_modes] for i in out_modes]
    u = np.asarray(u)
    return np.ascontiguousarray(u[np.asarray(out_modes)][:, np.asarray(in_modes)])


def occupation_factorials(modes) -> int:
    """prod over modes of (number of photons in the mode)!"""
    out = 1
    for c in Counter(int(x) for x in modes).values():
        out *= math.factorial(c)
    return out


def prob_exact(u, in_modes, out_modes, workers: int | None = None) -> Fraction:
    """Exact Pr[S -> T] of Eq. (1) for the given (finite binary64) U."""
    a = gather_u_st(u, in_modes, out_modes)
    if workers is not None and workers > 1:
        pr, pi = perm_exact_parallel(a, workers)
    else:
        pr, pi = perm_exact(a)
    return (pr * pr + pi * pi) / (occupation_factorials(in_modes) * occupation_factorials(out_modes))


def perm_multiplicity(cols, mult):
    """Per of the n x n matrix whose columns are ``cols[l]`` (length-n vectors)
    repeated ``mult[l]`` times, by the grouped form of Eq. (S1).  Exact."""
    cols = [list(c) for c in cols]
    n = sum(mult)
    if n == 0:
        return Fraction(1), Fraction(0)
    if any(len(c) != n for c in cols):
        raise ValueError("each column must have n = sum(mult) entries")
    # exact Gaussian integers: scale every entry by the common denominator d
    parts = [[_as_rational_parts(x) for x in c] for c in cols]
    d = 1
    for c in parts:
        for re_, im_ in c:
            d = math.lcm(d, re_.denominator, im_.denominator)
    gcols = [[(int(re_ * d), int(im_ * d)) for re_, im_ in c] for c in parts]
    re = im = 0
    for ks in itertools.product(*[range(m + 1) for m in mult]):
        coeff = 1
        for m, k in zip(mult, ks):
            coeff *= math.comb(m, k)
        p_re, p_im = 1, 0
        for i in range(n):
            sr = sum(k * gcols[l][i][0] for l, k in enumerate(ks))
            si = sum(k * gcols[l][i][1] for l, k in enumerate(ks))
            p_re, p_im = p_re * sr - p_im * si, p_re * si + p_im * sr
        s = -1 if sum(ks) % 2 else 1
        re += s * coeff * p_re
        im += s * coeff * p_im
    if n % 2:
        re, im = -re, -im
    den = d ** n
    return Fraction(re, den), Fraction(im, den)


def prob_multiplicity(u, in_modes, out_modes) -> Fraction:
    """Pr[S -> T] of Eq. (1) through ``perm_multiplicity`` (independent of the
    Glynn route): transpose U_{S,T} so the repeated output rows become
    repeated columns."""
    u = np.asarray(u)
    in_modes = [int(x) for x in in_modes]
    cnt = Counter(int(x) for x in out_modes)
    modes = sorted(cnt)
    # column l of U_{S,T}^T is row `mode` of U restricted to the input modes
    cols = [[complex(u[mode, s]) for s in in_modes] for mode in modes]
    mult = [cnt[m] for m in modes]
    pr, pi = perm_multiplicity(cols, mult)
    return (pr * pr + pi * pi) / (occupation_factorials(in_modes) * occupation_factorials(out_modes))
