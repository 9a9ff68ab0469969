"""Exact CPU oracle for the permanent of an n x n complex matrix.

TEST INFRASTRUCTURE ONLY.  This module is imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of ``bench.py``;
the product path (the HIP library and its Python binding) never imports,
links or runs anything under ``oracle/``.  It shares no code with the GPU
path.

What it computes (and from which passage of the paper):

* Definition.  Per(A) = sum over permutations s of prod_i a_{i, s(i)}.  The
  paper never writes the sum out, but its "theory" values r^n * n! for all-r
  matrices (Supplementary error tables) follow from it.  ``perm_brute``
  writes the definition out (small n only).

* Ryser's formula, Supplementary "Parallelization and Optimization",
  Eq. (S1): Per(A) = (-1)^n sum_{S subset of columns} (-1)^{|S|}
  prod_i sum_{j in S} a_ij.  ``ryser_subsets`` evaluates it in plain subset
  order, each subset's row sums formed from scratch (the original
  O(n^2 2^n) order the paper ran).  ``ryser_paired_int`` takes the load-
  balanced order of Algorithm S3: half the subsets, each with its
  complement.

* BB/FG (Glynn) formula, same section, Eq. (S2): Per(A) =
  [sum_delta (prod_k delta_k) prod_i sum_j delta_j a_ij] / 2^(n-1), with
  delta_1 = +1 and delta_k in {-1, +1}.  ``glynn_direct`` enumerates delta
  from scratch; ``glynn_gray_raw`` walks delta in reflected Gray-code order so
  that consecutive delta differ in one entry and each row sum changes by one
  column -- the O(n)-per-term order the same section names (and rejects on
  its cluster because of the data dependency; in exact arithmetic the order
  is irrelevant).

All arithmetic is exact.  A binary64 number is m * 2^e exactly, so a complex128
matrix times 2^E (E the largest binary exponent of a denominator) is a matrix
of Gaussian integers; every formula above is evaluated on that integer matrix
with Python ints and the power of two is divided out at the end as an exact
rational.  Results are returned as an ``(re, im)`` pair of ``Fraction``.

Readings of the paper taken here:
* Per of the 0 x 0 matrix is 1 (empty product); the 1 x 1 case is a_00.
* The fixed entry delta_1 = +1 of Eq. (S2) is column 0 (0-based).  Gray word
  g(k) = k XOR (k >> 1); bit b of g set means delta of column b+1 is -1, so
  k = 0 is the all-(+1) vector.
* Eq. (S2) sums delta over columns inside row sums (prod over rows i of
  sum over columns j); the parallel listing of the same algorithm writes the
  transposed form.  Per(A) = Per(A^T), so both are the same exact value.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np

# --------------------------------------------------------------- conversions


def _as_rational_parts(x):
    """Exact (re, im) rationals of one entry (Python int/float/complex/Fraction,
    numpy scalar, or an (re, im) pair)."""
    if isinstance(x, tuple):
        return Fraction(x[0]), Fraction(x[1])
    if isinstance(x, (int, np.integer)):
        return Fraction(int(x)), Fraction(0)
    if isinstance(x, Fraction):
        return x, Fraction(0)
    c = complex(x)
    return Fraction(c.real), Fraction(c.imag)


def to_gaussian_integers(a):
    """Scale a matrix to an exact Gaussian-integer matrix.

    Returns ``(G, D)`` where ``G[i][j] = (p, q)`` are Python ints and
    ``a[i][j] = (p + i q) / D`` exactly, with ``D`` the least common multiple
    of all denominators (a power of two for binary64 input).
    """
    rows = [[_as_rational_parts(x) for x in row] for row in _rows_of(a)]
    d = 1
    for row in rows:
        for re, im in row:
            d = math.lcm(d, re.denominator, im.denominator)
    g = [[(int(re * d), int(im * d)) for re, im in row] for row in rows]
    return g, d


def _rows_of(a):
    if isinstance(a, np.ndarray):
        if a.ndim != 2 or a.shape[0] != a.shape[1]:
            raise ValueError("square matrix expected")
        return [list(r) for r in a.tolist()]
    rows = [list(r) for r in a]
    if any(len(r) != len(rows) for r in rows):
        raise ValueError("square matrix expected")
    return rows


# ----------------------------------------------------- Gaussian-integer helpers


def _cmul(x, y):
    return (x[0] * y[0] - x[1] * y[1], x[0] * y[1] + x[1] * y[0])


def _prod(values):
    p = (1, 0)
    for v in values:
        p = _cmul(p, v)
    return p


# ----------------------------------------------------------------- definition


def perm_brute_int(g):
    """Definition of the permanent on a Gaussian-integer matrix: sum over all
    permutations s of prod_i g[i][s(i)].  Only for small n (n! terms)."""
    n = len(g)
    re = im = 0
    for s in itertools.permutations(range(n)):
        p = _prod(g[i][s[i]] for i in range(n))
        re += p[0]
        im += p[1]
    return re, im


# ------------------------------------------------------------ Ryser, Eq. (S1)


def ryser_subsets_int(g):
    """Eq. (S1) on a Gaussian-integer matrix, subsets in plain binary order,
    each subset's row sums formed from scratch.  Returns Per as an int pair."""
    n = len(g)
    if n == 0:
        return 1, 0
    re = im = 0
    for mask in range(1 << n):
        cols = [j for j in range(n) if (mask >> j) & 1]
        rowsums = []
        for i in range(n):
            sr = si = 0
            for j in cols:
                sr += g[i][j][0]
                si += g[i][j][1]
            rowsums.append((sr, si))
        p = _prod(rowsums)
        if len(cols) % 2:
            re -= p[0]
            im -= p[1]
        else:
            re += p[0]
            im += p[1]
    if n % 2:
        re, im = -re, -im
    return re, im


def ryser_paired_int(g):
    """Ryser's formula with the load balance of Supplementary Algorithm S3 on
    a Gaussian-integer matrix: the loop index it runs over [0, 2^(n-1)), bit
    i of it puts column i (of the first n - 1) in S, and each S contributes
    its own term of Eq. (S1) and the term of its complement S_C among all n
    columns -- so every subset of the n columns appears exactly once, and
    every iteration costs the same.  Row sums from scratch, as in the loop;
    returns Per as an int pair."""
    n = len(g)
    if n == 0:
        return 1, 0
    re = im = 0
    for it in range(1 << (n - 1)):
        s = [j for j in range(n - 1) if (it >> j) & 1]
        s_c = [j for j in range(n) if j not in s]
        for cols in (s, s_c):
            rowsums = [(sum(g[i][j][0] for j in cols), sum(g[i][j][1] for j in cols)) for i in range(n)]
            p = _prod(rowsums)
            if len(cols) % 2:
                re -= p[0]
                im -= p[1]
            else:
                re += p[0]
                im += p[1]
    if n % 2:
        re, im = -re, -im
    return re, im


def ryser_gray_raw(g, k_begin: int = 0, k_end: int | None = None):
    """Eq. (S1) before its (-1)^n factor, over the Gray indices k in
    [k_begin, k_end) of a Gaussian-integer matrix: the subset of index k is
    S = {columns b : bit b of gray(k) is set}, and its term
    (-1)^|S| prod_i sum_{j in S} g_ij is formed from scratch.  Returns the
    exact partial sum as ints (the empty set contributes 0 for n >= 1)."""
    n = len(g)
    total = 1 << n
    if k_end is None:
        k_end = total
    if not 0 <= k_begin <= k_end <= total:
        raise ValueError("Gray range out of bounds")
    re = im = 0
    for k in range(k_begin, k_end):
        word = gray(k)
        cols = [j for j in range(n) if (word >> j) & 1]
        rowsums = [(sum(g[i][j][0] for j in cols), sum(g[i][j][1] for j in cols)) for i in range(n)]
        p = _prod(rowsums)
        if len(cols) % 2:
            re -= p[0]
            im -= p[1]
        else:
            re += p[0]
            im += p[1]
    return re, im


# ------------------------------------------------------------ Glynn, Eq. (S2)


def glynn_direct_raw(g):
    """Numerator of Eq. (S2) on a Gaussian-integer matrix, every delta vector
    built from scratch (delta_0 = +1, delta_j = -1 iff bit j-1 of the counter
    is set).  Returns the raw sum (not divided by 2^(n-1))."""
    n = len(g)
    re = im = 0
    for mask in range(1 << (n - 1)):
        delta = [1] + [(-1 if (mask >> (j - 1)) & 1 else 1) for j in range(1, n)]
        sign = 1
        for d in delta:
            sign *= d
        rowsums = []
        for i in range(n):
            sr = si = 0
            for j in range(n):
                sr += delta[j] * g[i][j][0]
                si += delta[j] * g[i][j][1]
            rowsums.append((sr, si))
        p = _prod(rowsums)
        re += sign * p[0]
        im += sign * p[1]
    return re, im


def gray(k: int) -> int:
    """Reflected binary Gray code of k."""
    return k ^ (k >> 1)


def delta_of_word(word: int, n: int):
    """delta vector of Eq. (S2) for a Gray word: delta_0 = +1 and
    delta_{b+1} = -1 iff bit b of the word is set."""
    return [1] + [(-1 if (word >> b) & 1 else 1) for b in range(n - 1)]


def flipped_column(old_word: int, new_word: int) -> int:
    """Column whose delta flips between two consecutive Gray words (they differ
    in one bit b, which drives column b+1)."""
    changed = old_word ^ new_word
    return changed.bit_length()


def glynn_gray_raw(g, k_begin: int = 0, k_end: int | None = None):
    """Numerator of Eq. (S2) over the Gray indices k in [k_begin, k_end).

    The walk keeps delta and the row sums r_i = sum_j delta_j g_ij.  At k_begin
    both are formed from scratch from the Gray word g(k_begin); each later
    index changes the Gray word in one bit, i.e. flips one delta_c, and every
    row sum moves by 2 * delta_c(new) * g_ic.  The term added at index k is
    (prod_k delta_k) * prod_i r_i.  Returns the exact partial sum as ints.
    """
    n = len(g)
    if n == 0:
        return (1, 0) if k_begin == 0 and (k_end is None or k_end > 0) else (0, 0)
    total = 1 << (n - 1)
    if k_end is None:
        k_end = total
    if not 0 <= k_begin <= k_end <= total:
        raise ValueError("Gray range out of bounds")
    if k_begin == k_end:
        return 0, 0
    word = gray(k_begin)
    delta = delta_of_word(word, n)
    sign = 1
    for d in delta:
        sign *= d
    r_re = [sum(delta[j] * g[i][j][0] for j in range(n)) for i in range(n)]
    r_im = [sum(delta[j] * g[i][j][1] for j in range(n)) for i in range(n)]
    acc_re = acc_im = 0
    for k in range(k_begin, k_end):
        if k != k_begin:
            new_word = gray(k)
            c = flipped_column(word, new_word)
            word = new_word
            delta[c] = -delta[c]
            sign = -sign
            two_d = 2 * delta[c]
            for i in range(n):
                r_re[i] += two_d * g[i][c][0]
                r_im[i] += two_d * g[i][c][1]
        p_re, p_im = r_re[0], r_im[0]
        for i in range(1, n):
            x, y = r_re[i], r_im[i]
            p_re, p_im = p_re * x - p_im * y, p_re * y + p_im * x
        if sign > 0:
            acc_re += p_re
            acc_im += p_im
        else:
            acc_re -= p_re
            acc_im -= p_im
    return acc_re, acc_im


def glynn_gray_int(g):
    """Per of a Gaussian-integer matrix by Eq. (S2) in Gray order.  Asserts that
    the raw sum is divisible by 2^(n-1) (it is 2^(n-1) Per, an integer)."""
    n = len(g)
    if n == 0:
        return 1, 0
    re, im = glynn_gray_raw(g)
    div = 1 << (n - 1)
    if re % div or im % div:
        raise ArithmeticError("Glynn numerator not divisible by 2^(n-1)")
    return re // div, im // div


# ------------------------------------------------------------ public wrappers


def _scaled(result, d, n):
    den = d ** n
    return Fraction(result[0], den), Fraction(result[1], den)


def perm_exact(a, method: str = "glynn"):
    """Exact permanent of ``a`` as an (re, im) pair of Fractions.

    method: "glynn" (Eq. (S2), Gray order), "glynn_direct", "ryser" (Eq. (S1),
    plain subset order), "ryser_paired" (Eq. (S1) with the complement pairing
    of Algorithm S3) or "brute" (the definition).
    """
    g, d = to_gaussian_integers(a)
    n = len(g)
    if method == "glynn":
        r = glynn_gray_int(g)
    elif method == "glynn_direct":
        if n == 0:
            r = (1, 0)
        else:
            raw = glynn_direct_raw(g)
            div = 1 << (n - 1)
            if raw[0] % div or raw[1] % div:
                raise ArithmeticError("Glynn numerator not divisible by 2^(n-1)")
            r = (raw[0] // div, raw[1] // div)
    elif method == "ryser":
        r = ryser_subsets_int(g)
    elif method == "ryser_paired":
        r = ryser_paired_int(g)
    elif method == "brute":
        r = perm_brute_int(g)
    else:
        raise ValueError(method)
    return _scaled(r, d, n)


def to_complex(x) -> complex:
    """Round an exact (re, im) pair to the nearest complex128 (each part
    correctly rounded)."""
    return complex(float(x[0]), float(x[1]))


def rel_err(value, exact) -> float:
    """Relative error of a computed permanent, the measure of the paper's
    Supplementary error tables (the distance to the theory value over the
    theory value's modulus): |value - exact| / |exact|, with |.| the complex
    modulus.  The difference and the quotient are taken in exact rational
    arithmetic (value is converted exactly) and only the square root is
    rounded; |exact| = 0 gives |value|, the absolute error."""
    vr, vi = _as_rational_parts(value)
    er, ei = exact
    num = (vr - er) ** 2 + (vi - ei) ** 2
    den = er * er + ei * ei
    if den == 0:
        return math.sqrt(float(num))
    return math.sqrt(float(num / den))


def minor(a: np.ndarray, i: int, j: int) -> np.ndarray:
    """a with row i and column j deleted."""
    a = np.asarray(a)
    return np.delete(np.delete(a, i, axis=0), j, axis=1)


def minor_perm_exact(a, i: int, j: int, method: str = "glynn"):
    """Per(minor_ij) = d Per(A) / d a_ij (row i expansion of the definition)."""
    return perm_exact(minor(np.asarray(a), i, j), method)


def certify_int_exact(a, ryser: bool = False) -> dict:
    """Decide whether a floating-point sweep over this integer matrix is exact
    in binary64 whatever the order of its products and sums.

    Exactness holds when every intermediate is an integer of magnitude below
    2^53.  With |x|_1 = |Re x| + |Im x| (which bounds both parts and satisfies
    |xy|_1 <= |x|_1 |y|_1), three bounds suffice:
      * every partial sum met while a row sum is formed from scratch, from
        entries a_ij or 2 a_ij with any signs, in any order:
        2 max_i sum_j |a_ij|_1 < 2^53;
      * every partial product of row sums (and every row sum reached by
        steps): max over terms of prod_i max(1, |r_i|_1) < 2^53;
      * every partial sum of terms, in any order: sum over terms of
        |term|_1 < 2^53.
    The walk is Eq. (S2) in Gray order (or Eq. (S1) over all subsets when
    ``ryser``).  Returns the three bounds and whether all hold.
    """
    g, d = to_gaussian_integers(a)
    if d != 1:
        return {"certified": False, "reason": "entries are not integers"}
    n = len(g)
    if n == 0:
        return {"certified": True, "seed_partial_sums": 0, "max_partial_product": 1, "sum_abs_terms": 1}
    seed_bound = 2 * max(sum(abs(x[0]) + abs(x[1]) for x in row) for row in g)
    max_pp = 0
    sum_abs = 0
    if ryser:
        for mask in range(1 << n):
            rs = [(sum(g[i][j][0] for j in range(n) if (mask >> j) & 1),
                   sum(g[i][j][1] for j in range(n) if (mask >> j) & 1)) for i in range(n)]
            pp = 1
            for x in rs:
                pp *= max(1, abs(x[0]) + abs(x[1]))
            max_pp = max(max_pp, pp)
            p = _prod(rs)
            sum_abs += abs(p[0]) + abs(p[1])
    else:
        for mask in range(1 << (n - 1)):
            delta = delta_of_word(mask, n)
            rs = [(sum(delta[j] * g[i][j][0] for j in range(n)),
                   sum(delta[j] * g[i][j][1] for j in range(n))) for i in range(n)]
            pp = 1
            for x in rs:
                pp *= max(1, abs(x[0]) + abs(x[1]))
            max_pp = max(max_pp, pp)
            p = _prod(rs)
            sum_abs += abs(p[0]) + abs(p[1])
    lim = 1 << 53
    return {"certified": seed_bound < lim and max_pp < lim and sum_abs < lim,
            "seed_partial_sums": seed_bound, "max_partial_product": max_pp, "sum_abs_terms": sum_abs}
