"""Pins of the exact oracle against things other than itself.

Each test ties the oracle to the definition of the permanent, to a closed
form, to an independent formula or library, or to a value the paper prints.
The mutation tests at the end plant plausible mistakes in a copy of the
oracle (on the CPU) and check that these pins notice them.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import inputs as I
import oracle as O
from oracle import exact as OX
from tests import _closed_forms as CF

GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def gauss_int_matrix(n, seed, lo=-3, hi=3):
    rng = np.random.default_rng(seed)
    return (rng.integers(lo, hi + 1, (n, n)) + 1j * rng.integers(lo, hi + 1, (n, n))).astype(np.complex128)


def fr(c):
    return (Fraction(c.real), Fraction(c.imag))


def cpow(z, k):
    re, im = Fraction(1), Fraction(0)
    for _ in range(k):
        re, im = re * z[0] - im * z[1], re * z[1] + im * z[0]
    return re, im


# ------------------------------------------------------- definition vs formulas

@pytest.mark.parametrize("n", range(0, 8))
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_four_routes_agree_on_gaussian_integers(n, seed):
    a = gauss_int_matrix(n, 100 * n + seed)
    ref = O.perm_exact(a, "brute")
    assert O.perm_exact(a, "glynn") == ref
    assert O.perm_exact(a, "ryser") == ref
    assert O.perm_exact(a, "ryser_paired") == ref
    if n > 0:
        assert O.perm_exact(a, "glynn_direct") == ref


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_definition_on_binary64_unitary_entries(n):
    a = I.submatrix(I.haar(50, 7), range(n), range(3, 3 + n))
    assert O.perm_exact(a, "glynn") == O.perm_exact(a, "brute")


def test_small_cases_and_empty_matrix():
    assert O.perm_exact(np.zeros((0, 0), np.complex128)) == (1, 0)
    assert O.perm_exact(np.array([[2.5 - 1j]])) == (Fraction(5, 2), Fraction(-1))
    a = np.array([[1, 2], [3, 4]], dtype=np.complex128)
    assert O.perm_exact(a) == (10, 0)  # 1*4 + 2*3


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", range(1, 13))
def test_all_ones_is_factorial(n):
    assert O.perm_exact(np.ones((n, n))) == (math.factorial(n), 0)


@pytest.mark.parametrize("r", [0.1, 0.2, 10.0, 1 + 1j, 10 + 10j, -0.75 + 0.3j])
@pytest.mark.parametrize("n", [1, 4, 9])
def test_all_r_is_r_pow_n_times_factorial(r, n):
    re, im = cpow(fr(complex(r)), n)
    f = math.factorial(n)
    assert O.perm_exact(I.all_r(n, r)) == (re * f, im * f)


@pytest.mark.parametrize("n", [1, 3, 8, 11])
def test_identity_and_permutation_matrices(n):
    assert O.perm_exact(np.eye(n)) == (1, 0)
    p = np.random.default_rng(n).permutation(n)
    assert O.perm_exact(np.eye(n)[p]) == (1, 0)


@pytest.mark.parametrize("n", [2, 6, 10])
def test_diagonal_is_product_of_diagonal(n):
    rng = np.random.default_rng(n)
    d = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    a = np.diag(d)
    re, im = Fraction(1), Fraction(0)
    for x in d:
        xr, xi = fr(complex(x))
        re, im = re * xr - im * xi, re * xi + im * xr
    assert O.perm_exact(a) == (re, im)


def test_rank_one_closed_form():
    # Per(u v^T) = n! prod u_i prod v_j (every permutation gives the same product)
    n = 6
    u = np.array([1, -2, 3, 1, 2, -1], dtype=np.complex128) + 1j * np.array([0, 1, 0, -1, 2, 0])
    v = np.array([2, 1, -1, 3, 1, 1], dtype=np.complex128)
    a = np.outer(u, v)
    pu = np.prod(u)
    pv = np.prod(v)
    want = complex(pu * pv) * math.factorial(n)
    assert O.perm_exact(a) == fr(want)


def test_block_diagonal_is_product_of_blocks():
    a1 = gauss_int_matrix(4, 5)
    a2 = gauss_int_matrix(3, 6)
    a = np.zeros((7, 7), np.complex128)
    a[:4, :4] = a1
    a[4:, 4:] = a2
    rng = np.random.default_rng(3)
    pr, pc = rng.permutation(7), rng.permutation(7)
    x = O.perm_exact(a1)
    y = O.perm_exact(a2)
    want = (x[0] * y[0] - x[1] * y[1], x[0] * y[1] + x[1] * y[0])
    assert O.perm_exact(a[pr][:, pc]) == want


# ------------------------------------------------------------------ invariants

@pytest.mark.parametrize("seed", range(4))
def test_row_column_permutation_and_transpose_invariance(seed):
    a = gauss_int_matrix(6, 900 + seed)
    rng = np.random.default_rng(seed)
    ref = O.perm_exact(a)
    assert O.perm_exact(a[rng.permutation(6)]) == ref
    assert O.perm_exact(a[:, rng.permutation(6)]) == ref
    assert O.perm_exact(a.T.copy()) == ref


@pytest.mark.parametrize("seed", range(3))
def test_multilinear_in_one_row(seed):
    rng = np.random.default_rng(seed)
    a = gauss_int_matrix(6, 700 + seed)
    i = int(rng.integers(6))
    x = rng.integers(-4, 5, 6) + 1j * rng.integers(-4, 5, 6)
    y = rng.integers(-4, 5, 6) + 1j * rng.integers(-4, 5, 6)
    ax, ay, axy = a.copy(), a.copy(), a.copy()
    ax[i], ay[i], axy[i] = x, y, x + y
    px, py = O.perm_exact(ax), O.perm_exact(ay)
    assert O.perm_exact(axy) == (px[0] + py[0], px[1] + py[1])


@pytest.mark.parametrize("seed", range(2))
def test_laplace_row_expansion_with_minors(seed):
    a = gauss_int_matrix(6, 500 + seed)
    p = O.perm_exact(a)
    for i in range(6):
        re = im = Fraction(0)
        for j in range(6):
            m = O.minor_perm_exact(a, i, j)
            ar, ai = fr(complex(a[i, j]))
            re += ar * m[0] - ai * m[1]
            im += ar * m[1] + ai * m[0]
        assert (re, im) == p


def test_mpmath_cross_check():
    mpmath = pytest.importorskip("mpmath")
    a = I.submatrix(I.haar(64, 3), range(5, 15), range(10))
    n = 10
    with mpmath.workdps(60):
        m = [[mpmath.mpc(complex(a[i, j])) for j in range(n)] for i in range(n)]
        # Eq. (S1) in mpmath arithmetic: an independent (inexact, 60-digit) route
        tot = mpmath.mpc(0)
        for mask in range(1, 1 << n):
            cols = [j for j in range(n) if (mask >> j) & 1]
            p = mpmath.mpc(1)
            for i in range(n):
                p *= mpmath.fsum(m[i][j] for j in cols)
            tot += (-1) ** len(cols) * p
        tot *= (-1) ** n
        ex = O.perm_exact(a)
        err = abs(tot - mpmath.mpc(mpmath.mpf(ex[0].numerator) / ex[0].denominator,
                                   mpmath.mpf(ex[1].numerator) / ex[1].denominator))
        assert err <= mpmath.mpf(10) ** -45 * abs(tot)


def test_gray_range_split_is_exact():
    g, _ = O.to_gaussian_integers(gauss_int_matrix(9, 11))
    full = O.glynn_gray_raw(g)
    total = 1 << 8
    for pieces in (1, 3, 7, 256):
        parts = [O.glynn_gray_raw(g, a, b) for a, b in O.split_range(total, pieces)]
        assert (sum(p[0] for p in parts), sum(p[1] for p in parts)) == full
    assert O.glynn_raw_parallel(g, 0, total, workers=2) == full


def _term_by_convention(a, k, algo):
    """The summand of Gray index k written straight from the convention the
    library documents for its partial sums (word w = k ^ (k >> 1); BB/FG:
    delta_0 = +1, delta_{b+1} = -1 iff bit b of w; Ryser: column b in S iff
    bit b of w), in exact integer arithmetic on an integer matrix."""
    n = a.shape[0]
    w = k ^ (k >> 1)
    if algo == "glynn":
        coef = [1] + [-1 if (w >> b) & 1 else 1 for b in range(n - 1)]
        sign = int(np.prod(coef))
    else:
        coef = [1 if (w >> b) & 1 else 0 for b in range(n)]
        sign = (-1) ** sum(coef)
    prod = 1
    for i in range(n):
        prod *= sum(coef[j] * complex(a[i, j]) for j in range(n))
    return complex(sign * prod)


@pytest.mark.parametrize("algo", ["glynn", "ryser"])
def test_single_index_ranges_follow_the_documented_word_convention(algo):
    # small integer entries: every product is exact in binary64
    a = gauss_int_matrix(5, 77, -2, 2)
    g, d = O.to_gaussian_integers(a)
    assert d == 1
    raw = O.glynn_gray_raw if algo == "glynn" else O.ryser_gray_raw
    for k in range(1 << (4 if algo == "glynn" else 5)):
        got = raw(g, k, k + 1)
        assert complex(got[0], got[1]) == _term_by_convention(a, k, algo), k


@pytest.mark.parametrize("n", range(1, 7))
def test_ryser_gray_range_is_eq_s1(n):
    for seed in (0, 1):
        a = gauss_int_matrix(n, 900 + seed)
        g, _ = O.to_gaussian_integers(a)
        re, im = O.ryser_gray_raw(g)
        sg = (-1) ** n
        assert (sg * re, sg * im) == O.perm_brute_int(g)
        assert (sg * re, sg * im) == O.ryser_subsets_int(g)


def test_ryser_gray_range_split_and_closed_form():
    g, _ = O.to_gaussian_integers(gauss_int_matrix(8, 12))
    full = O.ryser_gray_raw(g)
    for pieces in (1, 3, 16, 256):
        parts = [O.ryser_gray_raw(g, a, b) for a, b in O.split_range(1 << 8, pieces)]
        assert (sum(p[0] for p in parts), sum(p[1] for p in parts)) == full
    assert O.ryser_gray_raw(g, 0, 1) == (0, 0)  # the empty set
    # all ones: sum_S (-1)^|S| |S|^n = (-1)^n n!
    for n in range(1, 8):
        ones = [[(1, 0)] * n for _ in range(n)]
        assert O.ryser_gray_raw(ones) == ((-1) ** n * math.factorial(n), 0)


@pytest.mark.parametrize("n", range(1, 8))
def test_ryser_paired_algorithm_s3(n):
    # Algorithm S3's pairing: S over the subsets of the first n - 1 columns,
    # S_C its complement among all n, covers every subset exactly once
    seen = set()
    for it in range(1 << (n - 1)):
        seen.update((it, ((1 << n) - 1) ^ it))
    assert len(seen) == 1 << n
    ones = [[(1, 0)] * n for _ in range(n)]
    assert O.ryser_paired_int(ones) == (math.factorial(n), 0)
    diag = [[(j + 2, 1 - j) if i == j else (0, 0) for j in range(n)] for i in range(n)]
    want = (1, 0)
    for j in range(n):
        want = (want[0] * (j + 2) - want[1] * (1 - j), want[0] * (1 - j) + want[1] * (j + 2))
    assert O.ryser_paired_int(diag) == want
    g, _ = O.to_gaussian_integers(gauss_int_matrix(n, 700 + n))
    assert O.ryser_paired_int(g) == O.perm_brute_int(g)


@pytest.mark.parametrize("n", range(1, 8))
def test_two_permutations_closed_form(n):
    # Per(D (P + Q)) = prod(D) 2^(cycles of P^-1 Q) for permutation matrices
    # P, Q and a diagonal D of units (the GPU tests use it at n up to 40):
    # Per(P + Q) = Per(I + P^-1 Q), and each cycle of P^-1 Q is a block whose
    # permanent is 2 (the identity and the cycle; a fixed point's entry is 2)
    for seed in range(4):
        a, want = CF.two_permutations(n, 100 * n + seed)
        assert O.to_complex(O.perm_exact(a, "brute")) == want


# ------------------------------------------------------ values the paper prints

def _printed_match(value: float, printed: str) -> bool:
    """value rounds to the printed string at the printed precision."""
    if "E" in printed or "e" in printed:
        mant = printed.upper().split("E")[0]
        digits = len(mant.replace("-", "").replace(".", "")) - 1
        return f"{value:.{digits}E}" == printed.upper() or (float(printed) == 0 and value == 0)
    decimals = len(printed.split(".")[1]) if "." in printed else 0
    return f"{value:.{decimals}f}" == printed


def _theory_rows():
    rows = []
    with open(f"{GOLDEN}/paper_allr_theory.txt") as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            kind, n, r, tre, tim = line.split()
            rows.append((kind, int(n), complex(r.replace("i", "j")), tre, tim))
    return rows


def test_printed_theory_values_are_r_pow_n_factorial():
    """Every Per_Theory value of the two BB/FG error tables equals r^n n! at the
    printed precision (r read as the decimal the table prints)."""
    rows = _theory_rows()
    assert len(rows) == 120
    for kind, n, r, tre, tim in rows:
        rr = (Fraction(str(r.real)), Fraction(str(r.imag)))
        re, im = cpow(rr, n)
        f = math.factorial(n)
        assert _printed_match(float(re * f), tre), (kind, n, r, tre)
        assert _printed_match(float(im * f), tim) or (abs(float(im * f)) < 1e-30 and float(tim) == 0), (kind, n, r, tim)


@pytest.mark.parametrize("n,r", [(17, 1), (17, 0.1), (17, 10), (17, 0.2), (18, 0.2), (17, 1 + 1j), (18, 1 + 1j),
                                 (17, 10 + 10j)])
def test_oracle_reproduces_printed_theory_values(n, r):
    """The oracle's exact permanent of the all-r matrix (r rounded to binary64)
    rounds to the value the paper prints."""
    rows = {(kind, m, rr): (tre, tim) for kind, m, rr, tre, tim in _theory_rows()}
    kind = "bbfg_complex" if complex(r).imag else "bbfg_real"
    tre, tim = rows[(kind, n, complex(r))]
    v = O.perm_exact(I.all_r(n, r))
    assert _printed_match(float(v[0]), tre)
    assert _printed_match(float(v[1]), tim) or (float(tim) == 0 and v[1] == 0)


def test_worked_example_diag_1_plus_i():
    """The paper's 45 x 45 diag(1+i) run: (1+i)^45.  The fixture's value is the
    exact power; the oracle's Glynn walk agrees on diag(1+i) at every n it can
    afford."""
    with open(f"{GOLDEN}/paper_worked_examples.txt") as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    name, n, dr, di, pr, pi = rows[0]
    assert name == "diag_1pi" and int(n) == 45
    assert cpow((Fraction(int(dr)), Fraction(int(di))), 45) == (int(pr), int(pi))
    for m in (1, 2, 7, 13):
        assert O.perm_exact(I.diag_matrix(m, 1 + 1j)) == cpow((Fraction(1), Fraction(1)), m)


# ----------------------------------------------------------------- boson layer

def test_completeness_of_output_distribution():
    """Eq. (1): summed over every output pattern (multisets of n modes out of m),
    the probabilities add up to 1 for a unitary U.  Pins the t_j! normalisation
    and the repeated-row gather."""
    m, n = 6, 4
    u = I.haar(m, 5)
    total = Fraction(0)
    count = 0
    for t in itertools.combinations_with_replacement(range(m), n):
        total += O.prob_exact(u, range(n), t)
        count += 1
    assert count == math.comb(m + n - 1, n)
    assert abs(float(total) - 1.0) < 1e-13


@pytest.mark.parametrize("seed", range(4))
def test_multiplicity_formula_matches_gather_plus_glynn(seed):
    rng = np.random.default_rng(seed)
    m, n = 40, 7
    u = I.haar(m, 9)
    modes = rng.choice(m, 4, replace=False)
    pat = np.sort(np.concatenate([np.repeat(modes[:1], 3), np.repeat(modes[1:2], 2), modes[2:]]))[:n]
    pat = np.sort(np.concatenate([pat, rng.choice(m, n - len(pat))]))
    assert len(pat) == n
    assert O.prob_multiplicity(u, range(n), pat) == O.prob_exact(u, range(n), pat)


def test_probability_without_collisions_is_abs_perm_squared():
    u = I.haar(20, 4)
    out = [1, 4, 7, 9, 15]
    p = O.perm_exact(O.gather_u_st(u, range(5), out))
    assert O.prob_exact(u, range(5), out) == p[0] ** 2 + p[1] ** 2


# ----------------------------------------------------- integer exactness check

def test_int12_matrix_is_certified():
    c = O.certify_int_exact(I.int12_matrix())
    assert c["certified"] and c["max_partial_product"] < 2 ** 53 and c["sum_abs_terms"] < 2 ** 53
    assert c["seed_partial_sums"] < 2 ** 53
    assert not O.certify_int_exact(I.all_r(12, 100))["certified"]


def _cancelling_rows(a, b):
    """Rows (a, 0, 0, 0), (b, 0, 0, 0), (1, 1, 0, 0), (1, -1, 0, 0).  For every
    delta of Eq. (S2) the last two row sums are 1 + delta_1 and 1 - delta_1,
    one of them 0: every term is 0 (so is the sum of |term|, and Per), while
    the partial product a * b * 2 is reached.  Seeds stay small."""
    m = np.zeros((4, 4), np.complex128)
    m[0, 0], m[1, 0] = a, b
    m[2, :2] = (1, 1)
    m[3, :2] = (1, -1)
    return m


def test_certificate_partial_product_boundary():
    ok = O.certify_int_exact(_cancelling_rows(2 ** 26, 2 ** 26 - 1))
    assert ok["certified"] and ok["max_partial_product"] == 2 ** 53 - 2 ** 27
    assert ok["sum_abs_terms"] == 0 and ok["seed_partial_sums"] == 2 ** 27
    bad = O.certify_int_exact(_cancelling_rows(2 ** 26, 2 ** 26))
    assert not bad["certified"] and bad["max_partial_product"] == 2 ** 53
    assert bad["sum_abs_terms"] == 0 and bad["seed_partial_sums"] == 2 ** 27
    assert O.perm_exact(_cancelling_rows(2 ** 26, 2 ** 26)) == (0, 0)


def test_certificate_term_sum_boundary():
    # diag(a, b): both BB/FG terms equal ab (sign and row sum flip together),
    # so the sum of |term|_1 is 2|ab|_1 while every partial product is
    # |a|_1 |b|_1 and the seeds stay small
    def d(a, b):
        return np.diag([a, b]).astype(np.complex128)
    ok = O.certify_int_exact(d(2 ** 26, 2 ** 26 - 1))
    assert ok["certified"] and ok["sum_abs_terms"] == 2 ** 53 - 2 ** 27 and ok["max_partial_product"] < 2 ** 52
    bad = O.certify_int_exact(d(2 ** 26, 2 ** 26))
    assert not bad["certified"] and bad["sum_abs_terms"] == 2 ** 53 and bad["max_partial_product"] == 2 ** 52
    assert bad["seed_partial_sums"] == 2 ** 27
    # the imaginary part counts in |.|_1 like the real one: |2^25 (1 + i)|_1 = 2^26
    bad_i = O.certify_int_exact(d(2 ** 26, 2 ** 25 * (1 + 1j)))
    assert not bad_i["certified"] and bad_i["sum_abs_terms"] == 2 ** 53 and bad_i["max_partial_product"] == 2 ** 52


def test_certificate_seed_boundary():
    # one row [x, -x]: its BB/FG row sums are 0 or 2x and the terms cancel
    # against the zero row below, but forming 2x from scratch passes through
    # partial sums up to 2 sum_j |a_ij|_1 = 4x in the worst order
    def m(x):
        return np.array([[x, -x], [0, 0]], dtype=np.complex128)
    assert O.certify_int_exact(m(2 ** 51 - 1))["seed_partial_sums"] == 2 ** 53 - 4
    assert O.certify_int_exact(m(2 ** 51 - 1))["certified"]
    assert not O.certify_int_exact(m(2 ** 51))["certified"]


# --------------------------------------------------- the relative-error checker

def _rel_err_cases():
    """(value, exact, expected) worked by hand.  RelErr is the measure of the
    paper's Supplementary error tables: |Per - Per_theory| / |Per_theory|,
    with the complex modulus."""
    third = Fraction(1, 3)
    return [
        # real part off by 2^-33 of 1: relative error 2^-33 exactly
        (1.0 + 2.0 ** -33, (Fraction(1), Fraction(0)), 2.0 ** -33),
        # an offset of 3 + 4i on the real value 10: |3 + 4i| / 10 = 0.5
        (13.0 + 4.0j, (Fraction(10), Fraction(0)), 0.5),
        # a purely imaginary offset on a complex exact value 3 + 4i: 2^-20 / 5
        (3.0 + (4.0 + 2.0 ** -20) * 1j, (Fraction(3), Fraction(4)), 2.0 ** -20 / 5),
        # a unit offset along the exact value's own direction: 1 / |3 + 4i|
        (3.6 + 4.8j, (Fraction(3), Fraction(4)), None),
        # exact value 0: the absolute error |3 + 4i| = 5
        (3.0 + 4.0j, (Fraction(0), Fraction(0)), 5.0),
        # an exact rational: the binary64 nearest 1/3 is 1/3 - 1/(3 2^54),
        # so the relative error is 2^-54 exactly
        (1.0 / 3.0, (third, Fraction(0)), 2.0 ** -54),
        # no error at all, exact value given as Fractions of a binary64 input
        (0.1 - 0.7j, (Fraction(0.1), Fraction(-0.7)), 0.0),
    ]


def _rel_err_pins_hold(fn) -> bool:
    for value, exact, want in _rel_err_cases():
        got = fn(value, exact)
        if want is None:
            # 3.6 + 4.8i is not exactly 1.2 (3 + 4i) in binary64; the exact
            # value of the offset is computed from the stored doubles
            d = (Fraction(3.6) - 3) ** 2 + (Fraction(4.8) - 4) ** 2
            want = math.sqrt(float(d / 25))
            if abs(want - 0.2) > 1e-15:
                return False
        if want == 0.0:
            if got != 0.0:
                return False
        elif not abs(got - want) <= 2e-16 * want:
            return False
    return True


def test_rel_err_on_hand_computed_cases():
    assert _rel_err_pins_hold(O.rel_err)
    for value, exact, want in _rel_err_cases():
        if want is not None and want != 0.0 and math.log2(want).is_integer():
            assert O.rel_err(value, exact) == want  # powers of two come out exactly


# ------------------------------------------------------------- mutation tests

def _pins_fail(monkeypatch, attr, mutant):
    """Apply a mutation to the oracle module and report whether the cheap pins
    above catch it."""
    monkeypatch.setattr(OX, attr, mutant)
    failures = 0
    for n in (3, 5, 6):
        a = gauss_int_matrix(n, 4242 + n)
        brute = O.perm_exact(a, "brute")
        try:
            if O.perm_exact(a, "glynn") != brute:
                failures += 1
            # the same walk cut into pieces, each seeded at its start
            g, _ = O.to_gaussian_integers(a)
            parts = [OX.glynn_gray_raw(g, k0, k1) for k0, k1 in O.split_range(1 << (n - 1), 3)]
            raw = (sum(p[0] for p in parts), sum(p[1] for p in parts))
            if raw != (brute[0] * (1 << (n - 1)), brute[1] * (1 << (n - 1))):
                failures += 1
        except ArithmeticError:
            failures += 1
    return failures > 0


def test_mutation_not_a_gray_code_is_caught(monkeypatch):
    # plain binary counting instead of the reflected Gray code
    assert _pins_fail(monkeypatch, "gray", lambda k: k)


def test_mutation_off_by_one_column_is_caught(monkeypatch):
    assert _pins_fail(monkeypatch, "flipped_column", lambda w0, w1: max(0, (w0 ^ w1).bit_length() - 1))


def test_mutation_wrong_fixed_delta_is_caught(monkeypatch):
    # off by one: bit b drives column b, so delta_0 is no longer fixed to +1
    assert _pins_fail(monkeypatch, "delta_of_word", lambda w, n: [(-1 if (w >> b) & 1 else 1) for b in range(n)])


def test_mutation_transposed_operand_in_complex_product_is_caught(monkeypatch):
    # (a+ib)(c+id) with the imaginary part's operands swapped wrongly
    assert _pins_fail(monkeypatch, "_cmul", lambda x, y: (x[0] * y[0] - x[1] * y[1], x[0] * y[0] + x[1] * y[1]))


# mutants of the relative-error checker and of the integer certificate: each
# plausible slip must break a pin above

def _mutant_rel_err_no_sqrt(value, exact):
    vr, vi = OX._as_rational_parts(value)
    num = (vr - exact[0]) ** 2 + (vi - exact[1]) ** 2
    den = exact[0] ** 2 + exact[1] ** 2
    return float(num / den) if den else float(num)


def _mutant_rel_err_over_value(value, exact):
    vr, vi = OX._as_rational_parts(value)
    num = (vr - exact[0]) ** 2 + (vi - exact[1]) ** 2
    den = vr * vr + vi * vi
    return math.sqrt(float(num / den)) if den else math.sqrt(float(num))


def _mutant_rel_err_real_only(value, exact):
    vr, _ = OX._as_rational_parts(value)
    den = exact[0] ** 2 + exact[1] ** 2
    return math.sqrt(float((vr - exact[0]) ** 2 / den)) if den else abs(float(vr - exact[0]))


def _mutant_rel_err_in_binary64(value, exact):
    ex = complex(float(exact[0]), float(exact[1]))
    return abs(complex(value) - ex) / abs(ex) if ex else abs(complex(value))


@pytest.mark.parametrize("mutant", [_mutant_rel_err_no_sqrt, _mutant_rel_err_over_value, _mutant_rel_err_real_only,
                                    _mutant_rel_err_in_binary64])
def test_mutation_rel_err_is_caught(mutant):
    assert not _rel_err_pins_hold(mutant)


def _certificate_pins_hold(monkeypatch, mutant_source):
    """Run the boundary pins of the integer certificate against a mutated copy
    of it (a textual edit of its source, executed in the oracle's namespace)."""
    import inspect

    src = inspect.getsource(OX.certify_int_exact)
    mutated = mutant_source(src)
    assert mutated != src, "mutation did not apply"
    ns = dict(vars(OX))
    exec(compile(mutated, "<mutant>", "exec"), ns)
    monkeypatch.setattr(O, "certify_int_exact", ns["certify_int_exact"])
    try:
        test_certificate_partial_product_boundary()
        test_certificate_term_sum_boundary()
        test_certificate_seed_boundary()
    except AssertionError:
        return False
    return True


@pytest.mark.parametrize("edit", [
    lambda s: s.replace("seed_bound < lim and ", ""),                    # seed bound dropped
    lambda s: s.replace("max_pp < lim and ", ""),                        # product bound dropped
    lambda s: s.replace(" and sum_abs < lim", ""),                       # term-sum bound dropped
    lambda s: s.replace("max_pp < lim", "max_pp <= lim"),                # off by one at 2^53
    lambda s: s.replace("abs(x[0]) + abs(x[1])", "abs(x[0])").replace("abs(p[0]) + abs(p[1])", "abs(p[0])"),
    # (imaginary parts ignored)
])
def test_mutation_certificate_is_caught(monkeypatch, edit):
    assert not _certificate_pins_hold(monkeypatch, edit)


def test_certificate_pins_hold_unmutated(monkeypatch):
    assert _certificate_pins_hold(monkeypatch, lambda s: s + "\n")
