"""Pins of the oracle's chain-rule sampler: its exact output distribution is
Eq. (1) on an exactly unitary matrix, its normalisation follows the Laplace
expansion, and planted mistakes break that."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from oracle import sampler as OS


def cmul(x, y):
    return (x[0] * y[0] - x[1] * y[1], x[0] * y[1] + x[1] * y[0])


def cdiv(x, y):
    d = y[0] * y[0] + y[1] * y[1]
    return ((x[0] * y[0] + x[1] * y[1]) / d, (x[1] * y[0] - x[0] * y[1]) / d)


def csub(x, y):
    return (x[0] - y[0], x[1] - y[1])


def cayley_unitary(m, seed):
    """U = (I - S)(I + S)^-1 for a rational skew-Hermitian S: exactly unitary,
    with rational entries (input data for the pins below)."""
    rng = np.random.default_rng(seed)
    Z = [[(Fraction(int(rng.integers(-3, 4)), 4), Fraction(int(rng.integers(-3, 4)), 4)) for _ in range(m)]
         for _ in range(m)]
    S = [[csub(Z[i][j], (Z[j][i][0], -Z[j][i][1])) for j in range(m)] for i in range(m)]
    one, zero = (Fraction(1), Fraction(0)), (Fraction(0), Fraction(0))
    P = [[(one if i == j else zero) for j in range(m)] for i in range(m)]
    Mi = [[csub(P[i][j], S[i][j]) for j in range(m)] for i in range(m)]   # I - S
    Mp = [[(P[i][j][0] + S[i][j][0], P[i][j][1] + S[i][j][1]) for j in range(m)] for i in range(m)]  # I + S
    # inverse of I + S by Gauss-Jordan
    aug = [Mp[i] + P[i] for i in range(m)]
    for c in range(m):
        piv = next(r for r in range(c, m) if aug[r][c] != zero)
        aug[c], aug[piv] = aug[piv], aug[c]
        inv = cdiv(one, aug[c][c])
        aug[c] = [cmul(v, inv) for v in aug[c]]
        for r in range(m):
            if r != c and aug[r][c] != zero:
                f = aug[r][c]
                aug[r] = [csub(v, cmul(f, w)) for v, w in zip(aug[r], aug[c])]
    Inv = [row[m:] for row in aug]
    U = [[None] * m for _ in range(m)]
    for i in range(m):
        for j in range(m):
            acc = zero
            for k in range(m):
                t = cmul(Mi[i][k], Inv[k][j])
                acc = (acc[0] + t[0], acc[1] + t[1])
            U[i][j] = acc
    return U


def is_unitary(U):
    m = len(U)
    for i in range(m):
        for j in range(m):
            acc = (Fraction(0), Fraction(0))
            for k in range(m):
                t = cmul((U[k][i][0], -U[k][i][1]), U[k][j])
                acc = (acc[0] + t[0], acc[1] + t[1])
            if acc != ((Fraction(1) if i == j else Fraction(0)), Fraction(0)):
                return False
    return True


def multisets(m, n):
    return list(itertools.combinations_with_replacement(range(m), n))


@pytest.mark.parametrize("m,n,ins,seed", [(4, 2, [0, 1], 1), (5, 3, [0, 2, 4], 2), (4, 3, [1, 2, 3], 3)])
def test_sampler_distribution_is_eq1_on_an_exact_unitary(m, n, ins, seed):
    U = cayley_unitary(m, seed)
    assert is_unitary(U)
    dist = OS.sampler_distribution(U, ins)
    eq1 = {T: O.prob_exact(U, ins, T) for T in multisets(m, n)}
    assert sum(eq1.values()) == 1
    assert set(dist) <= set(eq1)
    for T, p in eq1.items():
        assert dist.get(T, Fraction(0)) == p, T


def test_choose_rule():
    w = [Fraction(1), Fraction(0), Fraction(2)]
    assert OS.choose(w, 0.0) == 0
    assert OS.choose(w, 0.3) == 0
    assert OS.choose(w, 1 / 3 + 1e-12) == 2  # the zero weight is never taken
    assert OS.choose(w, 0.999999) == 2
    assert OS.choose([Fraction(0), Fraction(5)], 0.0) == 1
    with pytest.raises(ValueError):
        OS.choose([Fraction(0)] * 3, 0.5)


def test_step_weights_closed_forms():
    U = cayley_unitary(5, 7)
    ins = [0, 1, 3]
    A = OS.columns_of_inputs(U, ins)
    perm = (2, 0, 1)
    # first photon: |a_i,c|^2 of the first column taken
    w1 = OS.step_weights(A, perm, [], 1)
    assert w1 == [A[i][2][0] ** 2 + A[i][2][1] ** 2 for i in range(5)]
    assert sum(w1) == 1
    # second photon: on a unitary the total is |a_r,c1|^2 + |a_r,c2|^2 (the
    # squared minors of the 1 x 2 matrix of the first row)
    for r in range(5):
        w2 = OS.step_weights(A, perm, [r], 2)
        assert sum(w2) == sum(A[r][c][0] ** 2 + A[r][c][1] ** 2 for c in perm[:2])


def test_sample_exact_decisions_follow_the_weights():
    U = cayley_unitary(5, 11)
    ins = [0, 1, 2]
    trace = []
    got = OS.sample_exact(U, ins, (1, 2, 0), [0.1, 0.7, 0.4], trace)
    assert len(trace) == 3 and got == tuple(sorted(r for _, r in trace))
    for (w, r), u in zip(trace, [0.1, 0.7, 0.4]):
        t = Fraction(u) * sum(w)
        assert sum(w[:r]) <= t < sum(w[: r + 1])
    with pytest.raises(ValueError):
        OS.sample_exact(U, [0, 0, 1], (0, 1, 2), [0.1, 0.2, 0.3])


def _distribution_breaks(monkeypatch, mutant):
    U = cayley_unitary(4, 1)
    monkeypatch.setattr(OS, "step_weights", mutant)
    dist = OS.sampler_distribution(U, [0, 1])
    return any(dist.get(T, Fraction(0)) != O.prob_exact(U, [0, 1], T) for T in multisets(4, 2))


def test_mutation_fixed_column_order_is_caught(monkeypatch):
    orig = OS.step_weights
    assert _distribution_breaks(monkeypatch, lambda a, perm, rows, k: orig(a, tuple(range(len(perm))), rows, k))


def test_mutation_weights_without_the_candidate_row_are_caught(monkeypatch):
    orig = OS.step_weights

    def mutant(a, perm, rows, k):
        w = orig(a, perm, rows, k)
        return [x if k == 1 else orig(a, perm, [], 1)[i] for i, x in enumerate(w)]

    assert _distribution_breaks(monkeypatch, mutant)
