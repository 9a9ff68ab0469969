"""Chain-rule boson sampler, exact arithmetic.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper's simulation exists to draw boson-sampling outputs, whose
probabilities are main-text Eq. (1), but it gives no sampling procedure.  The
reading taken here is Clifford and Clifford's exact chain-rule algorithm
("The classical complexity of boson sampling", 2018, their Algorithm B),
restated:

* A = U[:, in_modes] (rows: output modes, columns: photons), input modes
  distinct; the columns are taken in a uniformly random order perm;
* photon k = 1..n goes to output mode r_k with probability proportional to
  w_k(i) = |Per(A[(r_1, ..., r_{k-1}, i), perm[0..k-1]])|^2 over all modes i;
* the sample is the sorted tuple (r_1, ..., r_n).

For an exactly unitary U the distribution of the sorted tuple, averaged over
perm, is Eq. (1); `sampler_distribution` computes it exactly so that a test
can check this against `prob_exact`.

The random choices are inputs: `perm`, and one uniform u_k in [0, 1) per
photon, with the rule r_k = the first i whose running sum of weights exceeds
u_k times their total.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

from .exact import perm_exact


def _entry(u, i, j):
    """Exact (re, im) of U[i][j] for numpy arrays, nested lists of numbers or
    of (re, im) Fraction pairs."""
    x = u[i][j]
    if isinstance(x, tuple):
        return Fraction(x[0]), Fraction(x[1])
    c = complex(x)
    return Fraction(c.real), Fraction(c.imag)


def columns_of_inputs(u, in_modes):
    """A = U[:, in_modes] as exact (re, im) pairs, rows = output modes."""
    m = len(u)
    if len(set(in_modes)) != len(in_modes):
        raise ValueError("the chain-rule sampler takes distinct input modes")
    return [[_entry(u, i, s) for s in in_modes] for i in range(m)]


def step_weights(a, perm, rows, k):
    """w_k(i) = |Per(A[(rows..., i), perm[:k]])|^2 for every output mode i
    (rows holds r_1..r_{k-1}), exact."""
    cols = list(perm[:k])
    out = []
    for i in range(len(a)):
        sub = [[a[r][c] for c in cols] for r in list(rows) + [i]]
        re, im = perm_exact(sub)
        out.append(re * re + im * im)
    return out


def choose(weights, u) -> int:
    """The first index whose running sum exceeds u times the total."""
    total = sum(weights)
    if total <= 0:
        raise ValueError("all weights are zero")
    target = Fraction(u) * total
    run = Fraction(0)
    last = None
    for i, w in enumerate(weights):
        run += w
        if w > 0:
            last = i
        if run > target:
            return i
    return last


def sample_exact(u, in_modes, perm, uniforms, trace=None):
    """One sample: sorted output modes, from the given column order and
    uniforms.  trace (a list), if given, receives (weights, choice) per step."""
    a = columns_of_inputs(u, in_modes)
    n = len(in_modes)
    if sorted(perm) != list(range(n)) or len(uniforms) != n:
        raise ValueError("perm must order 0..n-1 and there is one uniform per photon")
    rows = []
    for k in range(1, n + 1):
        w = step_weights(a, perm, rows, k)
        r = choose(w, uniforms[k - 1])
        if trace is not None:
            trace.append((w, r))
        rows.append(r)
    return tuple(sorted(rows))


def sampler_distribution(u, in_modes):
    """Exact probability of every sorted output tuple under the sampler,
    averaged over all n! column orders (each order's chain of conditional
    probabilities summed over every ordered placement)."""
    a = columns_of_inputs(u, in_modes)
    n = len(in_modes)
    dist = {}
    for perm in itertools.permutations(range(n)):
        # depth-first over ordered placements with their probabilities
        stack = [((), Fraction(1))]
        while stack:
            rows, p = stack.pop()
            k = len(rows) + 1
            if k > n:
                key = tuple(sorted(rows))
                dist[key] = dist.get(key, Fraction(0)) + p
                continue
            w = step_weights(a, perm, rows, k)
            tot = sum(w)
            for i, wi in enumerate(w):
                if wi:
                    stack.append((rows + (i,), p * wi / tot))
    f = math.factorial(n)
    return {key: v / f for key, v in dist.items()}
