"""Inputs with exactly known permanents for the GPU tests at sizes the exact
oracle cannot reach.  The closed form is pinned against the definition on the
CPU (test_two_permutations_closed_form in tests/test_oracle_pins.py)."""
import numpy as np


def cycle_count(perm) -> int:
    seen, count = set(), 0
    for i in range(len(perm)):
        if i not in seen:
            count += 1
            while i not in seen:
                seen.add(i)
                i = int(perm[i])
    return count


def two_permutations(n: int, seed: int):
    """D (P + Q) for random permutation matrices P, Q and a random diagonal D
    of units {1, i, -1, -i}, and its permanent prod(D) 2^(cycles of P^-1 Q):
    Per(P + Q) = Per(I + P^-1 Q), and each cycle of P^-1 Q is a block of
    permanent 2 (the identity and the cycle; a fixed point's entry is 2).
    Every row sum of Eq. (S1) or (S2) on it has modulus at most 2, so every
    term is an exact integer below 2^53 for n <= 52 and the sums are exact."""
    rng = np.random.default_rng(seed)
    p, q = rng.permutation(n), rng.permutation(n)
    a = np.zeros((n, n), np.complex128)
    a[np.arange(n), p] += 1
    a[np.arange(n), q] += 1
    units = np.array([1, 1j, -1, -1j])[rng.integers(0, 4, n)]
    want = complex(np.prod(units)) * 2.0 ** cycle_count(np.argsort(p)[q])
    return units[:, None] * a, want
