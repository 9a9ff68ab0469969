"""Stored oracle values (written by tests/golden/make_golden.py, which calls
only oracle/ and inputs/)."""
import os
from fractions import Fraction

import inputs as I

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(kind: str):
    """name -> (n, sha256, (re, im) Fractions)."""
    path = os.path.join(GOLDEN, f"{kind}_perms.txt")
    out = {}
    if not os.path.exists(path):
        return out
    with open(path) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            name, n, sha, e, re, im = line.split()
            den = 1 << int(e)
            out[name] = (int(n), sha, (Fraction(int(re), den), Fraction(int(im), den)))
    return out


def value_for(kind: str, name: str, a):
    """Stored exact value for input `a`, checking that `a` is the same bytes
    the value was computed from.  None if absent."""
    g = load(kind).get(name)
    if g is None:
        return None
    n, sha, v = g
    assert a.shape[0] == n and I.sha256_of(a) == sha, f"input for {name} differs from the stored one"
    return v
