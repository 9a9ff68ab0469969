"""Parity of Ryser's formula in the load-balanced order of Algorithm S3
(ph_perm_ryser_paired) with the exact CPU oracle.

Bar: bit-exact on small Gaussian-integer matrices (every row sum, product and
partial sum is an integer the double-double sum holds exactly); on Haar-unitary
submatrices the bound of the plain Ryser sweep (1e-10 up to n = 20, 1e-6
above, where Ryser's terms dwarf the result; stored exact values from
tests/golden/make_golden.py).  Sizes span one chunk, several chunks, partial
workgroups and the register-heavy orders above 18.
"""
import numpy as np
import pytest

import inputs as I
import oracle as O
from tests import _closed_forms as CF
from tests import _golden as G

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ph():
    import paper_1606_05836_amd as ph

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return ph


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def small_gauss(n, seed):
    # entries in {-1, 0, 1} + i{-1, 0, 1}: at n <= 12 every term is an exact
    # integer below 2^53 and the double-double sum of them is exact
    rng = np.random.default_rng(seed)
    return (rng.integers(-1, 2, (n, n)) + 1j * rng.integers(-1, 2, (n, n))).astype(np.complex128)


def ryser_tol(n):
    return 1e-10 if n <= 20 else 1e-6


@pytest.mark.parametrize("n", list(range(0, 13)))
def test_integer_matrices_bit_exact(ph, n):
    a = small_gauss(n, 900 + n)
    want = O.to_complex(O.perm_exact(a, "ryser_paired"))
    assert want == O.to_complex(O.perm_exact(a, "glynn"))
    assert complex(ph.perm_ryser_paired(cuda(a)).cpu()) == want
    if n <= 8:  # partial sums stay below 2^53: the plain sum is exact too
        assert complex(ph.perm_ryser_paired(cuda(a), accum="plain").cpu()) == want


@pytest.mark.parametrize("c", [1, 3, 5])
def test_chunk_lengths_bit_exact(ph, c):
    a = small_gauss(11, 77)
    want = O.to_complex(O.perm_exact(a))
    assert complex(ph.perm_ryser_paired(cuda(a), chunk_log2=c).cpu()) == want


def test_haar400_block20_in_place(ph):
    u = cuda(I.haar(400, 11))
    a = I.haar400_block20()
    ex = G.value_for("haar", "haar400_block20", a)
    got = complex(ph.perm_ryser_paired(u[:20, :20]).cpu())
    assert O.rel_err(got, ex) <= ryser_tol(20)
    # the same bits from a contiguous copy, and from a second call
    assert complex(ph.perm_ryser_paired(u[:20, :20].contiguous()).cpu()) == got
    assert complex(ph.perm_ryser_paired(u[:20, :20]).cpu()) == got


@pytest.mark.parametrize("n", [22, 26, 30])
def test_haar_against_stored_exact(ph, n):
    a = I.haar1600_block(n)
    ex = G.value_for("haar", f"haar1600_block_n{n}", a)
    if ex is None:
        pytest.skip(f"no stored exact value for n={n}")
    got = complex(ph.perm_ryser_paired(cuda(a)).cpu())
    assert O.rel_err(got, ex) <= ryser_tol(n)


def test_all_ones_and_diagonal_closed_forms(ph):
    import math

    # all ones: every term |S|^n is an exact integer up to n = 12, so n! comes
    # out exactly (larger n meet Ryser's cancellation, the paper's precision issue)
    for n in (1, 7, 12):
        ones = np.ones((n, n), np.complex128)
        assert complex(ph.perm_ryser_paired(cuda(ones)).cpu()) == float(math.factorial(n)), n
    # diag(1 + i): only S = all columns (the complement of the empty S) is nonzero
    d = np.diag(np.full(32, 1 + 1j))
    got = complex(ph.perm_ryser_paired(cuda(d)).cpu())
    assert got == complex((1 + 1j) ** 32)


def test_orders_beyond_the_kernels_raise(ph):
    with pytest.raises(ph.PermhipError):
        ph.perm_ryser_paired(cuda(np.ones((33, 33), np.complex128)))


@pytest.mark.parametrize("n", [13, 17, 18, 19, 20, 23, 26, 31, 32])
def test_two_permutations_closed_form_bit_exact(ph, n):
    # Per(D (P + Q)) = prod(D) 2^(cycles of P^-1 Q) for permutation matrices P, Q
    # and a diagonal D of units: every row sum and complement sum has modulus
    # <= 2, so every term is an exact integer and the sum is exact.  Covers the
    # one-lane walk (n <= 18) and the two-lane walk, odd n with its padding row.
    # The closed form is pinned against the definition on the CPU
    # (test_two_permutations_closed_form in tests/test_oracle_pins.py).
    a, want = CF.two_permutations(n, 4000 + n)
    assert complex(ph.perm_ryser_paired(cuda(a)).cpu()) == want
    assert complex(ph.perm(cuda(a)).cpu()) == want  # BB/FG on the same matrix


@pytest.mark.parametrize("c", [2, 4, 5, 9, 14])
def test_two_lane_chunk_lengths_bit_exact(ph, c):
    # the two-lane walk (n >= 19) steps in blocks of 16: shorter requested
    # chunks become 16 indices; every chunk length gives the exact closed form
    a, want = CF.two_permutations(23, 5000 + c)
    assert complex(ph.perm_ryser_paired(cuda(a), chunk_log2=c).cpu()) == want
    assert complex(ph.perm_ryser_paired(cuda(a), chunk_log2=c, accum="plain").cpu()) == want
