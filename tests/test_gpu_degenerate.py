"""Degenerate inputs through every entry point: a zero row makes every term of
Eq. (S1) and Eq. (S2) exactly zero (its row sum is a sum of zeros), so the
permanent is exactly 0 whatever the order of the sums; the gradient's other
rows are exactly 0 too (their minors keep the zero row), while the zero row's
own entries are the minors along it.  Non-finite entries propagate (the
boundary does not check for them) instead of failing.
"""
import numpy as np
import pytest

import inputs as I
import oracle as O

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


def with_zero_row(n, row, seed=0):
    a = I.haar1600_block(n).copy() if n >= 20 else I.haar(64, 900 + seed)[:n, :n].copy()
    a[row] = 0
    return a


@pytest.mark.parametrize("n", [1, 2, 7, 20, 33])
def test_zero_row_gives_exactly_zero(ph, n):
    for row in sorted({0, n // 2, n - 1}):
        a = cuda(with_zero_row(n, row, n))
        for algo in ("glynn", "ryser"):
            for accum in ("dd", "plain"):
                assert complex(ph.perm(a, algo=algo, accum=accum).cpu()) == 0, (n, row, algo, accum)
        if n <= 32:
            assert complex(ph.perm_ryser_paired(a).cpu()) == 0, (n, row)


@pytest.mark.parametrize("n", [40, 44, 46, 52])
def test_zero_row_large_orders_share_is_zero(ph, n):
    # one share of 64 chunks high in the range (one lane per term up to 44,
    # two lanes from 45), both formulas
    for algo in ("glynn", "ryser"):
        c = ph.perm_chunk_log2(n, algo)
        k0 = ph.gray_terms(n, algo) // 2 + (5 << c)
        part = ph.perm_partial(cuda(with_zero_row(n, n - 2)), k0, k0 + (64 << c), algo=algo)
        assert (part.cpu().numpy() == 0).all(), (n, algo)


def test_zero_row_batched_and_shares(ph):
    mats = [with_zero_row(n, row, n) for n, row in ((3, 2), (9, 4), (17, 16), (24, 0), (26, 13), (30, 7))]
    got = ph.perm_batched([cuda(m) for m in mats]).cpu().numpy()
    assert (got == 0).all(), got
    # shares of one zero-row permanent are zero partials that combine to 0
    a = cuda(with_zero_row(22, 4))
    half = ph.gray_terms(22) // 2
    parts = torch.stack([ph.perm_partial(a, 0, half), ph.perm_partial(a, half, 2 * half)])
    assert (parts.cpu().numpy() == 0).all()
    assert complex(ph.perm_combine(parts, 22).cpu()) == 0


@pytest.mark.parametrize("n", [3, 8, 9])
def test_zero_row_gradient(ph, n):
    # integer entries: the minors are exact in binary64
    rng = np.random.default_rng(40 + n)
    a = (rng.integers(-2, 3, (n, n)) + 1j * rng.integers(-2, 3, (n, n))).astype(np.complex128)
    z = n // 3
    a[z] = 0
    p, g = ph.perm_grad(cuda(a))
    assert complex(p.cpu()) == 0
    g = g.cpu().numpy()
    others = np.delete(g, z, axis=0)
    assert (others == 0).all()
    for j in range(n):
        want = O.to_complex(O.minor_perm_exact(a, z, j))
        assert g[z, j] == np.conj(want), (j, g[z, j], want)


def test_non_finite_entries_propagate(ph):
    for bad in (float("nan"), float("inf")):
        a = I.haar1600_block(20).copy()
        a[3, 5] = complex(bad, 0.0)
        for algo in ("glynn", "ryser"):
            v = complex(ph.perm(cuda(a), algo=algo).cpu())
            assert not (np.isfinite(v.real) and np.isfinite(v.imag)), (bad, algo, v)
