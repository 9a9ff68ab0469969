"""Gradient sweep (ph_perm_grad) against the oracle's minor permanents,
finite differences and the Laplace / Euler identities."""
import math

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


def minors_exact(a):
    n = a.shape[0]
    return [[O.minor_perm_exact(a, i, j) for j in range(n)] for i in range(n)]


@pytest.mark.parametrize("n", list(range(1, 11)) + [13])
def test_all_minors_against_oracle(ph, n):
    u = I.haar(64, 100 + n)
    a = I.submatrix(u, range(2, 2 + n), range(n))
    p, g = ph.perm_grad(cuda(a))
    m = np.conj(g.cpu().numpy())  # grad_out = 1 -> conj(M)
    ex = minors_exact(a) if n > 1 else [[(1, 0)]]
    scale = max(abs(O.to_complex(ex[i][j])) for i in range(n) for j in range(n))
    for i in range(n):
        for j in range(n):
            e = O.to_complex(ex[i][j])
            assert abs(complex(m[i, j]) - e) <= 1e-12 * scale, (n, i, j)
    assert O.rel_err(complex(p.cpu()), O.perm_exact(a)) <= 1e-12


@pytest.mark.parametrize("n", [6, 9, 12])
def test_integer_matrix_minors(ph, n):
    rng = np.random.default_rng(n)
    a = (rng.integers(-2, 3, (n, n)) + 1j * rng.integers(-2, 3, (n, n))).astype(np.complex128)
    _, g = ph.perm_grad(cuda(a))
    m = np.conj(g.cpu().numpy())
    for i, j in [(0, 0), (n - 1, 0), (n // 2, n - 1), (1, 2)]:
        assert complex(m[i, j]) == O.to_complex(O.minor_perm_exact(a, i, j)), (i, j)


def test_batch_matches_single_and_upstream_scaling(ph):
    a = I.grad_batch_20(6)
    p, g = ph.perm_grad(cuda(a))
    w = torch.tensor([1 + 2j, -0.5, 3j, 1, 2, -1 - 1j], dtype=torch.complex128, device="cuda")
    p2, g2 = ph.perm_grad(cuda(a), grad_out=w)
    for b in range(6):
        pb, gb = ph.perm_grad(cuda(a[b]))
        assert torch.equal(p[b], pb) and torch.equal(g[b], gb)
        assert torch.allclose(g2[b], w[b] * g[b], rtol=1e-14, atol=0)
        fwd = complex(ph.perm(cuda(a[b])).cpu())
        assert abs(complex(pb.cpu()) - fwd) <= 1e-12 * abs(fwd)


def test_laplace_and_euler_identities_grad_batch(ph):
    """sum_j a_ij M_ij = Per(A) for every row i, sum_ij a_ij M_ij = n Per(A),
    on the 1024 x (20 x 20) benchmark batch."""
    a = I.grad_batch_20()
    p, g = ph.perm_grad(cuda(a))
    m = torch.conj(g)
    at = cuda(a)
    rows = (at * m).sum(dim=2)  # (batch, n)
    pp = p.unsqueeze(1)
    rel = ((rows - pp).abs() / pp.abs()).max().item()
    assert rel <= 1e-10, rel
    euler = (at * m).sum(dim=(1, 2))
    assert (((euler - 20 * p).abs() / (20 * p).abs()).max().item()) <= 1e-10


def test_finite_differences_n20(ph):
    """Central differences (h = 1e-6) of L = |Per(A)|^2 on the real and
    imaginary part of sampled entries, against dL/dA = 2 Per conj(M)."""
    a = I.grad_batch_20(1)[0]
    p, g = ph.perm_grad(cuda(a))
    p = complex(p.cpu())
    # g = conj(M) (upstream gradient 1); PyTorch's convention for L = |p|^2:
    # dL/dRe a + i dL/dIm a = 2 p conj(M)
    grad = 2 * p * g.cpu().numpy()
    rng = np.random.default_rng(7)
    h = 1e-6
    for _ in range(6):
        i, j = rng.integers(0, 20, 2)
        fd = []
        for d in (h, 1j * h):
            ap, am = a.copy(), a.copy()
            ap[i, j] += d
            am[i, j] -= d
            lp = abs(complex(ph.perm(cuda(ap)).cpu())) ** 2
            lm = abs(complex(ph.perm(cuda(am)).cpu())) ** 2
            fd.append((lp - lm) / (2 * h))
        num = fd[0] + 1j * fd[1]
        got = complex(grad[i, j])
        assert abs(num - got) <= 1e-5 * abs(got), (i, j, num, got)


def test_sampled_minors_of_grad_batch_matrix0(ph):
    a = I.grad_batch_20(1)[0]
    _, g = ph.perm_grad(cuda(a))
    m = np.conj(g.cpu().numpy())
    gold = G.load("minors")
    names = [k for k in gold if k.startswith("grad_batch_m0_")]
    if not names:
        for i, j in [(0, 0), (19, 7)]:
            ex = O.perm_exact_parallel(O.minor(a, i, j))
            assert O.rel_err(complex(m[i, j]), ex) <= 1e-10
        return
    for k in names:
        i, j = map(int, k.split("_")[-2:])
        _, sha, ex = gold[k]
        assert I.sha256_of(O.minor(a, i, j)) == sha
        assert O.rel_err(complex(m[i, j]), ex) <= 1e-10, (i, j)


def test_autograd_function(ph):
    n = 5
    a = cuda(I.submatrix(I.haar(30, 2), range(n), range(n))).requires_grad_(True)
    assert torch.autograd.gradcheck(ph.permanent, (a,), eps=1e-6, atol=1e-8, rtol=1e-6)
    b = cuda(I.grad_batch_20(3)).requires_grad_(True)
    loss = (ph.permanent(b).abs() ** 2).sum()
    loss.backward()
    p, g = ph.perm_grad(b.detach())
    assert torch.allclose(b.grad, 2 * p.view(3, 1, 1) * g, rtol=1e-12, atol=0)


@pytest.mark.parametrize("n", [21, 25, 30, 32])
def test_larger_n_identities(ph, n):
    a = I.haar1600_block(n) if n <= 30 else I.submatrix(I.haar(1600, 31), range(n), range(n))
    p, g = ph.perm_grad(cuda(a))
    m = torch.conj(g)
    rows = (cuda(a) * m).sum(dim=1)
    rel = ((rows - p).abs() / p.abs()).max().item()
    assert rel <= 1e-9, rel
    fwd = complex(ph.perm(cuda(a)).cpu())
    assert abs(complex(p.cpu()) - fwd) <= 1e-11 * abs(fwd)


@pytest.mark.parametrize("n", [8, 9, 16, 17])
def test_sampled_minors_at_layout_boundaries(ph, n):
    # the sweep changes its lane layout with n (4 -> 8 lanes per term above 8,
    # 2 -> 3 rows per lane above 16); exact minors on both sides
    a = I.submatrix(I.haar(64, 300 + n), range(3, 3 + n), range(n))
    p, g = ph.perm_grad(cuda(a))
    m = np.conj(g.cpu().numpy())
    rng = np.random.default_rng(n)
    picks = [(0, 0), (n - 1, n - 1), (n // 2, 1)] + [tuple(rng.integers(0, n, 2)) for _ in range(2)]
    for i, j in picks:
        assert O.rel_err(complex(m[i, j]), O.minor_perm_exact(a, int(i), int(j))) <= 1e-10, (n, i, j)
    assert O.rel_err(complex(p.cpu()), O.perm_exact(a)) <= 1e-10


@pytest.mark.parametrize("n", [22, 24, 26, 28, 30])
def test_sweep_permanent_against_stored_exact(ph, n):
    # the permanent the gradient sweep produces on the way (3 and 4 rows per
    # lane) against the oracle's stored exact value
    a = I.haar1600_block(n)
    ex = G.value_for("haar", f"haar1600_block_n{n}", a)
    if ex is None:
        pytest.skip("stored value absent")
    p, _ = ph.perm_grad(cuda(a))
    assert O.rel_err(complex(p.cpu()), ex) <= 1e-10


@pytest.mark.parametrize("n", [5, 12, 17, 20, 21, 24, 25, 32])
def test_two_permutations_exact_minors(ph, n):
    # D (P + Q) (tests/_closed_forms.py): every row sum of the sweep has modulus
    # <= 2, so every leave-one-out product and running sum is an exact integer
    # and the minors come out exactly.  One case per lane layout (4 x 2, 8 x 2,
    # 4 x 5, 8 x 3, 8 x 4 rows); the Laplace expansions along every row and
    # every column (two nonzero entries each) give Per bit for bit.
    a, want = CF.two_permutations(n, 7000 + n)
    p, g = ph.perm_grad(cuda(a))
    assert complex(p.cpu()) == want
    m = np.conj(g.cpu().numpy())
    assert np.array_equal(m.real, np.round(m.real)) and np.array_equal(m.imag, np.round(m.imag))
    assert np.all((a * m).sum(axis=1) == want)
    assert np.all((a * m).sum(axis=0) == want)
