"""Minors along one row (ph_perm_row_minors): against the exact oracle, the
Laplace expansion against the forward sweep, and the gradient sweep's last
row; and the sampler at step sizes that use them."""
import numpy as np
import pytest

import inputs as I
import oracle as O
from tests import _closed_forms as CF
from oracle import sampler as OS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ph():
    import paper_1606_05836_amd as ph

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return ph


def blocks(n, count, seed):
    u = I.haar(max(4 * n, 8), seed)
    rng = np.random.default_rng(seed)
    return np.stack([u[np.sort(rng.choice(u.shape[0], n, replace=False))][:, : n + 1] for _ in range(count)])


@pytest.mark.parametrize("n,count", [(0, 2), (1, 3), (2, 3), (5, 3), (10, 2), (12, 1), (13, 1)])
def test_minors_against_oracle(ph, n, count):
    b = blocks(n, count, 100 + n) if n else np.zeros((count, 0, 1), np.complex128)
    got = ph.perm_row_minors(torch.from_numpy(b).to("cuda")).cpu().numpy()
    assert got.shape == (count, n + 1)
    for q in range(count):
        ex = [O.to_complex(O.perm_exact(np.delete(b[q], l, axis=1))) for l in range(n + 1)]
        big = max(abs(e) for e in ex)
        for l in range(n + 1):
            assert abs(got[q, l] - ex[l]) <= 1e-12 * big, (q, l)


@pytest.mark.parametrize("n", [20, 25, 31])
def test_laplace_expansion_and_gradient_row(ph, n):
    b = blocks(n, 2, 200 + n)
    bt = torch.from_numpy(b).to("cuda")
    p = ph.perm_row_minors(bt)
    rng = np.random.default_rng(n)
    for q in range(2):
        x = (rng.standard_normal(n + 1) + 1j * rng.standard_normal(n + 1)) / np.sqrt(2 * n)
        full = np.vstack([b[q], x[None, :]])
        per = complex(ph.perm(torch.from_numpy(full).to("cuda")).cpu())
        lap = complex((p[q] * torch.from_numpy(x).to("cuda")).sum().cpu())
        assert abs(lap - per) <= 1e-11 * abs(per), (q, lap, per)
    # the gradient sweep of [B; 0] gives the same minors in its last row
    sq = np.concatenate([b, np.zeros((2, 1, n + 1), np.complex128)], axis=1)
    _, g = ph.perm_grad(torch.from_numpy(sq).to("cuda"))
    via_grad = np.conj(g.cpu().numpy()[:, n, :])
    pn = p.cpu().numpy()
    assert np.max(np.abs(pn - via_grad)) <= 1e-12 * np.max(np.abs(via_grad))


def test_sampler_steps_through_row_minors_match_oracle(ph):
    # 14 photons: steps 13 and 14 expand along minors of 12 and 13 rows
    u = I.haar(16, 12)
    ins = list(range(0, 16, 1))[:14]
    perms, unis = ph.sample_inputs(3, 14, 13)
    got = ph.boson_sample(torch.from_numpy(u).to("cuda"), ins, perms=perms, uniforms=unis).cpu().numpy()
    from fractions import Fraction

    compared = 0
    for s in range(3):
        trace = []
        want = OS.sample_exact(u, ins, tuple(int(x) for x in perms[s]), [float(x) for x in unis[s]], trace)
        clear = True
        for (w, r), uu in zip(trace, unis[s]):
            tot = sum(w)
            t = Fraction(float(uu)) * tot
            if min(t - sum(w[:r]), sum(w[: r + 1]) - t) <= Fraction(1e-9) * tot:
                clear = False
        if clear:
            assert tuple(int(x) for x in got[s]) == want, s
            compared += 1
    assert compared >= 2


def test_plain_accumulation_and_batch_shapes(ph):
    # the plain binary64 outer sum agrees with double-double to rounding, for
    # both paths; leading batch dimensions come back as given
    for n in (9, 16):
        b = blocks(n, 6, 300 + n).reshape(2, 3, n, n + 1)
        bt = torch.from_numpy(b).to("cuda")
        dd = ph.perm_row_minors(bt)
        pl = ph.perm_row_minors(bt, accum="plain")
        assert dd.shape == (2, 3, n + 1)
        big = dd.abs().max().item()
        assert (dd - pl).abs().max().item() <= 1e-12 * big
    with pytest.raises(ValueError):
        ph.perm_row_minors(torch.zeros((3, 3), dtype=torch.complex128, device="cuda"))


@pytest.mark.parametrize("n", [5, 11, 12, 16, 20, 25, 29, 31])
def test_two_permutations_row_expansion_exact(ph, n):
    # C = D (P + Q), (n + 1) x (n + 1) (tests/_closed_forms.py), and B its
    # first n rows: every row sum of the sweep has modulus <= 2, so the n + 1
    # minors of B are exact Gaussian integers and the expansion along C's last
    # row is Per(C) bit for bit (the gradient path below 12 rows, the row sweep
    # from 12)
    c, want = CF.two_permutations(n + 1, 8000 + n)
    minors = ph.perm_row_minors(torch.from_numpy(np.ascontiguousarray(c[:n])).to("cuda")).cpu().numpy()
    assert np.array_equal(minors.real, np.round(minors.real)) and np.array_equal(minors.imag, np.round(minors.imag))
    assert complex((c[n] * minors).sum()) == want
