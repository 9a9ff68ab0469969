"""Boson-sampling layer (ph_boson_probs / ph_boson_probs_grad): Eq. (1)
probabilities against the oracle's exact values, completeness of the output
distribution, the gradient against exact minors, and at the full workload
(U 900 x 900, 30 photons, 256 collision patterns) the identities that hold
at any size."""
import itertools
import math

import numpy as np
import pytest

import inputs as I
import oracle as O
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
    return torch.from_numpy(np.array(a, copy=True)).to("cuda")


def all_patterns(m, n):
    return np.array(list(itertools.combinations_with_replacement(range(m), n)), dtype=np.int64).reshape(-1, n)


def rel(a, b):
    return abs(a - b) / abs(b)


# A permanent is accurate to 1e-10 relative (complex inputs, BB/FG with a
# double-double outer sum); Pr = |Per|^2 / D then carries twice that.
PERM_TOL = 1e-10
PROB_TOL = 2 * PERM_TOL


@pytest.mark.parametrize("ins", [[0, 1, 2], [0, 0, 3], [5, 1, 1, 2], [2, 2, 2]])
def test_all_patterns_small_against_oracle_and_completeness(ph, ins):
    m = 6
    u = I.haar(m, 7)
    pats = all_patterns(m, len(ins))
    pr = ph.boson_probs(cuda(u), ins, pats).cpu().numpy()
    ex = [float(O.prob_exact(u, ins, p)) for p in pats]
    for k, p in enumerate(pats):
        assert abs(pr[k] - ex[k]) <= 1e-12 * ex[k] + 1e-16, (list(p), pr[k], ex[k])
    # sum over every output pattern of n photons is 1 for a unitary U
    assert abs(math.fsum(pr) - 1.0) <= 1e-12


def test_collisions_against_multiplicity_route(ph):
    # repeated output rows checked against the grouped Ryser form (a route
    # that never builds the repeated matrix)
    m, n = 12, 7
    u = I.haar(m, 8)
    rng = np.random.default_rng(9)
    pats = np.stack([np.sort(rng.choice(m, n, replace=True)) for _ in range(12)])
    ins = [0, 1, 2, 3, 3, 5, 6]
    pr = ph.boson_probs(cuda(u), ins, pats).cpu().numpy()
    for k, p in enumerate(pats):
        e = float(O.prob_multiplicity(u, ins, p))
        assert rel(pr[k], e) <= 1e-11, (list(p), pr[k], e)


def test_grouped_sweeps_against_multiplicity_route(ph):
    # patterns with 5+ single-photon modes and doubly / triply occupied modes
    # take the multiplicity-grouped sweeps; the oracle's grouped Ryser route
    # is independent of them
    m, n = 40, 12
    u = I.haar(m, 18)
    rng = np.random.default_rng(19)
    pats = []
    for c2, c3 in [(1, 0), (2, 1), (0, 1), (3, 0), (1, 1), (2, 0)]:
        modes = rng.choice(m, n - c2 - 2 * c3, replace=False)
        pats.append(np.sort(np.concatenate([modes, modes[:c2], np.repeat(modes[c2:c2 + c3], 2)])))
    pats = np.stack(pats)
    ins = list(range(n))
    pr = ph.boson_probs(cuda(u), ins, pats).cpu().numpy()
    pu = ph.boson_probs(cuda(u), ins, pats, ungrouped=True).cpu().numpy()
    for k, p in enumerate(pats):
        e = float(O.prob_multiplicity(u, ins, p))
        assert rel(pr[k], e) <= 1e-11, (list(p), pr[k], e)
        assert rel(pu[k], e) <= 1e-11, (list(p), pu[k], e)


def test_reduced_workload_against_oracle(ph):
    # the full workload's recipe (Haar(900), collision patterns) at 16 photons
    u, ins, pats = I.boson_workload(n=16, patterns=8)
    pr = ph.boson_probs(cuda(u), ins, pats).cpu().numpy()
    for k in range(len(pats)):
        e = float(O.prob_exact(u, ins, pats[k]))
        assert rel(pr[k], e) <= 1e-11, (k, pr[k], e)
    # the gradient sweep's by-product probabilities agree as well
    pg, _ = ph.boson_probs_grad(cuda(u), ins, pats)
    assert np.max(np.abs(pg.cpu().numpy() - pr) / pr) <= 1e-11


def exact_du(u, ins, pats, w):
    """dU[r, k] = sum over (p, i) with T_p[i] = r of g_p conj(M_p[i, k]),
    g_p = 2 w_p Per_p / (prod s! prod t!), from exact minors."""
    m, n = u.shape[0], len(ins)
    du = np.zeros((m, n), dtype=np.complex128)
    for p, pat in enumerate(pats):
        a = O.gather_u_st(u, ins, pat)
        per = O.to_complex(O.perm_exact(a))
        d = O.occupation_factorials(ins) * O.occupation_factorials(pat)
        g = 2.0 * w[p] * per / d
        for i in range(n):
            for k in range(n):
                mik = O.to_complex(O.minor_perm_exact(a, i, k)) if n > 1 else 1.0
                du[pat[i], k] += g * np.conj(mik)
    return du


@pytest.mark.parametrize("ins", [[0, 1, 2], [1, 1, 4], [0, 2, 3, 5]])
def test_grad_small_against_exact_minors(ph, ins):
    m = 6
    u = I.haar(m, 11)
    pats = all_patterns(m, len(ins))
    w = np.random.default_rng(12).uniform(-1.0, 2.0, len(pats))
    pr, du = ph.boson_probs_grad(cuda(u), ins, pats, weights=cuda(w))
    ex = exact_du(u, ins, pats, w)
    scale = np.max(np.abs(ex))
    assert np.max(np.abs(du.cpu().numpy() - ex)) <= 1e-12 * scale
    ep = np.array([float(O.prob_exact(u, ins, p)) for p in pats])
    assert np.max(np.abs(pr.cpu().numpy() - ep)) <= 1e-14


def test_grouped_gradient_against_exact_minors(ph):
    # 7..9 photons, at least 5 in single-photon modes: the gradient goes
    # through the multiplicity-grouped sweeps (and, flagged, full sweeps)
    m = 14
    u = I.haar(m, 20)
    rng = np.random.default_rng(21)
    # (9 photons with 5 single-photon modes: the 8-lane gradient walks at
    # least 6 columns, so that pattern takes one full sweep)
    cases = [(7, [3, 3, 0, 1, 2, 4, 5]), (8, [0, 0, 1, 1, 2, 3, 4, 5]), (9, [6, 6, 6, 7, 8, 9, 10, 11, 12]),
             (9, [6, 6, 7, 7, 8, 9, 10, 11, 12])]
    for n, pat in cases:
        ins = sorted(rng.choice(m, n, replace=False).tolist())
        pats = np.array([sorted(pat), sorted(rng.choice(m, n, replace=False).tolist())])
        w = np.array([1.5, -0.25])
        ex = exact_du(u, ins, pats, w)
        scale = np.max(np.abs(ex))
        for ungrouped in (False, True):
            pr, du = ph.boson_probs_grad(cuda(u), ins, pats, weights=cuda(w), ungrouped=ungrouped)
            assert np.max(np.abs(du.cpu().numpy() - ex)) <= 1e-12 * scale, (n, ungrouped)
            ep = np.array([float(O.prob_exact(u, ins, p)) for p in pats])
            assert np.max(np.abs(pr.cpu().numpy() - ep) / ep) <= 1e-12, (n, ungrouped)


def test_grad_single_photon(ph):
    # n = 1: Pr = |U[t, s]|^2, dL/dU[:, s] = 2 w U[t, s] at row t
    m = 5
    u = I.haar(m, 13)
    pats = np.array([[0], [3], [3], [4]])
    w = np.array([1.0, 0.5, 0.25, -1.0])
    pr, du = ph.boson_probs_grad(cuda(u), [2], pats, weights=cuda(w))
    exp = np.zeros((m, 1), dtype=np.complex128)
    for p, t in enumerate(pats[:, 0]):
        exp[t, 0] += 2 * w[p] * u[t, 2]
    assert np.allclose(du.cpu().numpy(), exp, rtol=0, atol=1e-15)
    assert np.allclose(pr.cpu().numpy(), np.abs(u[pats[:, 0], 2]) ** 2, rtol=1e-15, atol=0)


def test_empty_pattern_list(ph):
    u = cuda(I.haar(4, 14))
    assert ph.boson_probs(u, [0, 1], np.zeros((0, 2), dtype=np.int64)).numel() == 0
    pr, du = ph.boson_probs_grad(u, [0, 1], np.zeros((0, 2), dtype=np.int64))
    assert pr.numel() == 0 and torch.count_nonzero(du).item() == 0


def test_zero_photons(ph):
    # n = 0: Per of the empty matrix is 1, so every (empty) pattern has Pr = 1
    u = cuda(I.haar(4, 15))
    pr = ph.boson_probs(u, [], np.zeros((3, 0), dtype=np.int64))
    assert pr.cpu().tolist() == [1.0, 1.0, 1.0]


def test_strided_u_rows(ph):
    m = 7
    big = I.haar(11, 16)
    u = big[:m, :m]  # a view with row stride 11
    ut = torch.from_numpy(big.copy()).to("cuda")[:m, :m]
    pats = all_patterns(m, 3)[::5]
    a = ph.boson_probs(ut, [0, 4, 6], pats).cpu().numpy()
    b = ph.boson_probs(cuda(u), [0, 4, 6], pats).cpu().numpy()
    assert np.array_equal(a, b)


def test_autograd_gradcheck(ph):
    # a non-unitary complex U: the gradient convention checked numerically
    rng = np.random.default_rng(17)
    m = 5
    u = torch.tensor(rng.normal(size=(m, m)) + 1j * rng.normal(size=(m, m)), dtype=torch.complex128,
                     device="cuda", requires_grad=True)
    ins = [0, 2, 2]
    pats = all_patterns(m, 3)[::3]
    f = lambda x: ph.boson_probabilities(x, ins, pats)  # noqa: E731
    assert torch.autograd.gradcheck(f, (u,), eps=1e-6, atol=1e-7, rtol=1e-6)


@pytest.fixture(scope="module")
def full_workload(ph):
    u, ins, pats = I.boson_workload()
    ud = cuda(u)
    w = np.random.default_rng(53).uniform(0.5, 1.5, len(pats))
    pf = ph.boson_probs(ud, ins, pats)
    pg, du = ph.boson_probs_grad(ud, ins, pats, weights=cuda(w))
    torch.cuda.synchronize()
    return u, ins, pats, w, pf.cpu().numpy(), pg.cpu().numpy(), du.cpu().numpy()


def test_full_workload_forward_paths_agree(ph, full_workload):
    u, ins, pats, w, pf, pg, du = full_workload
    assert np.all(pf > 0) and np.all(np.isfinite(pf))
    # batched forward sweep vs the gradient sweep's permanents: two kernels
    # with different chunkings, each within PROB_TOL of the exact value
    assert np.max(np.abs(pf - pg) / pf) <= 2 * PROB_TOL
    # the permanents of the gathered matrices through the plain batched entry
    # point (full sweeps) against the multiplicity-grouped sweeps
    a = np.stack([O.gather_u_st(u, ins, p) for p in pats])
    per = ph.perm_batched(cuda(a)).cpu().numpy()
    d = np.array([O.occupation_factorials(ins) * O.occupation_factorials(p) for p in pats], dtype=np.float64)
    assert np.max(np.abs(np.abs(per) ** 2 / d - pf) / pf) <= 2 * PROB_TOL


def test_full_workload_against_stored_exact(ph, full_workload):
    # exact Per of three of the 256 thirty-photon patterns, written by the
    # oracle (tests/golden/make_golden.py boson): patterns 11 and 234 (3888
    # multiplicity-grouped sweeps of 14 single-photon columns each, the most
    # any pattern of the workload takes) and 5 (3 grouped sweeps of 28
    # columns); Eq. (1) normalises by prod t_j!.  The probability call, the
    # gradient call's by-product and the whole 2^29-term sweep of the gathered
    # 30 x 30 matrix (perm_batched) are each held to the exact value.
    from fractions import Fraction

    u, ins, pats, w, pf, pg, du = full_workload
    gold = G.load("boson")
    checked = 0
    for p in (11, 234, 5):
        name = f"boson_workload_p{p}"
        if name not in gold:
            continue
        a = O.gather_u_st(u, ins, pats[p])
        ex_re, ex_im = G.value_for("boson", name, a)
        d = O.occupation_factorials(ins) * O.occupation_factorials(pats[p])
        exact = (ex_re * ex_re + ex_im * ex_im) / d
        whole = complex(ph.perm_batched(cuda(a[None])).cpu()[0])
        for got in (pf[p], pg[p], abs(whole) ** 2 / float(d)):
            assert abs(Fraction(float(got)) - exact) <= Fraction(PROB_TOL) * exact, (p, got, float(exact))
        checked += 1
    assert checked == 3, "stored exact values of the thirty-photon patterns are missing"


def test_full_workload_row_and_column_laplace(ph, full_workload):
    # Laplace expansion of every Per_p along row i and along column k gives
    #   sum_k U[r, S_k] conj(dU[r, k]) = 2 sum_p w_p Pr_p t_{p, r}   (each output mode r)
    #   sum_r U[r, S_k] conj(dU[r, k]) = 2 sum_p w_p Pr_p            (each photon k)
    u, ins, pats, w, pf, pg, du = full_workload
    m, n = u.shape[0], len(ins)
    us = u[:, ins]
    row = np.sum(us * np.conj(du), axis=1)
    t = np.zeros(m)
    for p, pat in enumerate(pats):
        np.add.at(t, pat, w[p] * pg[p])
    used = np.unique(pats)
    # each minor is within PERM_TOL of exact, so the n-term Laplace sums are
    # within PERM_TOL * sum |U||dU| (no cancellation assumed); the right-hand
    # sides within PROB_TOL
    mag = np.abs(us) * np.abs(du)
    tol_r = PERM_TOL * mag.sum(axis=1) + PROB_TOL * 2 * t
    assert np.all(np.abs(row[used] - 2 * t[used]) <= tol_r[used])
    unused = np.setdiff1d(np.arange(m), used)
    assert np.count_nonzero(du[unused]) == 0
    col = np.sum(us * np.conj(du), axis=0)
    total = 2 * np.sum(w * pg)
    tol_k = PERM_TOL * mag.sum(axis=0) + PROB_TOL * total
    assert np.all(np.abs(col - total) <= tol_k)
    assert n == du.shape[1]


def test_full_workload_grouped_against_ungrouped(ph, full_workload):
    # multiplicity-grouped sweeps (fewer terms) against one full sweep per
    # pattern: two different sums of the same permanents
    u, ins, pats, w, pf, pg, du = full_workload
    pu = ph.boson_probs(cuda(u), ins, pats, ungrouped=True).cpu().numpy()
    assert np.max(np.abs(pu - pf) / pf) <= 2 * PROB_TOL


def test_full_workload_gradient_grouped_against_ungrouped(ph, full_workload):
    u, ins, pats, w, pf, pg, du = full_workload
    pu, duu = ph.boson_probs_grad(cuda(u), ins, pats, weights=cuda(w), ungrouped=True)
    duu = duu.cpu().numpy()
    assert np.max(np.abs(pu.cpu().numpy() - pg) / pg) <= 2 * PROB_TOL
    # entries of dU are sums of terms of either sign; compare on the scale of
    # each row
    scale = np.max(np.abs(duu), axis=1, keepdims=True) + 1e-300
    assert np.max(np.abs(du - duu) / scale) <= 1e-9


def test_full_workload_phase_invariance(ph, full_workload):
    # phases on the input columns and output rows of U leave every Pr unchanged
    u, ins, pats, w, pf, pg, du = full_workload
    m = u.shape[0]
    rng = np.random.default_rng(54)
    ph_r = np.exp(2j * np.pi * rng.random(m))
    ph_c = np.exp(2j * np.pi * rng.random(m))
    u2 = (ph_r[:, None] * u) * ph_c[None, :]
    p2 = ph.boson_probs(cuda(u2), ins, pats).cpu().numpy()
    assert np.max(np.abs(p2 - pf) / pf) <= 2 * PROB_TOL


@pytest.mark.parametrize("m,ins,pat_seed", [(6, [1, 1, 4], 31), (14, [2, 2, 5, 6, 7, 8, 9, 10], 32),
                                            (14, [0, 3, 3, 3, 4, 5, 6, 7, 8], 33)])
def test_full_du_folds_photons_onto_columns(ph, m, ins, pat_seed):
    # PH_FLAG_DU_FULL: the m x m gradient with respect to U, the columns of
    # photons that share an input mode added in increasing photon order, the
    # columns of modes without a photon zero; both paths (3 photons: one sweep
    # per pattern; 8 and 9: multiplicity-grouped sweeps)
    u = cuda(I.haar(m, 40))
    n = len(ins)
    rng = np.random.default_rng(pat_seed)
    pats = np.sort(np.stack([rng.choice(m, n, replace=True) for _ in range(5)]), axis=1)
    pats[0] = np.sort(np.concatenate([[pats[0, 0]] * 2, rng.choice(m, n - 2, replace=False)]))
    w = cuda(rng.uniform(-1.0, 2.0, len(pats)))
    pr, du = ph.boson_probs_grad(u, ins, pats, weights=w)
    pf, full = ph.boson_probs_grad(u, ins, pats, weights=w, full=True)
    assert full.shape == (m, m)
    assert torch.equal(pr, pf)
    du, full = du.cpu().numpy(), full.cpu().numpy()
    want = np.zeros((m, m), dtype=np.complex128)
    for k in range(n):
        want[:, ins[k]] += du[:, k]
    assert np.array_equal(full, want)
    assert not np.any(full[:, [j for j in range(m) if j not in ins]])


def test_grouped_sweep_budget_runs_out(ph):
    # 70 thirty-photon patterns of 6 triply occupied and 12 single modes: each
    # needs 4^6 = 4096 grouped sweeps, so the call's budget of 2^18 grouped
    # sweeps lasts for the first 64 and the last 6 are swept whole.  The mixed
    # call agrees with the all-whole (ungrouped) call, for the probabilities
    # and the gradient.
    m, n = 200, 30
    u = I.haar(m, 61)
    ins = list(range(n))
    rng = np.random.default_rng(62)
    pats = []
    for _ in range(70):
        modes = rng.choice(m, 18, replace=False)
        pats.append(np.sort(np.concatenate([np.repeat(modes[:6], 3), modes[6:]])))
    pats = np.array(pats, dtype=np.int64)
    ud = cuda(u)
    pf = ph.boson_probs(ud, ins, pats).cpu().numpy()
    pu = ph.boson_probs(ud, ins, pats, ungrouped=True).cpu().numpy()
    assert np.all(pf > 0)
    assert np.max(np.abs(pf - pu) / pu) <= 2 * PROB_TOL
    w = cuda(np.random.default_rng(63).uniform(0.5, 1.5, len(pats)))
    pg, du = ph.boson_probs_grad(ud, ins, pats, weights=w)
    pgu, duu = ph.boson_probs_grad(ud, ins, pats, weights=w, ungrouped=True)
    assert np.max(np.abs(pg.cpu().numpy() - pu) / pu) <= 2 * PROB_TOL
    du, duu = du.cpu().numpy(), duu.cpu().numpy()
    scale = np.max(np.abs(duu), axis=1, keepdims=True) + 1e-300
    assert np.max(np.abs(du - duu) / scale) <= 1e-9
