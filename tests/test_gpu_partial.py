"""Shares of the Gray-code sum (ph_perm_partial / ph_perm_combine) and the
checkpointed segment runner on the GPU, against the exact oracle's partial
sums over the same index ranges."""
from fractions import Fraction

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


def small_int(n, seed):
    # entries in {-1, 0, 1} + i{-1, 0, 1}
    rng = np.random.default_rng(seed)
    return (rng.integers(-1, 2, (n, n)) + 1j * rng.integers(-1, 2, (n, n))).astype(np.complex128)


def cuts(total, c, pieces, seed):
    """Aligned cut points of [0, total): uneven shares, an empty one and a
    single-chunk one included when there is room."""
    L = 1 << c
    nch = total // L
    rng = np.random.default_rng(seed)
    inner = sorted(set(int(x) for x in rng.integers(0, nch + 1, pieces - 1)) | ({1} if nch > 1 else set()))
    pts = [0] + inner + [inner[-1] if inner else 0] + [nch]  # the repeat gives an empty share
    return [(pts[i] * L, pts[i + 1] * L) for i in range(len(pts) - 1)]


def raw_exact(g, algo, kb, ke):
    return O.glynn_gray_raw(g, kb, ke) if algo == "glynn" else O.ryser_gray_raw(g, kb, ke)


def dd_value(p):
    return Fraction(p[0]) + Fraction(p[1]), Fraction(p[2]) + Fraction(p[3])


@pytest.mark.parametrize("algo,n", [("glynn", 1), ("glynn", 2), ("glynn", 3), ("glynn", 6), ("glynn", 11),
                                    ("ryser", 1), ("ryser", 2), ("ryser", 5), ("ryser", 11)])
def test_integer_partials_bit_exact(ph, algo, n):
    # |row sum| <= n sqrt(2), so every product is below 15.6^11 < 2^44 and a
    # block of 16 of them summed in binary64 before a double-double flush stays
    # below 2^53: the partials are exact
    a = small_int(n, 300 + n)
    g, d = O.to_gaussian_integers(a)
    assert d == 1
    c = ph.perm_chunk_log2(n, algo)
    total = ph.gray_terms(n, algo)
    at = cuda(a)
    parts = []
    for kb, ke in cuts(total, c, 5, n):
        p = ph.perm_partial(at, kb, ke, algo=algo).cpu().tolist()
        ex = raw_exact(g, algo, kb, ke)
        assert dd_value(p) == (Fraction(ex[0]), Fraction(ex[1])), (kb, ke)
        if kb == ke:
            assert p == [0.0, 0.0, 0.0, 0.0]
        parts.append(p)
    per = ph.perm_combine(torch.tensor(parts, dtype=torch.float64, device="cuda"), n, algo=algo)
    assert complex(per.cpu()) == O.to_complex(O.perm_exact(a))


@pytest.mark.parametrize("algo", ["glynn", "ryser"])
def test_haar_shares_against_oracle(ph, algo):
    n = 14 if algo == "glynn" else 12
    a = I.submatrix(I.haar(64, 5), range(3, 3 + n), range(n))
    g, d = O.to_gaussian_integers(a)
    scale = Fraction(1, d ** n)
    c = ph.perm_chunk_log2(n, algo)
    shares = cuts(ph.gray_terms(n, algo), c, 6, 7)
    at = cuda(a)
    got = [ph.perm_partial(at, kb, ke, algo=algo).cpu().tolist() for kb, ke in shares]
    exact = []
    for kb, ke in shares:
        re, im = raw_exact(g, algo, kb, ke)
        exact.append(complex(float(re * scale), float(im * scale)))
    big = max(abs(e) for e in exact)
    for p, e, (kb, ke) in zip(got, exact, shares):
        v = complex(p[0] + p[1], p[2] + p[3])
        assert abs(v - e) <= (1e-13 if algo == "glynn" else 1e-11) * big, (kb, ke, v, e)
    per = complex(ph.perm_combine(torch.tensor(got, dtype=torch.float64, device="cuda"), n, algo=algo).cpu())
    assert O.rel_err(per, O.perm_exact(a)) <= (1e-12 if algo == "glynn" else 1e-10)


def test_one_share_is_the_whole_permanent(ph):
    for n, accum in ((20, "dd"), (20, "plain"), (27, "dd")):
        a = cuda(I.haar1600_block(n))
        whole = complex(ph.perm(a, accum=accum).cpu())
        p = ph.perm_partial(a, 0, ph.gray_terms(n), accum=accum)
        if accum == "plain":
            assert p[1].item() == 0.0 and p[3].item() == 0.0
        one = complex(ph.perm_combine(p.reshape(1, 4), n, accum=accum).cpu())
        assert abs(one - whole) <= 1e-15 * abs(whole)
        # five uneven shares give the same value up to the rounding of the reduction
        shares = cuts(ph.gray_terms(n), ph.perm_chunk_log2(n), 5, n)
        parts = torch.stack([ph.perm_partial(a, kb, ke, accum=accum) for kb, ke in shares])
        five = complex(ph.perm_combine(parts, n, accum=accum).cpu())
        assert abs(five - whole) <= (1e-15 if accum == "dd" else 1e-12) * abs(whole)


def test_misaligned_and_out_of_range_shares_raise(ph):
    a = cuda(I.haar1600_block(20))
    L = 1 << ph.perm_chunk_log2(20)
    with pytest.raises(ph.PermhipError):
        ph.perm_partial(a, 1, L)
    with pytest.raises(ph.PermhipError):
        ph.perm_partial(a, 0, ph.gray_terms(20) + L)
    with pytest.raises(ph.PermhipError):
        ph.perm_partial(a, 2 * L, L)


def test_eight_shares_of_n40_as_eight_devices(ph):
    # the contiguous split the sharded design gives 8 devices, each share at its real shape
    n = 40
    a = cuda(I.haar1600_block(n))
    total = ph.gray_terms(n)
    parts = torch.stack([ph.perm_partial(a, total * g // 8, total * (g + 1) // 8) for g in range(8)])
    per = complex(ph.perm_combine(parts, n).cpu())
    whole = complex(ph.perm(a).cpu())
    assert abs(per - whole) <= 1e-14 * abs(whole)


@pytest.mark.parametrize("n", [48, 52])
def test_large_n_share_exact_on_diag_one_plus_i(ph, n):
    # every BB/FG term of diag(d) equals prod d (the delta signs cancel), so a
    # share of m terms sums to m (1+i)^n exactly: (2i)^(n/2) = 2^(n/2) i^(n/2)
    a = cuda(I.diag_matrix(n, 1 + 1j))
    m = 1 << 36
    kb = (1 << (n - 2)) + (5 << 36)
    p = ph.perm_partial(a, kb, kb + m).cpu().tolist()
    want = m * (2 ** (n // 2)) * (1j ** (n // 2))
    assert complex(p[0] + p[1], p[2] + p[3]) == want
    assert p[1] == 0.0 and p[3] == 0.0


def test_split_additivity_at_n46(ph):
    n = 46
    a = cuda(I.haar1600_block(n))
    kb = 3 << 40
    h = 1 << 35
    p12 = ph.perm_partial(a, kb, kb + 2 * h).cpu().tolist()
    p1 = ph.perm_partial(a, kb, kb + h).cpu().tolist()
    p2 = ph.perm_partial(a, kb + h, kb + 2 * h).cpu().tolist()
    v12 = complex(p12[0] + p12[1], p12[2] + p12[3])
    v = complex(p1[0] + p1[1], p1[2] + p1[3]) + complex(p2[0] + p2[1], p2[2] + p2[3])
    # the same chunks with the same rounding; only the reduction is grouped differently
    assert abs(v - v12) <= 1e-14 * abs(v12)


def test_segmented_run_resumes_to_the_same_bits(ph, tmp_path):
    from paper_1606_05836_amd.segments import segmented_perm

    n = 24
    a = cuda(I.haar1600_block(n))
    ref = segmented_perm(a, segment_log2=20)  # 8 segments, no checkpoint
    assert ref.done and ref.nseg_total == 8
    path = str(tmp_path / "n24.json")
    r = segmented_perm(a, segment_log2=20, checkpoint=path, max_segments=3)
    assert not r.done and r.next_segment == 3
    r = segmented_perm(a, segment_log2=20, checkpoint=path)  # a restart picks up segment 3
    assert r.done
    assert [[x.hex() for x in p] for p in r.partials] == [[x.hex() for x in p] for p in ref.partials]
    assert r.total() == ref.total()
    whole = complex(ph.perm(a).cpu())
    assert abs(r.total() - whole) <= 1e-15 * abs(whole)
    # shards of the same split give the same value
    from paper_1606_05836_amd.segments import combine_shards

    shards = [segmented_perm(a, segment_log2=20, shard=(g, 3)) for g in range(3)]
    assert combine_shards(shards) == ref.total()


@pytest.mark.parametrize("algo,n,c", [
    # one lane per term: n = 33 (the first size range with three resident
    # columns in batches), the n = 40 workload matrix itself, 41..44 (two
    # resident columns), with short and default (2^12) chunks
    ("glynn", 33, 6), ("glynn", 40, 6), ("glynn", 40, 0), ("glynn", 41, 6), ("glynn", 42, 6),
    ("glynn", 43, 6), ("glynn", 44, 6), ("glynn", 44, 0), ("ryser", 33, 6), ("ryser", 40, 6),
    ("ryser", 41, 6), ("ryser", 44, 6),
    # one lane per term with every step's column staged at n = 45..48, two
    # lanes per term from n = 49 (rows split in halves, odd n padded)
    ("glynn", 45, 6), ("glynn", 48, 6), ("glynn", 52, 6), ("ryser", 45, 6),
    ("ryser", 47, 6), ("ryser", 52, 6), ("glynn", 48, 0), ("glynn", 49, 6), ("glynn", 50, 0),
    # chunks of one and two blocks of 16 steps for every layout with a staged
    # update column: no block boundary in the chunk (the staged load goes
    # unused) and one boundary (staged, then the unused load after it)
    ("glynn", 26, 4), ("ryser", 30, 5), ("glynn", 36, 4), ("glynn", 36, 5), ("ryser", 38, 5),
    ("glynn", 42, 4), ("glynn", 43, 5), ("ryser", 44, 5), ("glynn", 47, 4), ("glynn", 47, 5),
    ("ryser", 50, 5)])
def test_large_n_haar_ranges_against_oracle(ph, algo, n, c):
    # the Haar blocks of the n = 40 / 44 workload recipe (and the same recipe
    # at the other orders): short ranges high in the index space, and the last
    # chunk, against the exact sums of Eq. (S2) / Eq. (S1) over the same terms
    a = I.haar1600_block(n)
    g, d = O.to_gaussian_integers(a)
    scale = Fraction(1, d ** n)
    cc = ph.perm_chunk_log2(n, algo, chunk_log2=c)
    L = 1 << cc
    total = ph.gray_terms(n, algo)
    k0 = (total // 3) // L * L + 5 * L
    nch = 3 if cc <= 6 else 1
    at = cuda(a)
    for kb, ke in ((k0, k0 + nch * L), (k0 + L, k0 + L), (total - L, total)):
        p = ph.perm_partial(at, kb, ke, algo=algo, chunk_log2=c).cpu().tolist()
        re, im = raw_exact(g, algo, kb, ke)
        e = complex(float(re * scale), float(im * scale))
        v = complex(p[0] + p[1], p[2] + p[3])
        if kb == ke:
            assert v == 0
        else:
            assert abs(v - e) <= 1e-12 * abs(e), (kb, ke, v, e)


@pytest.mark.parametrize("n", [45, 47, 49, 51])
def test_odd_large_n_shares_exact_on_diag_one_plus_i(ph, n):
    # odd orders: one lane per term up to 47; from 49 two lanes share a term
    # and the upper half is padded with a row whose sum stays 1
    a = cuda(I.diag_matrix(n, 1 + 1j))
    m = 1 << 30
    kb = (1 << (n - 3)) + (7 << 30)
    p = ph.perm_partial(a, kb, kb + m).cpu().tolist()
    want = m * (1 + 1j) * 2 ** ((n - 1) // 2) * 1j ** ((n - 1) // 2)
    assert complex(p[0] + p[1], p[2] + p[3]) == want


@pytest.mark.parametrize("n", [45, 46, 51])
def test_ryser_diag_full_set_term(ph, n):
    # Eq. (S1) on diag(d): only S = all columns contributes, (-1)^n prod d,
    # at the index whose Gray word has every bit set
    a = cuda(I.diag_matrix(n, 1 + 1j))
    k_all = 0
    for i in range(n):
        if (n - i) % 2:
            k_all |= 1 << i
    assert k_all ^ (k_all >> 1) == (1 << n) - 1
    L = 1 << ph.perm_chunk_log2(n, "ryser")
    kb = k_all // L * L
    p = ph.perm_partial(a, kb, kb + L, algo="ryser").cpu().tolist()
    want = (-1) ** n * (1 + 1j) ** (n % 2) * 2 ** (n // 2) * 1j ** (n // 2)
    assert complex(p[0] + p[1], p[2] + p[3]) == want
    p = ph.perm_partial(a, kb - 4 * L, kb, algo="ryser").cpu().tolist()
    assert p == [0.0, 0.0, 0.0, 0.0]


def test_command_line_runs_and_resumes(ph, tmp_path):
    import json
    import os
    import subprocess
    import sys

    n = 24
    a = I.haar1600_block(n)
    f = tmp_path / "a.npy"
    np.save(f, a)
    ck = tmp_path / "ck.json"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cmd = [sys.executable, "-m", "paper_1606_05836_amd.segments", str(f), "--segment-log2", "20",
           "--checkpoint", str(ck)]
    first = subprocess.run(cmd + ["--max-segments", "3"], cwd=root, capture_output=True, text=True, timeout=120)
    assert first.returncode == 0, first.stderr
    st = json.loads(first.stdout.strip().splitlines()[-1])
    assert not st["done"] and st["next_segment"] == 3
    second = subprocess.run(cmd, cwd=root, capture_output=True, text=True, timeout=120)
    assert second.returncode == 0, second.stderr
    lines = second.stdout.strip().splitlines()
    assert sum(1 for x in lines if x.startswith("segment ")) == 5  # only the missing segments ran
    out = json.loads(lines[-1])
    assert out["done"]
    per = complex(*out["permanent"])
    whole = complex(ph.perm(cuda(a)).cpu())
    assert abs(per - whole) <= 1e-15 * abs(whole)


@pytest.mark.parametrize("n", [1, 5, 16, 33, 44, 45, 49, 52])
@pytest.mark.parametrize("algo", ["glynn", "ryser"])
def test_strided_rows_match_contiguous(ph, n, algo):
    # every workgroup builds its table from A through lda: a view with row and
    # column offsets inside a 64 x 64 parent (lda = 64) must give the bits of
    # its contiguous copy, on the one-lane (n <= 48) and two-lane (n >= 49) sweeps
    u = cuda(I.haar(64, 7))
    view = u[3:3 + n, 5:5 + n]
    assert view.stride(0) == 64
    dense = view.contiguous()
    L = 1 << ph.perm_chunk_log2(n, algo)
    total = ph.gray_terms(n, algo)
    kb = min(total // 3 // L * L, max(0, total - 64 * L))
    ke = min(total, kb + 64 * L)
    assert torch.equal(ph.perm_partial(view, kb, ke, algo=algo), ph.perm_partial(dense, kb, ke, algo=algo))
    if n <= 16:
        assert torch.equal(ph.perm(view, algo=algo), ph.perm(dense, algo=algo))
    if n <= 5:
        assert O.rel_err(complex(ph.perm(view, algo=algo).cpu()), O.perm_exact(view.cpu().numpy())) <= 1e-12


@pytest.mark.parametrize("algo", ["glynn", "ryser"])
def test_longest_chunk_exact(ph, algo):
    # the largest chunk length any call takes (PH_CHUNK_LOG2_MAX = 24; longer
    # requests are clamped to it): n = 26 on D(P + Q), whose every term is an
    # exact integer, in 2 (BB/FG) or 4 (Ryser) chunks of 2^24 terms
    from tests._closed_forms import two_permutations

    a, want = two_permutations(26, 2626)
    assert ph.perm_chunk_log2(26, algo, chunk_log2=40) == ph.PH_CHUNK_LOG2_MAX == 24
    got = complex(ph.perm(cuda(a), algo=algo, chunk_log2=40).cpu())
    assert got == want


@pytest.mark.parametrize("n", [46, 50])
def test_longest_chunk_large_n_exact(ph, n):
    # the longest chunk on the one-lane sweep with every column staged
    # (n = 46) and on the two-lane sweep (n = 50): two chunks of 2^24 terms of
    # diag(1+i), high in the index space; every term is (1+i)^n = 2^(n/2) i^(n/2)
    a = cuda(I.diag_matrix(n, 1 + 1j))
    L = 1 << 24
    kb = (1 << (n - 2)) + 5 * L
    p = ph.perm_partial(a, kb, kb + 2 * L, chunk_log2=24).cpu().tolist()
    assert complex(p[0] + p[1], p[2] + p[3]) == 2 * L * 2 ** (n // 2) * 1j ** (n // 2)
