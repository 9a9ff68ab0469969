"""ph_perm_noalloc (the one-matrix permanent without device allocation)
against ph_perm, through the C ABI: the same kernels and launch shape, so the
same bits, call after call (the second call smaller than the first, so that
the static scratch keeps stale partial sums from the first)."""
import ctypes

import numpy as np
import pytest

import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_1606_05836_amd import permhip as P

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P


def c_abi(P, fn, a, out, o):
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    n = a.shape[0]
    lda = a.stride(0) if n > 0 else 1
    P.check(getattr(P.lib(), fn)(ctypes.c_void_p(a.data_ptr()), n, lda, ctypes.c_void_p(out.data_ptr()),
                                 ctypes.byref(o), st))


@pytest.mark.parametrize("algo,accum", [("glynn", "dd"), ("ryser", "plain")])
def test_noalloc_matches_perm_call_after_call(P, algo, accum):
    o = P.opts(algo, accum)
    u = torch.from_numpy(I.haar(1600, 31)).to("cuda")
    for n in (30, 20, 12, 0, 26):  # each after a larger one, bar the last
        a = u[:n, :n]  # a strided view (lda 1600), read in place
        want = torch.empty((), dtype=torch.complex128, device="cuda")
        got = torch.full((), complex("nan"), dtype=torch.complex128, device="cuda")
        c_abi(P, "ph_perm", a, want, o)
        c_abi(P, "ph_perm_noalloc", a, got, o)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (n, complex(got.cpu()), complex(want.cpu()))
    # two calls in a row on the same stream with nothing in between
    a1, a2 = u[40:64, 40:64], u[100:110, 100:110]
    w1, w2, g1, g2 = (torch.empty((), dtype=torch.complex128, device="cuda") for _ in range(4))
    c_abi(P, "ph_perm", a1, w1, o)
    c_abi(P, "ph_perm", a2, w2, o)
    c_abi(P, "ph_perm_noalloc", a1, g1, o)
    c_abi(P, "ph_perm_noalloc", a2, g2, o)
    torch.cuda.synchronize()
    assert torch.equal(g1, w1) and torch.equal(g2, w2)


def test_noalloc_integer_bit_exact_and_errors(P):
    import oracle as O

    b = torch.from_numpy(I.int12_matrix()).to("cuda")
    out = torch.empty((), dtype=torch.complex128, device="cuda")
    P.perm_noalloc(b, out)
    assert complex(out.cpu()) == O.to_complex(O.perm_exact(I.int12_matrix()))
    # argument errors come back before anything is enqueued
    L = P.lib()
    fake = ctypes.c_void_p(0x1000)
    assert L.ph_perm_noalloc(fake, P.PH_NMAX + 1, 64, fake, None, None) == P.PH_ERANGE
    assert L.ph_perm_noalloc(fake, 10, 9, fake, None, None) == P.PH_EINVAL
    assert L.ph_perm_noalloc(fake, 10, 10, None, None, None) == P.PH_EINVAL
    with pytest.raises(ValueError, match="contiguous"):
        P.perm_noalloc(b.t(), out)
