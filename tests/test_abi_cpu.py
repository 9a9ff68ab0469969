"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "permhip.h")


@pytest.fixture(scope="module")
def L():
    from paper_1606_05836_amd import permhip as P

    if not os.path.exists(P.LIB_PATH):
        from paper_1606_05836_amd.build import build

        build()
    return P.lib()


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(ph_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for want in ("ph_perm", "ph_perm_batched", "ph_plan_create", "ph_plan_execute", "ph_plan_destroy",
                 "ph_perm_grad", "ph_boson_probs", "ph_boson_probs_grad", "ph_last_error", "ph_version"):
        assert want in names


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_binding_lists_match_header():
    from paper_1606_05836_amd import permhip as P

    assert sorted(P.EXPORTS) == declared_functions()


def test_version(L):
    assert L.ph_version() >= 10000


def _perm(L, a, n, lda, out, o=None):
    from paper_1606_05836_amd import permhip as P

    return L.ph_perm(ctypes.c_void_p(a), n, lda, ctypes.c_void_p(out), ctypes.byref(o) if o else None, None)


def test_argument_errors_are_reported_before_any_device_work(L):
    from paper_1606_05836_amd import permhip as P

    fake = 0x1000  # never dereferenced: validation fails first
    assert _perm(L, fake, -1, 1, fake) == P.PH_EINVAL
    assert b"n=-1" in L.ph_last_error()
    assert _perm(L, fake, P.PH_NMAX + 1, 64, fake) == P.PH_ERANGE
    assert _perm(L, fake, 10, 9, fake) == P.PH_EINVAL
    assert _perm(L, fake, 10, 10, 0) == P.PH_EINVAL
    assert _perm(L, 0, 10, 10, fake) == P.PH_EINVAL
    assert _perm(L, fake, 10, 10, fake, P.PhOpts(7, 0, 0, 0, 0)) == P.PH_EINVAL
    assert _perm(L, fake, 10, 10, fake, P.PhOpts(0, 5, 0, 0, 0)) == P.PH_EINVAL
    assert _perm(L, fake, 10, 10, fake, P.PhOpts(0, 0, 0, 9, 0)) == P.PH_EINVAL
    assert _perm(L, fake, 10, 10, fake, P.PhOpts(0, 0, 0, 0, 8)) == P.PH_EINVAL  # unknown flag bit
    assert _perm(L, fake, 10, 10, fake, P.PhOpts(0, 0, -1, 0, 0)) == P.PH_EINVAL  # negative chunk_log2


def test_paired_ryser_argument_errors_before_any_device_work(L):
    from paper_1606_05836_amd import permhip as P

    fake = 0x1000  # never dereferenced: validation fails first

    def paired(a, n, lda, out, o=None):
        return L.ph_perm_ryser_paired(ctypes.c_void_p(a), n, lda, ctypes.c_void_p(out),
                                      ctypes.byref(o) if o else None, None)

    assert paired(fake, -1, 1, fake) == P.PH_EINVAL
    assert paired(fake, 33, 64, fake) == P.PH_ERANGE
    assert b"n=33" in L.ph_last_error()
    assert paired(fake, 10, 9, fake) == P.PH_EINVAL
    assert paired(fake, 10, 10, 0) == P.PH_EINVAL
    assert paired(0, 10, 10, fake) == P.PH_EINVAL
    assert paired(fake, 10, 10, fake, P.PhOpts(1, 5, 0, 0, 0)) == P.PH_EINVAL


def test_python_binding_rejects_non_device_tensors():
    import torch

    import paper_1606_05836_amd as ph

    with pytest.raises(TypeError):
        ph.perm(torch.zeros((3, 3), dtype=torch.complex128))
    with pytest.raises(TypeError):
        ph.perm(torch.zeros((3, 3), dtype=torch.float64))


def test_boson_argument_errors_are_reported_before_any_device_work(L):
    from paper_1606_05836_amd import permhip as P

    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    I32 = ctypes.c_int32

    def probs(m, ldu, ins, pats, npat, out=fake, u=fake):
        n = len(ins)
        a = (I32 * max(1, n))(*ins)
        p = (I32 * max(1, len(pats)))(*pats)
        return L.ph_boson_probs(u, m, ldu, a, n, p, npat, out, None, None)

    def grad(m, ins, pats, npat, lddu, du=fake, o=None):
        n = len(ins)
        a = (I32 * max(1, n))(*ins)
        p = (I32 * max(1, len(pats)))(*pats)
        return L.ph_boson_probs_grad(fake, m, m, a, n, p, npat, None, None, du, lddu,
                                     ctypes.byref(o) if o else None, None)

    assert probs(4, 4, [0, 5], [0, 1], 1) == P.PH_EINVAL  # input mode >= m
    assert b"in_modes[1]=5" in L.ph_last_error()
    assert probs(4, 4, [0, 1], [0, -1], 1) == P.PH_EINVAL  # output mode < 0
    assert probs(4, 3, [0, 1], [0, 1], 1) == P.PH_EINVAL  # ldu < m
    assert probs(0, 4, [], [], 0) == P.PH_EINVAL  # m < 1
    assert probs(4, 4, [0, 1], [0, 1], -1) == P.PH_EINVAL
    assert probs(4, 4, [0, 1], [0, 1], 1, out=None) == P.PH_EINVAL
    assert probs(4, 4, [0, 1], [0, 1], 1, u=None) == P.PH_EINVAL
    big = list(range(P.PH_NMAX + 1))
    assert probs(64, 64, big, big, 1) == P.PH_ERANGE
    g = list(range(P.PH_NMAX_GRAD + 1))
    assert grad(64, g, g, 1, 64) == P.PH_ERANGE
    assert grad(4, [0, 1], [0, 1], 1, 1) == P.PH_EINVAL  # lddu < n
    full = P.PhOpts(0, 0, 0, 0, P.PH_FLAG_DU_FULL)
    assert grad(4, [0, 1], [0, 1], 1, 3, o=full) == P.PH_EINVAL  # the m x m form needs lddu >= m
    assert b"lddu=3 < 4" in L.ph_last_error()
    assert grad(4, [0, 1], [0, 1], 1, 2, du=None) == P.PH_EINVAL
    assert grad(4, [], [], 0, 1) == P.PH_EINVAL  # the gradient needs n >= 1
    assert grad(4, [0, 1], [0, 1], 1, 2, o=P.PhOpts(P.PH_RYSER, 0, 0, 0, 0)) == P.PH_EINVAL
    assert b"PH_GLYNN" in L.ph_last_error()


def test_chunk_length_query(L):
    from paper_1606_05836_amd import permhip as P

    # default: 2^min(12, nb - 17) terms per chunk, at least 2^4 (2^1 for nb < 4), at most the whole sum
    assert P.perm_chunk_log2(40) == 12
    assert P.perm_chunk_log2(29) == 11  # 2^(28 - 11) = 2^17 chunks
    assert P.perm_chunk_log2(26) == 8
    assert P.perm_chunk_log2(26, "ryser") == 9
    assert P.perm_chunk_log2(20) == 4  # the shortest chunk the sweeps take
    assert P.perm_chunk_log2(3) == 1
    assert P.perm_chunk_log2(1) == 0
    assert P.perm_chunk_log2(1, "ryser") == 1
    assert P.perm_chunk_log2(30, chunk_log2=9) == 9
    assert P.perm_chunk_log2(8, chunk_log2=40) == 7  # clamped to the 2^7 terms
    # never above PH_CHUNK_LOG2_MAX, whatever the order and the request
    assert P.perm_chunk_log2(50, chunk_log2=40) == P.PH_CHUNK_LOG2_MAX == 24
    assert P.perm_chunk_log2(48, "ryser", chunk_log2=2**31 - 1) == P.PH_CHUNK_LOG2_MAX
    assert P.perm_chunk_log2(26, chunk_log2=25) == P.PH_CHUNK_LOG2_MAX  # 2^25 terms, chunks of at most 2^24
    assert P.perm_chunk_log2(20, chunk_log2=24) == 19  # the whole range
    assert P.gray_terms(40) == 1 << 39 and P.gray_terms(40, "ryser") == 1 << 40
    c = ctypes.c_int32(0)
    assert L.ph_perm_chunk_log2(0, None, ctypes.byref(c)) == P.PH_EINVAL
    assert L.ph_perm_chunk_log2(P.PH_NMAX + 1, None, ctypes.byref(c)) == P.PH_ERANGE
    assert L.ph_perm_chunk_log2(10, None, None) == P.PH_EINVAL


def test_partial_and_combine_argument_errors(L):
    from paper_1606_05836_amd import permhip as P

    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first

    def part(n, kb, ke, lda=None, a=fake, out=fake, o=None):
        return L.ph_perm_partial(a, n, n if lda is None else lda, kb, ke, out, ctypes.byref(o) if o else None, None)

    L16 = 1 << 12  # n = 40: chunks of 2^12 terms
    assert part(0, 0, 0) == P.PH_EINVAL
    assert part(P.PH_NMAX + 1, 0, 0) == P.PH_ERANGE
    assert part(40, 0, L16, a=None) == P.PH_EINVAL
    assert part(40, 0, L16, out=None) == P.PH_EINVAL
    assert part(40, 0, L16, lda=39) == P.PH_EINVAL
    assert part(40, L16, 0) == P.PH_EINVAL  # begin > end
    assert part(40, 0, (1 << 39) + L16) == P.PH_EINVAL  # past the 2^39 terms
    assert b"outside" in L.ph_last_error()
    assert part(40, 1, L16) == P.PH_EINVAL  # not a chunk boundary
    assert b"aligned" in L.ph_last_error()
    assert part(40, 0, L16 + 8) == P.PH_EINVAL
    assert part(40, 0, 1 << 12, o=P.PhOpts(0, 0, 13, 0, 0)) == P.PH_EINVAL  # 2^12 is not a 2^13 multiple
    assert part(40, 0, L16, o=P.PhOpts(3, 0, 0, 0, 0)) == P.PH_EINVAL

    def comb(parts, count, n, out=fake):
        return L.ph_perm_combine(parts, count, n, out, None, None)

    assert comb(fake, 1, 0) == P.PH_EINVAL
    assert comb(fake, 1, P.PH_NMAX + 1) == P.PH_ERANGE
    assert comb(fake, -1, 10) == P.PH_EINVAL
    assert comb(None, 2, 10) == P.PH_EINVAL
    assert comb(fake, 1, 10, out=None) == P.PH_EINVAL


def test_sampler_argument_errors_are_reported_before_any_device_work(L):
    import numpy as np

    from paper_1606_05836_amd import permhip as P

    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    I32, F64 = ctypes.c_int32, ctypes.c_double

    def sample(m, ins, perms, unis, ns=None, o=None, ldu=None, out=fake):
        n = len(ins)
        a = (I32 * max(1, n))(*ins)
        pp = np.ascontiguousarray(np.asarray(perms, dtype=np.int32).reshape(-1))
        uu = np.ascontiguousarray(np.asarray(unis, dtype=np.float64).reshape(-1))
        ns = len(pp) // max(1, n) if ns is None else ns
        return L.ph_boson_sample(fake, m, m if ldu is None else ldu, a, n, ns,
                                 pp.ctypes.data_as(ctypes.POINTER(I32)), uu.ctypes.data_as(ctypes.POINTER(F64)),
                                 out, ctypes.byref(o) if o else None, None)

    ok_p, ok_u = [[0, 1], [1, 0]], [[0.1, 0.9], [0.0, 0.5]]
    assert sample(4, [0, 0], ok_p, ok_u) == P.PH_EINVAL  # repeated input mode
    assert b"repeats" in L.ph_last_error()
    assert sample(4, [0, 4], ok_p, ok_u) == P.PH_EINVAL  # input mode >= m
    assert sample(4, [0, 1], [[0, 0], [1, 0]], ok_u) == P.PH_EINVAL  # not a permutation
    assert b"permutation" in L.ph_last_error()
    assert sample(4, [0, 1], [[0, 2], [1, 0]], ok_u) == P.PH_EINVAL
    assert sample(4, [0, 1], ok_p, [[0.1, 1.0], [0.0, 0.5]]) == P.PH_EINVAL  # uniform not below 1
    assert sample(4, [0, 1], ok_p, [[0.1, float("nan")], [0.0, 0.5]]) == P.PH_EINVAL
    assert sample(4, [0, 1], ok_p, [[-0.1, 0.2], [0.0, 0.5]]) == P.PH_EINVAL
    assert sample(4, [0, 1], ok_p, ok_u, ldu=3) == P.PH_EINVAL
    assert sample(4, [0, 1], ok_p, ok_u, ns=-1) == P.PH_EINVAL
    assert sample(4, [0, 1], ok_p, ok_u, out=None) == P.PH_EINVAL
    assert sample(4, [], [], []) == P.PH_EINVAL  # n >= 1
    big = list(range(P.PH_NMAX_GRAD + 1))
    assert sample(64, big, [big], [[0.5] * len(big)]) == P.PH_ERANGE
    assert sample(4, [0, 1], ok_p, ok_u, o=P.PhOpts(P.PH_RYSER, 0, 0, 0, 0)) == P.PH_EINVAL
    assert sample(4, [0, 1], ok_p, ok_u, ns=0) == P.PH_OK  # nothing to draw, nothing enqueued


def test_accumulation_default_from_the_environment(L, monkeypatch):
    import ctypes as C

    from paper_1606_05836_amd import permhip as P

    c = C.c_int32(0)
    for v in ("dd", "plain", ""):
        monkeypatch.setenv("PERMHIP_ACCUM", v)
        assert L.ph_perm_chunk_log2(20, None, C.byref(c)) == P.PH_OK
    monkeypatch.setenv("PERMHIP_ACCUM", "quad")
    assert L.ph_perm_chunk_log2(20, None, C.byref(c)) == P.PH_EINVAL
    assert b"PERMHIP_ACCUM" in L.ph_last_error()
    # explicit options do not read it
    o = P.PhOpts(0, 0, 0, 0, 0)
    assert L.ph_perm_chunk_log2(20, C.byref(o), C.byref(c)) == P.PH_OK


def test_trace_ranges_switch_on_without_side_effects(L):
    # PERMHIP_ROCTX=1 loads libroctx64 on the first traced call; the calls still
    # validate and fail as before (read once per process, hence a subprocess)
    import subprocess
    import sys

    code = (
        "import ctypes, sys\n"
        "sys.path.insert(0, %r)\n"
        "from paper_1606_05836_amd import permhip as P\n"
        "L = P.lib()\n"
        "assert L.ph_perm(ctypes.c_void_p(0x1000), -1, 1, ctypes.c_void_p(0x1000), None, None) == P.PH_EINVAL\n"
        "assert L.ph_perm_combine(None, -1, 10, ctypes.c_void_p(0x1000), None, None) == P.PH_EINVAL\n"
        "print('ok')\n" % ROOT
    )
    env = dict(os.environ, PERMHIP_ROCTX="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr


def test_header_constants_match_the_binding():
    from paper_1606_05836_amd import permhip as P

    txt = open(HEADER).read()
    defs = dict(re.findall(r"^#define (PH_\w+) (\d+)u?", txt, re.M))
    for name in ("PH_NMAX", "PH_NMAX_GRAD", "PH_CHUNK_LOG2_MAX", "PH_FLAG_UNGROUPED", "PH_FLAG_UNSORTED",
                 "PH_FLAG_DU_FULL"):
        assert int(defs[name]) == getattr(P, name), name


def test_binding_rejects_mismatched_buffers_before_the_call():
    # the C ABI cannot see device buffer sizes, so the binding checks them
    import torch

    from paper_1606_05836_amd import permhip as P

    with pytest.raises(ValueError, match="n x n"):
        P._pack([torch.zeros(3, 3, dtype=torch.complex128), torch.zeros(2, 3, dtype=torch.complex128)])
    with pytest.raises(ValueError, match="n x n"):
        P._pack([torch.zeros(4, dtype=torch.complex128)])
    with pytest.raises(TypeError, match="CUDA"):
        P._need_out("out", torch.zeros(1, dtype=torch.complex128), torch.complex128, 1, torch.device("cpu"))
    with pytest.raises(TypeError, match="complex128"):
        P._need_out("out", torch.zeros(1, dtype=torch.float64), torch.complex128, 1, torch.device("cpu"))


def test_shared_options_match_fresh_ones(L):
    # the small-call paths reuse one options struct per distinct argument
    # tuple; its fields must be those opts() builds, and the chunk-length
    # query must read the same values through either
    from paper_1606_05836_amd import permhip as P

    fields = [f for f, _ in P.PhOpts._fields_]
    for args in (("glynn", "dd", 0, 0), ("ryser", "plain", 7, 2), (P.PH_RYSER, P.PH_ACC_DD, 40, 0),
                 ("glynn", "plain", 0, 0, P.PH_FLAG_UNGROUPED)):
        a = P._opts_shared(*args)
        assert a is P._opts_shared(*args)
        b = P.opts(*args)
        assert [getattr(a, f) for f in fields] == [getattr(b, f) for f in fields], args
        ca, cb = ctypes.c_int32(0), ctypes.c_int32(0)
        assert L.ph_perm_chunk_log2(44, a, ctypes.byref(ca)) == 0
        assert L.ph_perm_chunk_log2(44, ctypes.byref(b), ctypes.byref(cb)) == 0
        assert ca.value == cb.value, args
    assert P._opts_shared("glynn", "dd") is not P._opts_shared("glynn", "plain")


def test_missing_library_fails_loudly(monkeypatch):
    # no CPU fallback: without libpermhip.so the binding raises instead of
    # computing anything elsewhere
    from paper_1606_05836_amd import permhip as P

    monkeypatch.setattr(P, "_lib", None)
    monkeypatch.setattr(P, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libpermhip.so"))
    with pytest.raises(RuntimeError, match="missing"):
        P.lib()
