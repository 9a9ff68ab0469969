"""ctypes binding of libpermhip.so (the C ABI in include/permhip.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Torch tensors supply device memory and the current stream.  If the
shared library is missing the calls raise instead of falling back to anything
else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpermhip.so")

PH_GLYNN, PH_RYSER = 0, 1
PH_ACC_DD, PH_ACC_PLAIN = 0, 1
PH_OK, PH_EINVAL, PH_ERANGE, PH_ENOMEM, PH_EHIP, PH_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
PH_NMAX, PH_NMAX_GRAD = 52, 32
PH_CHUNK_LOG2_MAX = 24
PH_FLAG_UNGROUPED = 1
PH_FLAG_UNSORTED = 2
PH_FLAG_DU_FULL = 4

EXPORTS = ("ph_perm", "ph_perm_noalloc", "ph_perm_ryser_paired", "ph_perm_chunk_log2", "ph_perm_partial", "ph_perm_combine", "ph_perm_batched", "ph_plan_create", "ph_plan_execute", "ph_plan_destroy", "ph_plan_shape",
           "ph_perm_grad", "ph_perm_row_minors", "ph_boson_probs", "ph_boson_probs_grad", "ph_boson_sample", "ph_fp64_peak", "ph_last_error",
           "ph_version")


class PhOpts(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("accum", ctypes.c_int32), ("chunk_log2", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class PermhipError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"permhip error {code}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load libpermhip.so once and declare the signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1606_05836_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    op = ctypes.POINTER(PhOpts)
    P = ctypes.POINTER
    L.ph_perm.argtypes = [vp, i32, i64, vp, op, vp]
    L.ph_perm_noalloc.argtypes = [vp, i32, i64, vp, op, vp]
    L.ph_perm_ryser_paired.argtypes = [vp, i32, i64, vp, op, vp]
    L.ph_perm_chunk_log2.argtypes = [i32, op, P(ctypes.c_int32)]
    L.ph_perm_partial.argtypes = [vp, i32, i64, ctypes.c_uint64, ctypes.c_uint64, vp, op, vp]
    L.ph_perm_combine.argtypes = [vp, i64, i32, vp, op, vp]
    L.ph_perm_batched.argtypes = [vp, P(ctypes.c_int64), P(ctypes.c_int32), i64, vp, op, vp]
    L.ph_plan_create.argtypes = [P(ctypes.c_int32), P(ctypes.c_int64), i64, op, vp, P(ctypes.c_void_p)]
    L.ph_plan_execute.argtypes = [vp, vp, vp, vp]
    L.ph_plan_destroy.argtypes = [vp]
    L.ph_plan_shape.argtypes = [vp, i32, P(ctypes.c_int32), P(ctypes.c_int32)]
    L.ph_perm_grad.argtypes = [vp, i32, i64, vp, vp, vp, op, vp]
    L.ph_boson_probs.argtypes = [vp, i32, i64, P(ctypes.c_int32), i32, P(ctypes.c_int32), i64, dp, op, vp]
    L.ph_boson_probs_grad.argtypes = [vp, i32, i64, P(ctypes.c_int32), i32, P(ctypes.c_int32), i64, dp, dp, vp,
                                      i64, op, vp]
    L.ph_perm_row_minors.argtypes = [vp, i32, i64, vp, op, vp]
    L.ph_boson_sample.argtypes = [vp, i32, i64, P(ctypes.c_int32), i32, i64, P(ctypes.c_int32), P(ctypes.c_double),
                                  vp, op, vp]
    L.ph_fp64_peak.argtypes = [i64, P(ctypes.c_double), P(ctypes.c_double), vp]
    L.ph_last_error.restype = ctypes.c_char_p
    L.ph_last_error.argtypes = []
    L.ph_version.restype = ctypes.c_int
    L.ph_version.argtypes = []
    for name in EXPORTS:
        if name not in ("ph_last_error", "ph_version"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != PH_OK:
        raise PermhipError(rc, lib().ph_last_error().decode())


def opts(algo: str | int = "glynn", accum: str | int = "dd", chunk_log2: int = 0, waves: int = 0,
         flags: int = 0) -> PhOpts:
    a = {"glynn": PH_GLYNN, "ryser": PH_RYSER}.get(algo, algo)
    c = {"dd": PH_ACC_DD, "plain": PH_ACC_PLAIN}.get(accum, accum)
    return PhOpts(int(a), int(c), int(chunk_log2), int(waves), int(flags))


_OPTS: dict = {}


def _opts_shared(algo="glynn", accum="dd", chunk_log2: int = 0, waves: int = 0, flags: int = 0) -> PhOpts:
    """opts() for the calls below, built once per distinct argument tuple: the
    library only reads the struct (a const ph_opts*), so one instance serves
    every call with the same options and a small call skips building it."""
    key = (algo, accum, chunk_log2, waves, flags)
    o = _OPTS.get(key)
    if o is None:
        o = opts(algo, accum, chunk_log2, waves, flags)
        if len(_OPTS) < 1024:
            _OPTS[key] = o
    return o


_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream_of(dev: torch.device) -> int:
    """Handle of the current stream on `dev`, as an integer for a void*
    argument (without building a torch.cuda.Stream object per call)."""
    if _raw_stream is not None:
        return _raw_stream(dev.index)
    return torch.cuda.current_stream(dev).cuda_stream


def _stream(t: torch.Tensor) -> int:
    return _stream_of(t.device)


def _ptr(t: torch.Tensor | None):
    """Device address for a void* argument (None passes NULL)."""
    return t.data_ptr() if t is not None else None


def _need_c128_cuda(name: str, t: torch.Tensor):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")


def _need_out(name: str, out: torch.Tensor, dtype: torch.dtype, numel: int, device: torch.device):
    """The library writes `numel` elements of `dtype` at out's address: reject
    anything else before the call (the C ABI cannot see device sizes)."""
    if not isinstance(out, torch.Tensor) or out.dtype != dtype or not out.is_cuda:
        raise TypeError(f"{name} must be a {dtype} CUDA tensor")
    if out.device != device:
        raise ValueError(f"{name} is on {out.device}, the input on {device}")
    if out.numel() != numel or not out.is_contiguous():
        raise ValueError(f"{name} must be contiguous with {numel} elements")


def perm(a: torch.Tensor, algo="glynn", accum="dd", chunk_log2: int = 0, waves: int = 0,
         out: torch.Tensor | None = None) -> torch.Tensor:
    """Per(a) for an n x n complex128 matrix on the GPU (rows may be strided):
    a 0-dim complex128 tensor.  For a (..., n, n) tensor the permanents of all
    matrices go through ph_perm_batched and come back with shape (...)."""
    _need_c128_cuda("a", a)
    shape = a.shape
    if len(shape) < 2 or shape[-1] != shape[-2]:
        raise ValueError("a must be (..., n, n)")
    if len(shape) > 2:
        if out is not None:
            raise ValueError("out is supported for a single matrix only")
        lead, n = shape[:-2], shape[-1]
        flat = a.reshape(-1, n, n)
        res = perm_batched(flat, algo, accum, chunk_log2, waves) if flat.shape[0] else \
            torch.empty(0, dtype=torch.complex128, device=a.device)
        return res.reshape(lead)
    n = shape[0]
    lda = 1
    if n > 0:
        lda, s1 = a.stride()
        if s1 != 1:
            a = a.contiguous()
            lda = n
    dev = a.device
    if out is None:
        out = torch.empty((), dtype=torch.complex128, device=dev)
    else:
        _need_out("out", out, torch.complex128, 1, dev)
    check(lib().ph_perm(a.data_ptr(), n, lda, out.data_ptr(), _opts_shared(algo, accum, chunk_log2, waves),
                        _stream_of(dev)))
    return out


def perm_noalloc(a: torch.Tensor, out: torch.Tensor, algo="glynn", accum="dd", chunk_log2: int = 0,
                 waves: int = 0) -> torch.Tensor:
    """Per(a) into the caller's 0-dim complex128 `out` through ph_perm_noalloc:
    the library allocates nothing (its partial sums live in a static device
    array shared by all calls on the device).  a: n x n, rows may be strided."""
    _need_c128_cuda("a", a)
    if a.dim() != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("a must be n x n")
    _need_out("out", out, torch.complex128, 1, a.device)
    n = a.shape[0]
    if n > 0 and a.stride(1) != 1:
        raise ValueError("a's rows must be contiguous (stride(1) == 1): no copy is made here")
    o = _opts_shared(algo, accum, chunk_log2, waves)
    check(lib().ph_perm_noalloc(_ptr(a), n, a.stride(0) if n > 0 else 1, _ptr(out), ctypes.byref(o), _stream(a)))
    return out


def perm_ryser_paired(a: torch.Tensor, accum="dd", chunk_log2: int = 0,
                      out: torch.Tensor | None = None) -> torch.Tensor:
    """Per(a) for an n x n complex128 matrix (n <= 32, rows may be strided) by
    Ryser's formula with the complement pairing of Algorithm S3
    (ph_perm_ryser_paired): a 0-dim complex128 tensor."""
    _need_c128_cuda("a", a)
    if a.dim() != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("a must be n x n")
    n = a.shape[0]
    if n > 0 and a.stride(1) != 1:
        a = a.contiguous()
    if out is None:
        out = torch.empty((), dtype=torch.complex128, device=a.device)
    else:
        _need_out("out", out, torch.complex128, 1, a.device)
    o = _opts_shared("ryser", accum, chunk_log2)
    check(lib().ph_perm_ryser_paired(_ptr(a), n, a.stride(0) if n > 0 else 1, _ptr(out), ctypes.byref(o),
                                     _stream(a)))
    return out


def perm_chunk_log2(n: int, algo="glynn", accum="dd", chunk_log2: int = 0) -> int:
    """log2 of the chunk length ph_perm / ph_perm_partial use for n; term
    ranges given to perm_partial are multiples of 2**this."""
    c = ctypes.c_int32(0)
    o = opts(algo, accum, chunk_log2)
    check(lib().ph_perm_chunk_log2(int(n), ctypes.byref(o), ctypes.byref(c)))
    return int(c.value)


def gray_terms(n: int, algo="glynn") -> int:
    """Number of terms of the Gray-code sum: 2^(n-1) (BB/FG) or 2^n (Ryser)."""
    return 1 << (n - 1 if opts(algo).algo == PH_GLYNN else n)


def perm_partial(a: torch.Tensor, k_begin: int, k_end: int, algo="glynn", accum="dd", chunk_log2: int = 0,
                 waves: int = 0, out: torch.Tensor | None = None) -> torch.Tensor:
    """Unscaled signed sum of the terms k in [k_begin, k_end) of Per(a)'s
    Gray-code sum (ph_perm_partial): a float64 CUDA tensor of 4 values
    {re_hi, re_lo, im_hi, im_lo}."""
    _need_c128_cuda("a", a)
    if a.dim() != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("a must be n x n")
    n = a.shape[0]
    if n > 0 and a.stride(1) != 1:
        a = a.contiguous()
    if out is None:
        out = torch.empty(4, dtype=torch.float64, device=a.device)
    else:
        _need_out("out", out, torch.float64, 4, a.device)
    o = _opts_shared(algo, accum, chunk_log2, waves)
    check(lib().ph_perm_partial(_ptr(a), n, a.stride(0) if n > 0 else 1, int(k_begin), int(k_end), _ptr(out),
                                ctypes.byref(o), _stream(a)))
    return out


def perm_combine(partials: torch.Tensor, n: int, algo="glynn", accum="dd",
                 out: torch.Tensor | None = None) -> torch.Tensor:
    """Per from partials (a (count, 4) float64 CUDA tensor, summed in row
    order) made by perm_partial with the same n, algo and accum."""
    if partials.dtype != torch.float64 or not partials.is_cuda or partials.shape[-1] != 4:
        raise TypeError("partials must be a (count, 4) float64 CUDA tensor")
    partials = partials.reshape(-1, 4).contiguous()
    if out is None:
        out = torch.empty((), dtype=torch.complex128, device=partials.device)
    else:
        _need_out("out", out, torch.complex128, 1, partials.device)
    o = opts(algo, accum)
    check(lib().ph_perm_combine(_ptr(partials), partials.shape[0], int(n), _ptr(out), ctypes.byref(o),
                                _stream(partials)))
    return out


def _pack(mats: Sequence[torch.Tensor]):
    for m in mats:
        if m.dim() != 2 or m.shape[0] != m.shape[1]:
            raise ValueError(f"every matrix must be n x n, got shape {tuple(m.shape)}")
    ns = [int(m.shape[0]) for m in mats]
    flat = torch.cat([m.reshape(-1) for m in mats]) if mats else None
    return ns, flat


class Plan:
    """A batched-permanent plan (ph_plan_create / execute / destroy)."""

    def __init__(self, ns: Sequence[int], offsets: Sequence[int] | None = None, algo="glynn", accum="dd",
                 chunk_log2: int = 0, waves: int = 0, device=None):
        self.ns = [int(x) for x in ns]
        self.batch = len(self.ns)
        dev = torch.device(device or "cuda")
        self.device = dev if dev.index is not None else torch.device("cuda", torch.cuda.current_device())
        self._n = (ctypes.c_int32 * max(1, self.batch))(*self.ns)
        self._off = None
        # elements the plan reads from a_packed: the end of the last matrix
        if offsets is not None:
            offs = [int(x) for x in offsets]
            if len(offs) != self.batch:
                raise ValueError("offsets needs one entry per matrix")
            self._off = (ctypes.c_int64 * max(1, self.batch))(*offs)
            self.elems = max((o + n * n for o, n in zip(offs, self.ns)), default=0)
        else:
            self.elems = sum(n * n for n in self.ns)
        self._opts = opts(algo, accum, chunk_log2, waves)
        h = ctypes.c_void_p(0)
        with torch.cuda.device(self.device):
            st = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
            check(lib().ph_plan_create(self._n, self._off, self.batch, ctypes.byref(self._opts), st,
                                       ctypes.byref(h)))
        self._h = h

    def __call__(self, a_packed: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        _need_c128_cuda("a_packed", a_packed)
        if not a_packed.is_contiguous():
            raise ValueError("a_packed must be contiguous")
        if a_packed.device != self.device:
            raise ValueError(f"a_packed is on {a_packed.device}, the plan on {self.device}")
        if a_packed.numel() < self.elems:
            raise ValueError(f"a_packed holds {a_packed.numel()} elements, the plan reads {self.elems}")
        if out is None:
            out = torch.empty(self.batch, dtype=torch.complex128, device=a_packed.device)
        else:
            _need_out("out", out, torch.complex128, self.batch, a_packed.device)
        check(lib().ph_plan_execute(self._h, _ptr(a_packed), _ptr(out), _stream(a_packed)))
        return out

    def shape(self, n: int):
        """(log2 chunk length, waves per SIMD; 0 = as many as fit) the plan
        sweeps its order-n matrices with (ph_plan_shape)."""
        c, w = ctypes.c_int32(0), ctypes.c_int32(0)
        check(lib().ph_plan_shape(self._h, int(n), ctypes.byref(c), ctypes.byref(w)))
        return int(c.value), int(w.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            check(lib().ph_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def perm_batched(mats: Sequence[torch.Tensor] | torch.Tensor, algo="glynn", accum="dd", chunk_log2: int = 0,
                 waves: int = 0) -> torch.Tensor:
    """Permanents of a list of square complex128 CUDA matrices (or a
    (batch, n, n) tensor) through ph_perm_batched."""
    if isinstance(mats, torch.Tensor):
        if mats.dim() != 3 or mats.shape[1] != mats.shape[2]:
            raise ValueError("expected (batch, n, n)")
        _need_c128_cuda("mats", mats)
        ns, flat = [int(mats.shape[1])] * int(mats.shape[0]), mats.contiguous().reshape(-1)
        mats = [mats] if mats.shape[0] else []
    else:
        for m in mats:
            _need_c128_cuda("matrix", m)
        ns, flat = _pack(mats)
    batch = len(ns)
    dev = mats[0].device if batch else torch.device("cuda")
    out = torch.empty(batch, dtype=torch.complex128, device=dev)
    if batch == 0:
        return out
    n_arr = (ctypes.c_int32 * batch)(*ns)
    o = opts(algo, accum, chunk_log2, waves)
    check(lib().ph_perm_batched(_ptr(flat), None, n_arr, batch, _ptr(out), ctypes.byref(o), _stream(flat)))
    return out


def perm_grad(a: torch.Tensor, grad_out: torch.Tensor | None = None, accum="dd", chunk_log2: int = 0,
              waves: int = 0, want_perm: bool = True):
    """(perm, grad) for a (batch, n, n) or (n, n) complex128 CUDA tensor:
    grad[b] = grad_out[b] * conj(dPer/dA[b]) (grad_out None means 1)."""
    _need_c128_cuda("a", a)
    single = a.dim() == 2
    a3 = a.unsqueeze(0) if single else a
    if a3.dim() != 3 or a3.shape[1] != a3.shape[2]:
        raise ValueError("expected (batch, n, n) or (n, n)")
    a3 = a3.contiguous()
    batch, n = a3.shape[0], a3.shape[1]
    g = None
    if grad_out is not None:
        _need_c128_cuda("grad_out", grad_out)
        if grad_out.numel() != batch or grad_out.device != a3.device:
            raise ValueError(f"grad_out needs {batch} values on {a3.device}")
        g = grad_out.reshape(batch).contiguous()
    p = torch.empty(batch, dtype=torch.complex128, device=a.device) if want_perm else None
    ga = torch.empty_like(a3)
    o = opts("glynn", accum, chunk_log2, waves)
    check(lib().ph_perm_grad(_ptr(a3), n, batch, _ptr(g), _ptr(p), _ptr(ga), ctypes.byref(o), _stream(a3)))
    if single:
        return (p[0] if p is not None else None), ga[0]
    return p, ga


def _modes(in_modes, patterns, m: int):
    """Host int32 copies of the mode lists: (in_modes (n,), patterns (npat, n))."""
    ins = np.ascontiguousarray(np.asarray(in_modes, dtype=np.int64).reshape(-1).astype(np.int32))
    n = ins.shape[0]
    pats = np.asarray(patterns, dtype=np.int64)
    if pats.ndim == 1 and pats.size == 0:
        pats = pats.reshape(0, n)
    if pats.ndim != 2 or pats.shape[1] != n:
        raise ValueError(f"patterns must have shape (n_patterns, {n})")
    pats = np.ascontiguousarray(pats.astype(np.int32))
    return ins, pats


def _i32p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _need_square_u(u: torch.Tensor):
    _need_c128_cuda("u", u)
    if u.dim() != 2 or u.shape[0] != u.shape[1]:
        raise ValueError("u must be an m x m matrix")
    return u if u.stride(1) == 1 else u.contiguous()


def boson_probs(u: torch.Tensor, in_modes, patterns, algo="glynn", accum="dd", ungrouped: bool = False) -> torch.Tensor:
    """Eq. (1) probabilities Pr[S -> T_p] for each row T_p of `patterns`.

    u: m x m complex128 CUDA tensor indexed [output mode, input mode];
    in_modes: the n input modes (repeats for multi-photon inputs);
    patterns: (n_patterns, n) output modes (repeats for collisions);
    ungrouped: one full sweep per pattern instead of the multiplicity-grouped
    sweeps (PH_FLAG_UNGROUPED)."""
    u = _need_square_u(u)
    m = u.shape[0]
    ins, pats = _modes(in_modes, patterns, m)
    n, npat = ins.shape[0], pats.shape[0]
    probs = torch.empty(npat, dtype=torch.float64, device=u.device)
    o = opts(algo, accum, flags=PH_FLAG_UNGROUPED if ungrouped else 0)
    check(lib().ph_boson_probs(_ptr(u), m, u.stride(0), _i32p(ins), n, _i32p(pats), npat, _ptr(probs),
                               ctypes.byref(o), _stream(u)))
    return probs


def boson_probs_grad(u: torch.Tensor, in_modes, patterns, weights: torch.Tensor | None = None, accum="dd",
                     ungrouped: bool = False, full: bool = False):
    """(probs, dU): dU (m x n) holds dL/dU[:, in_modes[k]] in column k for
    L = sum_p w_p Pr[S -> T_p] (PyTorch's conjugate-Wirtinger convention).
    ungrouped: one full sweep per pattern (PH_FLAG_UNGROUPED).  full: dU is
    the m x m gradient with respect to all of U, photons that share an input
    mode added into its column (PH_FLAG_DU_FULL)."""
    u = _need_square_u(u)
    m = u.shape[0]
    ins, pats = _modes(in_modes, patterns, m)
    n, npat = ins.shape[0], pats.shape[0]
    probs = torch.empty(npat, dtype=torch.float64, device=u.device)
    du = torch.empty((m, m if full else n), dtype=torch.complex128, device=u.device)
    w = None
    if weights is not None:
        w = weights.to(device=u.device, dtype=torch.float64).contiguous()
        if w.numel() != npat:
            raise ValueError("weights needs one entry per pattern")
    o = opts("glynn", accum, flags=(PH_FLAG_UNGROUPED if ungrouped else 0) | (PH_FLAG_DU_FULL if full else 0))
    check(lib().ph_boson_probs_grad(_ptr(u), m, u.stride(0), _i32p(ins), n, _i32p(pats), npat, _ptr(w),
                                    _ptr(probs), _ptr(du), du.stride(0), ctypes.byref(o), _stream(u)))
    return probs, du


def perm_row_minors(b: torch.Tensor, accum="dd", out: torch.Tensor | None = None) -> torch.Tensor:
    """Per of b without column l, for each l: b is (..., n, n+1) complex128 on
    the GPU; the result is (..., n+1) (ph_perm_row_minors)."""
    _need_c128_cuda("b", b)
    if b.dim() < 2 or b.shape[-1] != b.shape[-2] + 1:
        raise ValueError("b must be (..., n, n + 1)")
    lead, n = b.shape[:-2], b.shape[-2]
    count = int(np.prod(lead)) if len(lead) else 1
    flat = b.reshape(count, n, n + 1).contiguous()
    if out is None:
        out = torch.empty(flat.shape[0], n + 1, dtype=torch.complex128, device=b.device)
    else:
        _need_out("out", out, torch.complex128, flat.shape[0] * (n + 1), b.device)
    o = opts("glynn", accum)
    check(lib().ph_perm_row_minors(_ptr(flat), n, flat.shape[0], _ptr(out), ctypes.byref(o), _stream(b)))
    return out.reshape(*lead, n + 1)


def sample_inputs(nsamples: int, n: int, seed=None):
    """Random inputs of the sampler: a uniformly random column order and n
    uniforms in [0, 1) per sample (numpy's default generator)."""
    rng = np.random.default_rng(seed)
    perms = rng.permuted(np.tile(np.arange(n, dtype=np.int32), (nsamples, 1)), axis=1)
    return np.ascontiguousarray(perms, dtype=np.int32), rng.random((nsamples, n))


def boson_sample(u: torch.Tensor, in_modes, nsamples: int | None = None, perms=None, uniforms=None, seed=None,
                 accum="dd", unsorted: bool = False, out: torch.Tensor | None = None) -> torch.Tensor:
    """Boson-sampling outputs (ph_boson_sample): an (nsamples, n) int32 CUDA
    tensor, each row the sorted output modes of one sample (the placement
    order r_1..r_n with unsorted=True, PH_FLAG_UNSORTED).  perms
    (nsamples x n, a permutation of 0..n-1 per row) and uniforms (nsamples x n
    in [0, 1)) are host arrays; when both are None they are drawn with
    sample_inputs(nsamples, n, seed)."""
    u = _need_square_u(u)
    m = u.shape[0]
    ins, _ = _modes(in_modes, np.zeros((0, len(in_modes)), np.int32), m)
    n = ins.shape[0]
    if perms is None and uniforms is None:
        if nsamples is None:
            raise ValueError("give nsamples, or perms and uniforms")
        perms, uniforms = sample_inputs(int(nsamples), n, seed)
    if perms is None or uniforms is None:
        raise ValueError("give both perms and uniforms, or neither")
    perms = np.ascontiguousarray(np.asarray(perms, dtype=np.int64).reshape(-1, n).astype(np.int32))
    uniforms = np.ascontiguousarray(np.asarray(uniforms, dtype=np.float64).reshape(-1, n))
    ns = perms.shape[0]
    if uniforms.shape[0] != ns or (nsamples is not None and int(nsamples) != ns):
        raise ValueError("perms and uniforms need one row per sample")
    if out is None:
        out = torch.empty((ns, n), dtype=torch.int32, device=u.device)
    elif out.dtype != torch.int32 or not out.is_cuda or tuple(out.shape) != (ns, n) or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous ({ns}, {n}) int32 CUDA tensor")
    o = opts("glynn", accum, flags=PH_FLAG_UNSORTED if unsorted else 0)
    check(lib().ph_boson_sample(_ptr(u), m, u.stride(0), _i32p(ins), n, ns, _i32p(perms),
                                uniforms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(out),
                                ctypes.byref(o), _stream(u)))
    return out


def fp64_peak(iters: int = 1 << 14, device=None):
    """(GFLOP/s, sustained shader clock in MHz) of the FP64 FMA microbenchmark."""
    g = ctypes.c_double(0.0)
    mhz = ctypes.c_double(0.0)
    dev = torch.device(device or "cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    check(lib().ph_fp64_peak(int(iters), ctypes.byref(g), ctypes.byref(mhz), st))
    return g.value, mhz.value


def version() -> int:
    return lib().ph_version()
