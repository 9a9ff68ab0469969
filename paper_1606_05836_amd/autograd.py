"""torch.autograd.Function wrapper of the HIP permanent and its gradient.

Forward: Per(A) for each n x n matrix of A (..., n, n) through ph_perm_grad's
sweep, which returns the permanent and, when the input needs a gradient,
nothing more is kept than A itself.  Backward: ph_perm_grad with the upstream
gradient g, giving g * conj(dPer/dA) -- PyTorch's conjugate-Wirtinger
convention for a holomorphic function.
"""
from __future__ import annotations

import torch

from . import permhip as _p


class PermFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a: torch.Tensor) -> torch.Tensor:
        if a.dim() < 2 or a.shape[-1] != a.shape[-2]:
            raise ValueError("expected (..., n, n)")
        lead = a.shape[:-2]
        n = a.shape[-1]
        a3 = a.reshape(-1, n, n).contiguous()
        out = _p.perm_batched(a3) if a3.shape[0] else torch.empty(0, dtype=a.dtype, device=a.device)
        ctx.save_for_backward(a3)
        ctx.lead = lead
        return out.reshape(lead)

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (a3,) = ctx.saved_tensors
        n = a3.shape[-1]
        if a3.shape[0] == 0:
            return torch.zeros(ctx.lead + (n, n), dtype=a3.dtype, device=a3.device)
        _, ga = _p.perm_grad(a3, grad_out=g.reshape(-1).to(a3.dtype).contiguous(), want_perm=False)
        return ga.reshape(ctx.lead + (n, n))


def permanent(a: torch.Tensor) -> torch.Tensor:
    """Differentiable permanent of (..., n, n) complex128 CUDA matrices."""
    return PermFn.apply(a)


class BosonProbsFn(torch.autograd.Function):
    """Eq. (1) probabilities Pr[S -> T_p] as a differentiable function of U.

    Backward: ph_boson_probs_grad with the upstream gradient as the pattern
    weights and the m x m form of dU (PH_FLAG_DU_FULL): photons that share an
    input mode add into the same column of U's gradient, in the library."""

    @staticmethod
    def forward(ctx, u: torch.Tensor, in_modes, patterns) -> torch.Tensor:
        ctx.save_for_backward(u)
        ctx.in_modes = in_modes
        ctx.patterns = patterns
        return _p.boson_probs(u, in_modes, patterns)

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (u,) = ctx.saved_tensors
        _, gu = _p.boson_probs_grad(u, ctx.in_modes, ctx.patterns, weights=g, full=True)
        return gu, None, None


def boson_probabilities(u: torch.Tensor, in_modes, patterns) -> torch.Tensor:
    """Differentiable Eq. (1) probabilities of output patterns (rows of
    `patterns`) for input modes `in_modes` of the m x m complex128 CUDA unitary u."""
    return BosonProbsFn.apply(u, in_modes, patterns)
