"""torch.autograd.Function over the hsbuild forward and its hand-written adjoint.

HSBuildFunction.apply(tau, T, builder, k_frac, g) returns the full Hermitian
H and S (mirrored from the upper triangles the library writes); backward
passes the Hermitian parts of the incoming gradients to hsbuild_backward,
which recomputes the coefficients instead of keeping them.  The Hermitian
part is exact for tau and for every Hermitian direction of T.
"""
from __future__ import annotations

import torch

from .hsbuild import HSBuilder, hermitian_full


class HSBuildFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, tau: torch.Tensor, T: torch.Tensor, builder: HSBuilder, k_frac, g: torch.Tensor):
        H, S = builder.forward(k_frac, g, tau.detach(), T.detach())
        ctx.builder = builder
        ctx.k_frac = tuple(float(x) for x in k_frac)
        ctx.save_for_backward(tau.detach(), T.detach(), g)
        return hermitian_full(H), hermitian_full(S)

    @staticmethod
    def backward(ctx, gH, gS):
        tau, T, g = ctx.saved_tensors
        n = g.shape[0]
        zeros = None
        if gH is None or gS is None:
            zeros = torch.zeros((n, n), dtype=torch.complex128, device=tau.device)
        gH = zeros if gH is None else 0.5 * (gH + gH.conj().transpose(0, 1))
        gS = zeros if gS is None else 0.5 * (gS + gS.conj().transpose(0, 1))
        gT, gtau = ctx.builder.backward(ctx.k_frac, g, tau, T, gH.contiguous(), gS.contiguous())
        return gtau, gT, None, None, None


def hs_build(tau: torch.Tensor, T: torch.Tensor, builder: HSBuilder, k_frac, g: torch.Tensor):
    """Differentiable (H, S) as full Hermitian matrices."""
    return HSBuildFunction.apply(tau, T, builder, k_frac, g)
