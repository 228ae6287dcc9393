"""Assembly as a differentiable function of the densities (torch.autograd).

K(rho) = sum_e E(rho_e) K_e^0 is linear in E(rho_e), so for any loss L(K)
dL/drho_e = E'(rho_e) <dL/dK, K_e^0> over the element's slots: the reverse of
assembly, computed by the library's backward kernel (soptx_assemble_backward).
With dL/dK = -u u^T restricted to the pattern this is the compliance
sensitivity of Appendix D (dc_e = -E'(rho_e) u_e^T K_e^0 u_e); entries of
fixed rows and columns are constants of the assembly and carry no gradient.
"""
from __future__ import annotations

import torch

from . import api

__all__ = ["assemble", "AssembleFunction"]


class AssembleFunction(torch.autograd.Function):
    """rho -> K values (FP64, [nnz]) with a hand-written backward."""

    @staticmethod
    def forward(ctx, rho, pattern: "api.Pattern", material: "api.Material", mask, prec: int, stream):
        K = pattern.assemble(material, rho.detach(), mask, prec=prec, stream=stream)
        ctx.save_for_backward(rho)
        ctx.pattern, ctx.material, ctx.mask, ctx.prec, ctx.stream = pattern, material, mask, prec, stream
        return K

    @staticmethod
    def backward(ctx, Kbar):
        (rho,) = ctx.saved_tensors
        if not ctx.needs_input_grad[0]:
            return None, None, None, None, None, None
        drho = ctx.pattern.backward(ctx.material, rho.detach(), Kbar.contiguous(), ctx.mask, prec=ctx.prec,
                                    stream=ctx.stream)
        return drho, None, None, None, None, None


def assemble(pattern: "api.Pattern", material: "api.Material", rho: torch.Tensor, mask=None,
             prec: int = api.FP64, stream=None) -> torch.Tensor:
    """Differentiable soptx_assemble: returns K values, gradients flow to rho."""
    return AssembleFunction.apply(rho, pattern, material, mask, prec, stream)
