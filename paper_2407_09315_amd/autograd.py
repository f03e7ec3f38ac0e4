"""torch.autograd.Function around the library's forward and hand-written adjoint.

Forward: rbe_structure_factor + rbe_kspace_force -> (U per system, F).
Backward: rbe_kspace_vjp, which recomputes the phases; only rho (2 P doubles)
is saved from the forward besides the inputs.  The wave vectors m and weights
w are not differentiated.
"""
from __future__ import annotations

import torch

from .rbe import Plan


class RBEKSpace(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y, z, q, m, w, plan: Plan):
        F, U, rho = plan.forward(x, y, z, q, m, w)
        ctx.save_for_backward(x, y, z, q, m, w, rho)
        ctx.plan = plan
        return U, F

    @staticmethod
    def backward(ctx, gU, gF):
        x, y, z, q, m, w, rho = ctx.saved_tensors
        plan: Plan = ctx.plan
        if gU is None:
            gU = torch.zeros(plan.batch.B, dtype=torch.float64, device=x.device)
        if gF is None:
            gF = torch.zeros((3, plan.n_total), dtype=plan.force_dtype, device=x.device)
        gr, gq = plan.kspace_vjp(x, y, z, q, m, w, rho, gU.to(torch.float64).contiguous(),
                                 gF.to(plan.force_dtype).contiguous())
        return gr[0], gr[1], gr[2], gq, None, None, None


def rbe_kspace(x, y, z, q, m, w, plan: Plan):
    """(U (B,), F (3, N)) with gradients flowing to x, y, z and q."""
    return RBEKSpace.apply(x, y, z, q, m, w, plan)
