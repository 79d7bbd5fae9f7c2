"""torch.autograd.Function mapping the design-region permittivity to the fields.

Forward: refactor with the new permittivity, then solve A x = b (Eq. 2).
Backward: the adjoint solve A^T lam = (dF/dx)^T (Eq. 4) with the factor cached
by the forward call (no second factorisation, Sec. II), then the gradient
dF/deps_n = -2 w^2 Re(lam_n x_n) (Eq. 3), summed over systems and right-hand
sides and restricted to the design block.

PyTorch hands the backward of a real loss L the tensor grad_x = 2 conj(dL/dx)
for a complex output x, so the adjoint source (dF/dx)^T is conj(grad_x) / 2.
"""
from __future__ import annotations

import torch

from .fdfd import FDFD_GRAD_SUM_SYSTEMS


class FDFDSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps_design, plan, base_eps, design, omegas, b, max_ir, tol):
        i0, i1, j0, j1 = design
        eps = base_eps.detach().clone()
        eps[..., j0:j1, i0:i1] = eps_design.detach()
        plan.refactor(eps.contiguous(), omegas)
        x = plan.solve(b, max_ir=max_ir, tol=tol)
        ctx.plan = plan
        ctx.generation = plan.generation
        ctx.eps = eps
        ctx.omegas = omegas
        ctx.design = design
        ctx.max_ir, ctx.tol = max_ir, tol
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, grad_x):
        (x,) = ctx.saved_tensors
        plan = ctx.plan
        if plan.generation != ctx.generation:
            # the plan was refactored for another permittivity since forward
            plan.refactor(ctx.eps.contiguous(), ctx.omegas)
            ctx.generation = plan.generation
        g = (grad_x.conj() * 0.5).contiguous()
        grad = plan.adjoint_grad(x, g, flags=FDFD_GRAD_SUM_SYSTEMS, max_ir=ctx.max_ir, tol=ctx.tol)
        i0, i1, j0, j1 = ctx.design
        gd = grad.view(plan.ny, plan.nx)[j0:j1, i0:i1]
        return gd, None, None, None, None, None, None, None


def fdfd_fields(eps_design, plan, base_eps, design, omegas, b, max_ir=0, tol=0.0):
    """Differentiable x(eps_design) of shape (nsys, nrhs, N)."""
    return FDFDSolve.apply(eps_design, plan, base_eps, tuple(design), omegas, b, max_ir, tol)


def mode_overlap(x, c):
    """F = sum over systems and right-hand sides of |c^H x|^2 (torch, on device)."""
    ov = torch.matmul(x, c.conj())
    return (ov.real ** 2 + ov.imag ** 2).sum()
