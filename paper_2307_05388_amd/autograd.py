"""torch.autograd.Function mapping the design-region permittivity to the fields.

Forward: refactor with the new permittivity, then solve A x = b (Eq. 2).
Backward: the adjoint solve A^T lam = (dF/dx)^T (Eq. 4) with the factor cached
by the forward call (no second factorisation, Sec. II), then the gradient
dF/deps_n = -2 w^2 Re(lam_n x_n) (Eq. 3), summed over right-hand sides and
restricted to the design block.  A design map shared by every system (shape
(h, w)) gets the gradient summed over systems; a per-system map (shape
(nsys, h, w), on a per-system base map) gets one gradient per system.

PyTorch hands the backward of a real loss L the tensor grad_x = 2 conj(dL/dx)
for a complex output x, so the adjoint source (dF/dx)^T is conj(grad_x) / 2.

Numerical conditions found on the device (non-finite values, a refinement that
misses its tolerance, a dependency wait that gave up) are read back after each
solve (fdfd_query) and raised as FDFDError, so a bad field or gradient never
reaches the caller silently.
"""
from __future__ import annotations

import torch

from .fdfd import FDFD_ERR_NUMERIC, FDFD_GRAD_SUM_SYSTEMS, FDFDError, param_backward, param_desc, param_forward

# Refinement used when the caller leaves max_ir at None: none for complex128
# factors, FP64 refinement to a relative residual of 1e-12 for complex64.
C64_DEFAULT_IR = (10, 1e-12)


def _check_status(plan, what):
    info = plan.query()
    if info["status"] == FDFD_ERR_NUMERIC:
        raise FDFDError(info["status"], f"{what}: {info.get('error', info['status_str'])}")
    return info


class FDFDSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps_design, plan, base_eps, design, omegas, b, max_ir, tol):
        i0, i1, j0, j1 = design
        per_sys = eps_design.dim() == 3
        if per_sys:
            if eps_design.shape[0] != plan.nsys or base_eps.dim() != 3:
                raise ValueError("a per-system design map (nsys, h, w) needs a per-system base map (nsys, ny, nx)")
        elif eps_design.dim() != 2:
            raise ValueError("eps_design must be (h, w) or (nsys, h, w)")
        eps = base_eps.detach().clone()
        eps[..., j0:j1, i0:i1] = eps_design.detach()
        plan.refactor(eps.contiguous(), omegas)
        x = plan.solve(b, max_ir=max_ir, tol=tol)
        _check_status(plan, "forward solve")
        ctx.plan = plan
        ctx.generation = plan.generation
        ctx.eps = eps
        ctx.omegas = omegas
        ctx.design = design
        ctx.per_sys = per_sys
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
        flags = 0 if ctx.per_sys else FDFD_GRAD_SUM_SYSTEMS
        grad = plan.adjoint_grad(x, g, flags=flags, max_ir=ctx.max_ir, tol=ctx.tol)
        _check_status(plan, "adjoint solve")
        i0, i1, j0, j1 = ctx.design
        if ctx.per_sys:
            gd = grad.view(plan.nsys, plan.ny, plan.nx)[:, j0:j1, i0:i1]
        else:
            gd = grad.view(plan.ny, plan.nx)[j0:j1, i0:i1]
        return gd, None, None, None, None, None, None, None


def fdfd_fields(eps_design, plan, base_eps, design, omegas, b, max_ir=None, tol=None):
    """Differentiable x(eps_design) of shape (nsys, nrhs, N).

    max_ir / tol default to no refinement for complex128 plans and to FP64
    refinement (at most 10 steps, relative residual 1e-12) for complex64
    plans, so a complex64 plan never returns single-precision fields silently.
    """
    if max_ir is None:
        max_ir, dtol = C64_DEFAULT_IR if plan.prec == "c64" else (0, 0.0)
        tol = dtol if tol is None else tol
    if tol is None:
        tol = 0.0
    return FDFDSolve.apply(eps_design, plan, base_eps, tuple(design), omegas, b, max_ir, tol)


def mode_overlap(x, c):
    """F = sum over systems and right-hand sides of |c^H x|^2 (torch, on device)."""
    ov = torch.matmul(x, c.conj())
    return (ov.real ** 2 + ov.imag ** 2).sum()


class DesignMap(torch.autograd.Function):
    """theta (h, w) in [0, 1] -> permittivity of the design block (h, w): the
    smoothing filter and the projection of Sec. III / IV, both in the
    library's kernels (fdfd_param_forward / fdfd_param_backward)."""

    @staticmethod
    def forward(ctx, theta, desc):
        theta = theta.detach().contiguous()
        rho = torch.empty_like(theta)
        eps = torch.empty_like(theta)
        param_forward(desc, theta, rho, eps)
        ctx.desc = desc
        ctx.save_for_backward(rho)
        return eps

    @staticmethod
    def backward(ctx, grad_eps):
        (rho,) = ctx.saved_tensors
        work = torch.empty_like(rho)
        grad_theta = torch.empty_like(rho)
        param_backward(ctx.desc, rho, grad_eps.contiguous(), work, grad_theta)
        return grad_theta, None


def design_map(theta, radius, beta, eta=0.5, eps_min=2.085, eps_max=12.11):
    """Differentiable eps of the design block from theta (float64, (h, w),
    on the GPU); radius in cells (the paper's 200 nm over dx)."""
    if theta.dim() != 2 or theta.dtype != torch.float64 or not theta.is_cuda:
        raise ValueError("theta must be a float64 (h, w) CUDA tensor")
    h, w = theta.shape
    return DesignMap.apply(theta, param_desc(w, h, radius, beta, eta, eps_min, eps_max))
