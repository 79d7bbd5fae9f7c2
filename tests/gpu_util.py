"""Helpers shared by the GPU tests: run the HIP path and the CPU oracle on the
same seeded inputs."""
import os
import sys

import numpy as np

from paper_2307_05388_amd import problems as P


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def make_plan(p, prec="c128", max_rhs=None, leaf=0, small_lds=None, like=None):
    """Plan for problem p; small_lds overrides the LDS budget of the fused
    small-front kernel (0 forces the blocked large-front path everywhere).
    like=q: the front layout the tuned table gives problem q (so that factors
    of p and q are computed identically)."""
    from paper_2307_05388_amd.fdfd import Plan
    sl = 0 if small_lds is None else (-1 if small_lds == 0 else small_lds)
    knobs = {}
    if like is not None and leaf == 0 and small_lds is None:
        from paper_2307_05388_amd.autotune import lookup
        hit = lookup(like.nx, like.ny, like.npml, like.nsys, like.nrhs, prec)
        if hit:
            leaf, sl = hit["leaf"], hit["small_lds"]
            knobs = {k: hit[k] for k in ("syrk_group", "split_kb", "block_split")}
    return Plan(p.nx, p.ny, p.npml, nsys=p.nsys, max_rhs=max_rhs or p.nrhs, prec=prec, leaf=leaf, small_lds=sl,
                **knobs)


def gpu_iteration(plan, p, eps, b, g=None, c=None, max_ir=0, tol=0.0):
    """refactor + forward solve + adjoint/gradient; returns host arrays."""
    torch = torch_cuda()
    dev = torch.device("cuda:0")
    eps_t = torch.from_numpy(np.ascontiguousarray(eps)).to(dev)
    b_t = torch.from_numpy(np.ascontiguousarray(b)).to(dev)
    plan.refactor(eps_t, P.omegas(p))
    x_t = plan.solve(b_t, max_ir=max_ir, tol=tol)
    if g is None:
        c_t = torch.from_numpy(c).to(dev)
        ov = torch.matmul(x_t, c_t.conj())
        g_t = (c_t.conj()[None, None, :] * ov.conj()[..., None]).contiguous()
    else:
        g_t = torch.from_numpy(np.ascontiguousarray(g)).to(dev)
    lam_t = torch.empty_like(b_t)
    grad_t = plan.adjoint_grad(x_t, g_t, lam=lam_t, max_ir=max_ir, tol=tol)
    torch.cuda.synchronize()
    info = plan.query()
    return {"x": x_t.cpu().numpy(), "lam": lam_t.cpu().numpy(), "grad": grad_t.cpu().numpy(),
            "g": g_t.cpu().numpy(), "info": info}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def entry_err(a, b, floor=1e-6):
    """Largest per-entry error relative to the reference entry's own
    magnitude, floored at floor * max|b|: unlike the 2-norm it also sees errors
    confined to low-magnitude regions such as the PML."""
    a = np.asarray(a)
    b = np.asarray(b)
    scale = np.maximum(np.abs(b), floor * np.abs(b).max())
    return float((np.abs(a - b) / scale).max())


def leaf_first_pivot_cell(plan, nx, ny, npml):
    """A grid cell (i, j) outside the PML that is the first pivot of a leaf
    front (a front no other front names as parent), from the analysis tables."""
    from paper_2307_05388_amd.fdfd import FDFD_TABLE_FRONTS, FDFD_TABLE_PERM
    fr = plan.table(FDFD_TABLE_FRONTS).reshape(-1, 4)
    perm = plan.table(FDFD_TABLE_PERM)
    parents = set(int(v) for v in fr[:, 3] if v >= 0)
    for f in range(fr.shape[0]):
        if f in parents:
            continue
        n = int(perm[fr[f, 0]])
        i, j = n % nx, n // nx
        if npml <= i <= nx - npml - 1 and npml <= j <= ny - npml - 1:
            return i, j
    raise AssertionError("no leaf starts outside the PML")
