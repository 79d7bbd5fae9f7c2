"""fdfd_solve_noalloc, the allocation-free forward solve (its work vectors in
the library's static device array), against fdfd_solve through the C ABI.

Two calls in a row on the same GPU, the second with a smaller input (fewer
systems, fewer right-hand sides, a smaller grid), in both precisions and with
FP64 refinement; the output buffers are filled with NaN first, so that nothing
left from an earlier call can pass.  Both entry points run the same kernels
on the same inputs, so their fields agree to the parity bar (they are in fact
bitwise equal).  A plan whose solve does not fit the array is refused with
FDFD_ERR_ARG before anything is enqueued, and the plan still solves normally.
"""
import ctypes

import numpy as np
import pytest

from paper_2307_05388_amd import problems as P
from gpu_util import rel, say, torch_cuda

pytestmark = pytest.mark.gpu


def _noalloc(plan, b, x, max_ir, tol):
    import torch
    lib = plan._lib
    nrhs = b.shape[-2]
    return lib.fdfd_solve_noalloc(plan._h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()), nrhs,
                                  max_ir, tol, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("prec,max_ir,tol", [("c128", 0, 0.0), ("c128", 2, 1e-13), ("c64", 10, 1e-12)])
def test_noalloc_solve_matches_solve(prec, max_ir, tol):
    torch = torch_cuda()
    from paper_2307_05388_amd.fdfd import FDFD_OK, Plan
    dev = torch.device("cuda:0")
    cases = [P.custom_problem(150, 131, 12, wavelengths_um=(1.50, 1.60), src_profiles=("gauss", "alt_gauss")),
             P.custom_problem(60, 60, 10)]
    for k, p in enumerate(cases):
        say(f"case noalloc {prec} max_ir={max_ir} call {k + 1}: {p.nx}x{p.ny} nsys={p.nsys} nrhs={p.nrhs}")
        plan = Plan(p.nx, p.ny, p.npml, nsys=p.nsys, max_rhs=p.nrhs, prec=prec)
        eps = torch.from_numpy(np.stack([P.design_eps(p, t=20 + s) for s in range(p.nsys)])).to(dev)
        b = torch.from_numpy(P.sources(p)).to(dev)
        plan.refactor(eps, P.omegas(p))
        x_ref = plan.solve(b, max_ir=max_ir, tol=tol)
        torch.cuda.synchronize()
        info_ref = plan.query()
        x = torch.full_like(b, complex(float("nan"), float("nan")))
        assert _noalloc(plan, b, x, max_ir, tol) == FDFD_OK
        torch.cuda.synchronize()
        info = plan.query()
        e = rel(x.cpu().numpy(), x_ref.cpu().numpy())
        say(f"  rel diff {e:.2e}, bitwise {bool(torch.equal(x, x_ref))}, status {info['status_str']}, "
            f"refinement steps {info['ir_steps_solve']}")
        assert info["status"] == info_ref["status"] and info["status"] in (0, 6)
        assert info["ir_steps_solve"] == info_ref["ir_steps_solve"]
        assert e < (1e-12 if prec == "c128" else 1e-10)
        plan.close()


def test_noalloc_refuses_oversized_solve():
    torch = torch_cuda()
    from paper_2307_05388_amd.fdfd import FDFD_ERR_ARG, Plan
    dev = torch.device("cuda:0")
    p = P.custom_problem(1000, 1000, 20)
    plan = Plan(p.nx, p.ny, p.npml, prec="c128")
    plan.refactor(torch.from_numpy(P.design_eps(p)).to(dev), P.omegas(p))
    b = torch.from_numpy(P.sources(p)).to(dev)
    x = torch.zeros_like(b)
    assert _noalloc(plan, b, x, 0, 0.0) == FDFD_ERR_ARG
    say("  refused:", plan._lib.fdfd_last_error(plan._h).decode())
    torch.cuda.synchronize()
    assert torch.count_nonzero(x).item() == 0
    x2 = plan.solve(b)
    torch.cuda.synchronize()
    assert plan.query()["status"] in (0, 6)
    assert torch.isfinite(x2).all()
    plan.close()
