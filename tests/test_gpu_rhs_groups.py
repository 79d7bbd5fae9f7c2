"""More right-hand sides than one sweep pass holds.  The sweeps keep a
front's right-hand-side block in LDS, so at large fronts only a few columns
fit; the solves then take the columns in groups, one forward and one backward
pass over the factor per group, with the caller's (nsys, nrhs, N) layout kept.

  * a small grid with the group forced to 1 and to 2 columns (FDFD_SWEEP_RHS)
    and the split sweep items forced (FDFD_BLOCK_SPLIT, FDFD_SPLIT_KB): fields,
    adjoint fields and gradient of 2 wavelengths x 3 sources against the
    oracle, in both precisions;
  * 2000 x 2000 with three sources (the three input modes of the paper's
    multiplexer, Sec. IV) in complex128: the plan is made with max_rhs = 3
    although one pass holds fewer; every column's oracle residual is within
    1e-10 after FP64 refinement, and every column of the grouped solve equals
    the same column solved alone.
"""
import dataclasses

import numpy as np
import pytest

from paper_2307_05388_amd import problems as P
from gpu_util import entry_err, gpu_iteration, rel, say, torch_cuda

pytestmark = pytest.mark.gpu

THREE = ("gauss", "alt_gauss", "line")


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("group", [1, 2])
def test_forced_groups_against_oracle(oracle, monkeypatch, prec, group):
    from paper_2307_05388_amd.fdfd import Plan
    p = P.custom_problem(150, 131, 12, wavelengths_um=(1.50, 1.60), src_profiles=THREE)
    eps = P.design_eps(p, t=13)
    b = P.sources(p)
    c = P.objective_vector(p)
    ref = oracle.design_iteration(p.nx, p.ny, p.npml, P.omegas(p), eps, b, c=c)
    monkeypatch.setenv("FDFD_SWEEP_RHS", str(group))
    monkeypatch.setenv("FDFD_BLOCK_SPLIT", "2")
    monkeypatch.setenv("FDFD_SPLIT_KB", "1")
    plan = Plan(p.nx, p.ny, p.npml, nsys=p.nsys, max_rhs=3, prec=prec)
    assert plan.query()["rhs_group"] == group
    ir = (10, 1e-12) if prec == "c64" else (0, 0.0)
    say(f"case rhs group {group} of 3, {prec}, nsys {p.nsys}")
    out = gpu_iteration(plan, p, eps, b, c=c, max_ir=ir[0], tol=ir[1])
    tol = 1e-10 if prec == "c128" else 1e-8
    say(f"  x {rel(out['x'], ref['x']):.2e} entry {entry_err(out['x'], ref['x']):.2e} "
        f"lam {rel(out['lam'], ref['lam']):.2e} grad {rel(out['grad'], ref['grad']):.2e}")
    assert out["info"]["status"] in (0, 6)
    assert rel(out["x"], ref["x"]) < tol and rel(out["lam"], ref["lam"]) < tol
    assert entry_err(out["x"], ref["x"]) < 1e3 * tol
    assert rel(out["grad"], ref["grad"]) < 10 * tol
    plan.close()


def test_large2000_three_sources(oracle):
    torch = torch_cuda()
    from paper_2307_05388_amd.fdfd import Plan
    p = dataclasses.replace(P.make_problem("large2000"), src_profiles=THREE)
    eps = P.design_eps(p)
    b = P.sources(p)
    om = P.omegas(p)
    dev = torch.device("cuda:0")
    plan = Plan(p.nx, p.ny, p.npml, nsys=1, max_rhs=3, prec="c128")
    info = plan.query()
    say(f"case large2000 three sources: max_front {info['max_front']}, rhs per pass {info['rhs_group']}")
    assert info["rhs_group"] < 3
    plan.refactor(torch.from_numpy(eps).to(dev), om)
    bt = torch.from_numpy(b).to(dev)
    x0 = plan.solve(bt).cpu().numpy()
    for r in range(3):
        alone = plan.solve(bt[:, r:r + 1].contiguous()).cpu().numpy()
        say(f"  column {r}: grouped vs alone {rel(x0[:, r], alone[:, 0]):.2e}")
        assert rel(x0[:, r], alone[:, 0]) < 1e-13
    x = plan.solve(bt, max_ir=2, tol=1e-10).cpu().numpy()
    info = plan.query()
    assert info["status"] in (0, 6), info
    for r in range(3):
        res = oracle.relative_residual(p.nx, p.ny, p.npml, om[0], eps, x[0, r], b[0, r])
        say(f"  column {r}: oracle residual {res:.2e}")
        assert res < 1e-10
    plan.close()
