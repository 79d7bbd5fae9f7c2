"""Autotuner for the front layout of the multifrontal solver.

Two knobs shape the fronts the GPU factors and sweeps:
  * leaf       -- cells per undivided nested-dissection leaf: the size of the
                  dense leaf fronts and the height of the separator tree;
  * small_lds  -- the LDS budget of the one-workgroup-per-front kernel: the
                  bottom levels whose fronts all fit run there, every level
                  above runs as a task graph over 64 x 64 tiles.
Both change only the factor's layout, never the solution.  The tuner times
whole design iterations (refactor + forward solve + objective + adjoint solve +
gradient, the unit of the paper's caching experiments) for each candidate on
the caller's GPU, with the caller's workload, and keeps the fastest.  Results
are cached in a JSON file keyed by grid, batch shape and precision, and the
committed table ``tuned.json`` next to this module holds the choices measured
on MI355X for the standard workloads; ``Plan`` consults it when the caller
leaves both knobs at 0.
"""
from __future__ import annotations

import json
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(_PKG, "tuned.json")

LEAVES = (16, 25, 36, 49, 64)
SMALL_LDS = (-1, 32768, 65536, 98304)


def key(nx, ny, npml, nsys, nrhs, prec):
    return f"{nx}x{ny}/pml{npml}/sys{nsys}/rhs{nrhs}/{prec}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(nx, ny, npml, nsys, nrhs, prec, path=TABLE):
    """Tuned (leaf, small_lds) for this workload, or None."""
    e = _load(path).get(key(nx, ny, npml, nsys, nrhs, prec))
    return (int(e["leaf"]), int(e["small_lds"])) if e else None


def time_iterations(plan, eps_list, b, c, omegas, max_ir=0, tol=1e-10, warmup=2):
    """Mean milliseconds of one design iteration over eps_list (after warmup)."""
    import torch
    from .fdfd import FDFD_GRAD_SUM_SYSTEMS
    e_in = torch.empty_like(eps_list[0])
    x = torch.empty_like(b)
    g = torch.empty_like(b)
    grad = torch.empty(b.shape[-1], dtype=torch.float64, device=b.device)
    cc = c.conj()

    def step(eps):
        e_in.copy_(eps)
        plan.refactor(e_in, omegas)
        plan.solve(b, x=x, max_ir=max_ir, tol=tol)
        ov = torch.matmul(x, cc)
        torch.mul(cc[None, None, :], ov.conj()[..., None], out=g)
        plan.adjoint_grad(x, g, grad=grad, flags=FDFD_GRAD_SUM_SYSTEMS, max_ir=max_ir, tol=tol)

    for k in range(warmup):
        step(eps_list[k % len(eps_list)])
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for eps in eps_list:
        step(eps)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / len(eps_list)


def autotune(p, prec="c128", max_ir=0, tol=1e-10, iters=6, leaves=LEAVES, small_lds=SMALL_LDS,
             cache=None, verbose=False):
    """Time every (leaf, small_lds) candidate on problem p (problems.Problem)
    and return {"leaf", "small_lds", "ms", "table"}.  Candidates whose schedule
    coincides with one already timed (same leaf, same number of bottom levels in
    the one-workgroup kernel) are skipped.  With cache=path the result is read
    from / merged into that JSON file."""
    import torch
    from . import problems as P
    from .fdfd import Plan

    k = key(p.nx, p.ny, p.npml, p.nsys, p.nrhs, prec)
    if cache:
        hit = _load(cache).get(k)
        if hit:
            return hit
    dev = torch.device("cuda:0")
    eps_list = [torch.from_numpy(np.ascontiguousarray(P.design_eps(p, t))).to(dev) for t in range(iters)]
    b = torch.from_numpy(P.sources(p)).to(dev)
    c = torch.from_numpy(P.objective_vector(p)).to(dev)
    om = P.omegas(p)
    table = []
    for leaf in leaves:
        seen = set()
        for sl in small_lds:
            plan = Plan(p.nx, p.ny, p.npml, nsys=p.nsys, max_rhs=p.nrhs, prec=prec, leaf=leaf, small_lds=sl)
            levels = plan.query()["small_levels"]
            if levels in seen:
                plan.close()
                continue
            seen.add(levels)
            ms = time_iterations(plan, eps_list, b, c, om, max_ir=max_ir, tol=tol)
            info = plan.query()
            plan.close()
            row = {"leaf": leaf, "small_lds": sl, "small_levels": levels, "ms": ms,
                   "status": info["status_str"]}
            table.append(row)
            if verbose:
                print("autotune", k, row, flush=True)
    ok = [r for r in table if r["status"] in ("ok", "pivots perturbed")]
    best = min(ok, key=lambda r: r["ms"])
    out = {"leaf": best["leaf"], "small_lds": best["small_lds"], "ms": best["ms"], "max_ir": max_ir,
           "ir_tol": tol, "table": table}
    if cache:
        d = _load(cache)
        d[k] = out
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return out


def main(argv=None):
    """python -m paper_2307_05388_amd.autotune --workloads plain300,mux400 --out tuned.json"""
    import argparse
    from . import problems as P
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--workloads", default="plain300,diff500,mux400")
    ap.add_argument("--precs", default="c128,c64")
    ap.add_argument("--max-ir", type=int, default=4, help="refinement steps for the complex64 form")
    ap.add_argument("--ir-tol", type=float, default=1e-10)
    ap.add_argument("--iters", type=int, default=6)
    ap.add_argument("--out", default=TABLE)
    a = ap.parse_args(argv)
    for name in a.workloads.split(","):
        p = P.make_problem(name)
        for prec in a.precs.split(","):
            r = autotune(p, prec=prec, max_ir=a.max_ir if prec == "c64" else 0, tol=a.ir_tol, iters=a.iters,
                         cache=a.out, verbose=True)
            print(name, prec, "->", {k: r[k] for k in ("leaf", "small_lds", "ms")}, flush=True)


if __name__ == "__main__":
    main()
