"""Autotuner for the layout of the multifrontal solver's work.

Five knobs shape what the GPU factors and sweeps; none changes the solution:
  * leaf        -- cells per undivided nested-dissection leaf: the size of the
                   dense leaf fronts and the height of the separator tree;
  * small_lds   -- the LDS budget of the one-workgroup-per-front kernel: the
                   bottom levels whose fronts all fit run there, every level
                   above runs as a task graph over 64 x 64 tiles;
  * syrk_group  -- pivot blocks a Schur-tile task accumulates on the matrix
                   cores before it writes the tile (deeper: fewer tile reads
                   and writes; shallower: more tasks to spread);
  * split_kb    -- L21 size from which the sweeps take a front's update rows
                   as 64-row chunk items of their own;
  * block_split -- pivot blocks from which the sweeps take a front's pivot
                   part one 64-row block per item.
(The tile width itself, 64, is built into the kernels' register and LDS
layouts and is not a knob.)  The tuner times whole design iterations
(refactor + forward solve + objective + adjoint solve + gradient, the unit of
the paper's caching experiments; complex64 with its refinement steps,
complex128 without) on the caller's GPU with the caller's workload: first every (leaf, small_lds) pair, then, at the best pair, each
schedule knob in turn over a few values, keeping the fastest.  Results are
keyed by GPU architecture, grid, batch shape and precision; the committed
table ``tuned.json`` next to this module holds the choices measured on MI355X
(gfx950) for the standard workloads, and ``Plan`` consults it when the caller
leaves every knob at 0.
"""
from __future__ import annotations

import json
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(_PKG, "tuned.json")

LEAVES = (16, 25, 36, 49, 64)
SMALL_LDS = (-1, 32768, 65536, 98304, 131072, 163840)
SYRK_GROUPS = (4, 8, 16)
SPLIT_KBS = (64, 256, 1024, 4096, -1)
BLOCK_SPLITS = (3, 4, 6, 10, -1)
KNOBS = ("leaf", "small_lds", "syrk_group", "split_kb", "block_split")


def device_arch():
    """The current GPU's architecture name (e.g. gfx950), or None."""
    try:
        import torch
        if not torch.cuda.is_available():
            return None
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return None


def key(arch, nx, ny, npml, nsys, nrhs, prec):
    return f"{arch}/{nx}x{ny}/pml{npml}/sys{nsys}/rhs{nrhs}/{prec}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(nx, ny, npml, nsys, nrhs, prec, path=TABLE, arch=None):
    """The tuned knobs {leaf, small_lds, syrk_group, split_kb, block_split}
    for this workload on this GPU architecture (default: the current
    device's), or None."""
    arch = arch or device_arch()
    if arch is None:
        return None
    e = _load(path).get(key(arch, nx, ny, npml, nsys, nrhs, prec))
    return {k: int(e[k]) for k in KNOBS} if e else None


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


# relative timing noise below which the tuner times candidate rows again
TIE = 0.005


def autotune(p, prec="c128", max_ir=0, tol=1e-10, iters=6, leaves=LEAVES, small_lds=SMALL_LDS,
             syrk_groups=SYRK_GROUPS, split_kbs=SPLIT_KBS, block_splits=BLOCK_SPLITS, cache=None,
             verbose=False):
    """Tune problem p (problems.Problem) on the current GPU and return
    {knobs..., "ms", "table"}: every (leaf, small_lds) pair (pairs whose
    schedule coincides with one already timed -- same leaf, same number of
    bottom levels in the one-workgroup kernel -- are skipped), then each of
    syrk_group, split_kb, block_split in turn at the best setting so far.
    With cache=path the result is read from / merged into that JSON file."""
    import torch
    from . import problems as P
    from .fdfd import Plan

    arch = device_arch()
    k = key(arch, p.nx, p.ny, p.npml, p.nsys, p.nrhs, prec)
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

    def run(cfg, plan=None):
        plan = plan or Plan(p.nx, p.ny, p.npml, nsys=p.nsys, max_rhs=p.nrhs, prec=prec, tuned=False, **cfg)
        levels = plan.query()["small_levels"]
        ms = time_iterations(plan, eps_list, b, c, om, max_ir=max_ir, tol=tol)
        info = plan.query()
        plan.close()
        # the values in effect (a 0 in cfg stands for the library's default)
        row = {kk: int(info[kk]) for kk in KNOBS}
        row.update(small_levels=levels, ms=ms, status=info["status_str"])
        table.append(row)
        if verbose:
            print("autotune", k, row, flush=True)
        return row

    def good(r):
        return r["status"] in ("ok", "pivots perturbed")

    base = {"syrk_group": 0, "split_kb": 0, "block_split": 0}
    for leaf in leaves:
        seen = set()
        for sl in small_lds:
            cfg = dict(base, leaf=leaf, small_lds=sl)
            plan = Plan(p.nx, p.ny, p.npml, nsys=p.nsys, max_rhs=p.nrhs, prec=prec, tuned=False, **cfg)
            levels = plan.query()["small_levels"]
            if levels in seen:
                plan.close()
                continue
            seen.add(levels)
            run(cfg, plan)
    best = min(filter(good, table), key=lambda r: r["ms"])
    for name, values in (("syrk_group", syrk_groups), ("split_kb", split_kbs), ("block_split", block_splits)):
        for v in values:
            cfg = {kk: best[kk] for kk in KNOBS}
            cfg[name] = v
            if any(all(r[kk] == cfg[kk] for kk in KNOBS) for r in table):
                continue
            run(cfg)
        best = min(filter(good, table), key=lambda r: r["ms"])
    # Rows within the timing noise of the best are timed again, three runs
    # each, and the choice is the fastest of those (marked "retimed"): one
    # run cannot order layouts a few tenths of a millisecond apart.
    near = [r for r in table if good(r) and r["ms"] <= best["ms"] * (1.0 + TIE)]
    if len(near) > 1:
        final = []
        for r in near:
            cfg = {kk: r[kk] for kk in KNOBS}
            plan = Plan(p.nx, p.ny, p.npml, nsys=p.nsys, max_rhs=p.nrhs, prec=prec, tuned=False, **cfg)
            ms = float(np.mean([time_iterations(plan, eps_list, b, c, om, max_ir=max_ir, tol=tol) for _ in range(3)]))
            info = plan.query()
            plan.close()
            row = dict(r, ms=ms, status=info["status_str"], retimed=True)
            table.append(row)
            final.append(row)
            if verbose:
                print("autotune", k, row, flush=True)
        best = min(filter(good, final), key=lambda r: r["ms"])
    out = {kk: best[kk] for kk in KNOBS}
    out.update(ms=best["ms"], max_ir=max_ir, ir_tol=tol, arch=arch, table=table)
    if cache:
        d = _load(cache)
        d[k] = out
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return out


def main(argv=None):
    """python -m paper_2307_05388_amd.autotune --workloads small60,plain300,diff500,mux400,large2000"""
    import argparse
    from . import problems as P
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--workloads", default="small60,plain300,diff500,mux400,large2000")
    ap.add_argument("--precs", default="c128,c64")
    # complex128 layouts are compared without refinement: whether a solve
    # takes its one step depends on the residual landing just above or below
    # the tolerance, which would add a whole sweep pass of noise between them
    ap.add_argument("--max-ir-c128", type=int, default=0, help="refinement steps for the complex128 form")
    ap.add_argument("--max-ir-c64", type=int, default=16, help="refinement steps for the complex64 form")
    ap.add_argument("--ir-tol", type=float, default=1e-10)
    ap.add_argument("--iters", type=int, default=6)
    ap.add_argument("--out", default=TABLE)
    a = ap.parse_args(argv)
    for name in a.workloads.split(","):
        p = P.make_problem(name)
        for prec in a.precs.split(","):
            r = autotune(p, prec=prec, max_ir=a.max_ir_c64 if prec == "c64" else a.max_ir_c128, tol=a.ir_tol,
                         iters=a.iters,
                         cache=a.out, verbose=True)
            print(name, prec, "->", {k: r[k] for k in KNOBS + ("ms",)}, flush=True)


if __name__ == "__main__":
    main()
