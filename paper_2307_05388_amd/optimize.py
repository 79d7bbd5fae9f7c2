"""The inverse-design loop around the cached-factorisation solver (paper
Sec. III and Sec. IV): design variables theta in [0, 1] -> smoothing filter ->
projection -> permittivity of the design block -> FDFD solves for every
wavelength and input mode (one analysis, one batched refactorisation per
iteration, one forward and one adjoint solve per mode with the same factor)
-> transmissions into the output ports -> objective -> gradient, minimised
by L-BFGS-B under the bounds 0 <= theta <= 1.

The device is a synthetic stand-in for the paper's 1 x 3 mode multiplexer
(its geometry and targets are not published): an input guide carrying the
TE0, TE1 and TE2 modes, three single-mode output guides, and a square design
block between them; the target routes input mode m into output guide m, at
every wavelength.  Transmissions are overlap powers normalised by a
straight-guide reference solved once with the same cached analysis:
    T[l, m, k] = |c[l, k]^H x[l, m]|^2 / P[l, m],
    F = sum_{l, m} (1 - T[l, m, m])^2 + sum_{l, m, k != m} T[l, m, k]^2.
The optimiser itself (scipy's L-BFGS-B) runs on the host, as in the paper;
every per-iteration array stays on the GPU except theta and its gradient.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import problems as P
from .modes import column_modes


@dataclass
class MuxDevice:
    nx: int = 200
    ny: int = 160
    npml: int = 15
    dx_nm: float = 40.0
    wavelengths_um: tuple = (1.50, 1.55, 1.60)
    nmodes: int = 3
    in_width: int = 18            # cells: carries TE0..TE2 at these wavelengths
    out_width: int = 5            # cells: single-mode (200 nm; the 2D cut-off is about 237 nm)
    design: tuple = (60, 140, 40, 120)   # i0, i1, j0, j1
    radius_nm: float = 200.0      # smoothing filter radius (Sec. III)
    beta: float = 4.0             # projection steepness
    extra: dict = field(default_factory=dict)

    @property
    def N(self):
        return self.nx * self.ny

    @property
    def omegas(self):
        return 2.0 * np.pi * self.dx_nm / (np.asarray(self.wavelengths_um) * 1000.0)

    def out_rows(self):
        """Row ranges of the three output guides, spread over the design height."""
        i0, i1, j0, j1 = self.design
        h = j1 - j0
        centres = [j0 + h // 6, j0 + h // 2, j0 + 5 * h // 6]
        return [(c - self.out_width // 2, c - self.out_width // 2 + self.out_width) for c in centres]

    def in_rows(self):
        c = self.ny // 2
        return (c - self.in_width // 2, c - self.in_width // 2 + self.in_width)

    def base_eps(self, straight=False):
        """Background with the guides (and, for the reference, the input guide
        continued straight through)."""
        eps = np.full((self.ny, self.nx), P.EPS_SIO2)
        i0, i1, _, _ = self.design
        r0, r1 = self.in_rows()
        if straight:
            eps[r0:r1, :] = P.EPS_SI
            return eps
        eps[r0:r1, :i0] = P.EPS_SI
        for (a, b) in self.out_rows():
            eps[a:b, i1:] = P.EPS_SI
        return eps

    @property
    def src_col(self):
        return self.npml + 5

    @property
    def obj_col(self):
        return self.nx - self.npml - 6

    def sources_and_overlaps(self):
        """b: (nsys, nmodes, N) input-mode sources; c: (nsys, 3, N) output
        TE0 overlap vectors; c_ref: (nsys, nmodes, N) input-mode overlaps on
        the output column of the straight reference guide."""
        ns = len(self.wavelengths_um)
        b = np.zeros((ns, self.nmodes, self.ny, self.nx), dtype=np.complex128)
        c = np.zeros((ns, 3, self.ny, self.nx), dtype=np.complex128)
        c_ref = np.zeros((ns, self.nmodes, self.ny, self.nx), dtype=np.complex128)
        e_in = self.base_eps()
        for s, om in enumerate(self.omegas):
            _, prof = column_modes(e_in[:, self.src_col], om, self.nmodes)
            for m in range(self.nmodes):
                b[s, m, :, self.src_col] = prof[m]
                c_ref[s, m, :, self.obj_col] = prof[m]
            for k, (a, bb) in enumerate(self.out_rows()):
                col = np.full(self.ny, P.EPS_SIO2)
                col[a:bb] = P.EPS_SI
                _, po = column_modes(col, om, 1)
                c[s, k, :, self.obj_col] = po[0]
        return (b.reshape(ns, self.nmodes, self.N), c.reshape(ns, 3, self.N),
                c_ref.reshape(ns, self.nmodes, self.N))


class MuxObjective:
    """F(theta) and dF/dtheta on the GPU for a MuxDevice (one plan, reused)."""

    def __init__(self, dev: MuxDevice, prec="c128", max_ir=None, tol=None):
        import torch
        from .fdfd import Plan
        self.dev = dev
        self.torch = torch
        cuda = torch.device("cuda:0")
        ns = len(dev.wavelengths_um)
        self.plan = Plan(dev.nx, dev.ny, dev.npml, nsys=ns, max_rhs=dev.nmodes, prec=prec)
        b, c, c_ref = dev.sources_and_overlaps()
        self.b = torch.from_numpy(b).to(cuda)
        self.c = torch.from_numpy(c).to(cuda)
        self.cT = self.c.conj().transpose(-1, -2).contiguous()        # (nsys, N, 3)
        self.base = torch.from_numpy(dev.base_eps()).to(cuda)
        self.max_ir, self.tol = max_ir, tol
        # reference powers: the straight guide, same cached analysis
        ref_eps = torch.from_numpy(dev.base_eps(straight=True)).to(cuda)
        self.plan.refactor(ref_eps.contiguous(), dev.omegas)
        ir = (max_ir or 0, tol or 0.0) if prec == "c128" else (max_ir or 10, tol or 1e-12)
        x = self.plan.solve(self.b, max_ir=ir[0], tol=ir[1])
        cr = torch.from_numpy(c_ref).to(cuda)
        ov = (x * cr.conj()).sum(-1)
        self.P = (ov.real ** 2 + ov.imag ** 2).detach()          # (nsys, nmodes)
        self.target = torch.zeros((ns, dev.nmodes, 3), dtype=torch.float64, device=cuda)
        for m in range(min(dev.nmodes, 3)):
            self.target[:, m, m] = 1.0
        self.evals = 0
        self.seconds = 0.0

    def transmissions(self, x):
        ov = self.torch.matmul(x, self.cT)                            # (nsys, nmodes, 3)
        return (ov.real ** 2 + ov.imag ** 2) / self.P[..., None]

    def __call__(self, theta_np):
        """(F, dF/dtheta) as float64 numpy, for scipy."""
        torch = self.torch
        from .autograd import design_map, fdfd_fields
        t0 = time.perf_counter()
        d = self.dev
        th = torch.from_numpy(np.ascontiguousarray(theta_np.reshape(self._shape()))).to("cuda:0")
        th.requires_grad_(True)
        eps_d = design_map(th, d.radius_nm / d.dx_nm, d.beta)
        x = fdfd_fields(eps_d, self.plan, self.base, d.design, d.omegas, self.b, max_ir=self.max_ir, tol=self.tol)
        T = self.transmissions(x)
        F = ((T - self.target) ** 2).sum()
        F.backward()
        g = th.grad.detach().cpu().numpy().reshape(-1)
        f = float(F.item())
        self.evals += 1
        self.seconds += time.perf_counter() - t0
        self.last_T = T.detach()
        return f, g

    def _shape(self):
        i0, i1, j0, j1 = self.dev.design
        return (j1 - j0, i1 - i0)

    def close(self):
        self.plan.close()


def run_lbfgsb(dev: MuxDevice, iters=20, prec="c128", theta0=None, seed=0, callback=None):
    """L-BFGS-B on theta in [0, 1]; returns the history of F and timings."""
    from scipy.optimize import minimize
    obj = MuxObjective(dev, prec=prec)
    shape = obj._shape()
    if theta0 is None:
        theta0 = np.random.default_rng([seed, 31]).uniform(0.4, 0.6, size=shape)
    hist = []

    def fun(t):
        f, g = obj(t)
        hist.append(f)
        if callback:
            callback(len(hist), f)
        return f, g

    t0 = time.perf_counter()
    res = minimize(fun, theta0.reshape(-1), jac=True, method="L-BFGS-B", bounds=[(0.0, 1.0)] * theta0.size,
                   options={"maxiter": iters, "maxfun": 4 * iters})
    wall = time.perf_counter() - t0
    out = {"F": hist, "evals": obj.evals, "seconds_in_objective": obj.seconds, "wall_s": wall,
           "iterations": int(res.nit), "message": str(res.message), "theta": res.x.reshape(shape),
           "T_last": obj.last_T.cpu().numpy()}
    obj.close()
    return out


if __name__ == "__main__":  # pragma: no cover - manual run
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--prec", default="c128")
    a = ap.parse_args()
    r = run_lbfgsb(MuxDevice(), iters=a.iters, prec=a.prec,
                   callback=lambda k, f: print(f"eval {k}: F = {f:.6f}", flush=True))
    print(json.dumps({k: v for k, v in r.items() if k not in ("theta", "T_last")}))
