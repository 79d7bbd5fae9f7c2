"""Seeded synthetic device workloads for the 2D TM FDFD inverse-design problem.

This module only *describes inputs*: grid sizes, wavelengths, permittivity maps,
source vectors and objective vectors.  It holds none of the solver's arithmetic
(no operator assembly, no factorization, no PML) and is the one module shared by
the GPU library's callers and by the CPU oracle used in tests.

The paper (Sec. III-V) designs silicon devices in a silica background with
wavelengths between 1.50 and 1.60 um.  Its device geometries, port modes and
design maps are not published, so the workloads here are synthetic stand-ins of
the same kind: a silica background (eps_r = 2.085), silicon strips and
waveguides (eps_r = 12.11) and a square design region whose permittivity is drawn
i.i.d. uniform in [2.085, 12.11] (a continuous design before binarisation).

Conventions
-----------
* Grid of ``nx * ny`` cells, Ez at cell centres, linear index ``n = i + nx * j``
  (``i`` along x, fastest).  Arrays of grid values have shape ``(ny, nx)``.
* Lengths are measured in cells; with c = 1 the normalised angular frequency is
  ``omega = 2 * pi * dx / lambda``.
* ``b`` has layout ``[nsys][nrhs][N]`` complex128, one system per wavelength and
  one right-hand side per source profile.
* Random draws use ``numpy.random.default_rng([seed, t])`` (PCG64) with ``t`` the
  design-iteration index; the design block is filled row-major (j outer, i inner).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

EPS_SIO2 = 2.085
EPS_SI = 12.11


@dataclass(frozen=True)
class Problem:
    name: str
    nx: int
    ny: int
    npml: int
    dx_nm: float
    wavelengths_um: tuple
    # rectangles [i0, i1) x [j0, j1) filled with silicon before the design block
    strips: tuple = ()
    # design block [i0, i1) x [j0, j1)
    design: tuple = (0, 0, 0, 0)
    # source column and profile kinds ("line", "gauss", "alt_gauss")
    src_col: int = 0
    src_profiles: tuple = ("line",)
    # objective column and Gaussian half-width (cells)
    obj_col: int = 0
    width_cells: float = 5.0
    iterations: int = 1
    description: str = ""
    extra: dict = field(default_factory=dict, compare=False, hash=False)

    @property
    def N(self) -> int:
        return self.nx * self.ny

    @property
    def nsys(self) -> int:
        return len(self.wavelengths_um)

    @property
    def nrhs(self) -> int:
        return len(self.src_profiles)

    @property
    def design_shape(self) -> tuple:
        i0, i1, j0, j1 = self.design
        return (j1 - j0, i1 - i0)


def omegas(p: Problem) -> np.ndarray:
    """Normalised angular frequency per system: 2*pi*dx/lambda (cells, c = 1)."""
    lam_nm = np.asarray(p.wavelengths_um, dtype=np.float64) * 1000.0
    return 2.0 * math.pi * p.dx_nm / lam_nm


def _centred_rows(ny: int, width: int) -> tuple:
    j0 = ny // 2 - width // 2
    return (j0, j0 + width)


def make_problem(name: str) -> Problem:
    """The five synthetic workloads (small case, plain method, differentiation,
    batched multiplexer, large footprint)."""
    if name == "small60":
        # 60x60 with 10-cell PML, dx = 50 nm, lambda = 1.55 um; 10-cell strip,
        # 20x20 design block, unit line source at x = 15.
        return Problem("small60", 60, 60, 10, 50.0, (1.55,),
                       strips=((0, 60, 25, 35),), design=(20, 40, 20, 40),
                       src_col=15, src_profiles=("line",), obj_col=45,
                       width_cells=5.0, iterations=1,
                       description="60x60, 10-cell PML, dx=50nm, lambda=1.55um, complex128")
    if name == "plain300":
        r = _centred_rows(300, 12)
        return Problem("plain300", 300, 300, 20, 40.0, (1.55,),
                       strips=((0, 300) + r,), design=(100, 200, 100, 200),
                       src_col=25, src_profiles=("line",), obj_col=275,
                       width_cells=6.0, iterations=20,
                       description="300x300 (N=90,000), 20-cell PML, dx=40nm, 100x100 design re-drawn each step")
    if name == "diff500":
        r = _centred_rows(500, 12)
        return Problem("diff500", 500, 500, 20, 40.0, (1.55,),
                       strips=((0, 175) + r, (325, 500) + r), design=(175, 325, 175, 325),
                       src_col=25, src_profiles=("gauss",), obj_col=475,
                       width_cells=6.0, iterations=1,
                       description="500x500 (N=250,000), 150x150 design, in/out strip guides")
    if name == "mux400":
        r = _centred_rows(400, 12)
        lams = tuple(float(v) for v in np.linspace(1.50, 1.60, 8))
        return Problem("mux400", 400, 400, 20, 40.0, lams,
                       strips=((0, 140) + r, (260, 400) + r), design=(140, 260, 140, 260),
                       src_col=25, src_profiles=("gauss", "alt_gauss"), obj_col=375,
                       width_cells=6.0, iterations=1,
                       description="400x400, 8 wavelengths 1.50-1.60um x 2 source profiles")
    if name == "large2000":
        r = _centred_rows(2000, 12)
        return Problem("large2000", 2000, 2000, 40, 40.0, (1.55,),
                       strips=((0, 2000) + r,), design=(200, 1800, 200, 1800),
                       src_col=45, src_profiles=("line",), obj_col=1955,
                       width_cells=6.0, iterations=10,
                       description="2000x2000 (N=4,000,000), 40-cell PML, 1600x1600 design")
    raise ValueError(f"unknown problem {name!r}")


def footprint_problem(side: int) -> Problem:
    """One point of the footprint sweep (Sec. V): a square domain of side
    cells at dx = 25 nm whose outer 1 um (40 cells) on each side is margin,
    20 cells of it PML; the design block is the footprint inside the margins
    (side - 80 cells, e.g. 240 cells = a 4 x 4 um footprint, 3480 = 85 x 85
    um), with a 0.5 um silicon input and output guide centred in y through
    the margins.  lambda = 1.55 um."""
    if side < 100:
        raise ValueError("side must be at least 100 cells")
    margin, npml = 40, 20
    r = _centred_rows(side, 20)
    return Problem(f"footprint{side}", side, side, npml, 25.0, (1.55,),
                   strips=((0, margin) + r, (side - margin, side) + r),
                   design=(margin, side - margin, margin, side - margin),
                   src_col=npml + 5, src_profiles=("gauss",), obj_col=side - npml - 6,
                   width_cells=10.0, iterations=1,
                   description=f"{side}x{side} at 25nm: {(side - 2 * margin) * 0.025:g} um footprint + 1 um margins")


def custom_problem(nx: int, ny: int, npml: int, dx_nm: float = 50.0,
                   wavelengths_um=(1.55,), design=None, src_profiles=("line",),
                   name: str = "custom") -> Problem:
    """A small problem of the same structure as the 60x60 case, for tests at any size."""
    if design is None:
        di = max(1, nx // 3)
        dj = max(1, ny // 3)
        design = (di, nx - di, dj, ny - dj)
    width = max(2, ny // 6)
    r = _centred_rows(ny, width)
    return Problem(name, nx, ny, npml, dx_nm, tuple(wavelengths_um),
                   strips=((0, nx) + r,), design=tuple(design),
                   src_col=min(nx - 1, npml + max(1, nx // 12)),
                   src_profiles=tuple(src_profiles),
                   obj_col=max(0, nx - npml - max(1, nx // 12) - 1),
                   width_cells=max(1.0, ny / 12.0), iterations=1)


def base_eps(p: Problem) -> np.ndarray:
    """Background silica with silicon strips, shape (ny, nx) float64."""
    eps = np.full((p.ny, p.nx), EPS_SIO2, dtype=np.float64)
    for (i0, i1, j0, j1) in p.strips:
        eps[j0:j1, i0:i1] = EPS_SI
    return eps


def design_values(p: Problem, t: int = 0, seed: int = 0) -> np.ndarray:
    """Design-block permittivity for iteration t: i.i.d. uniform [2.085, 12.11]."""
    rng = np.random.default_rng([seed, t])
    dh, dw = p.design_shape
    return rng.uniform(EPS_SIO2, EPS_SI, size=(dh, dw))


def design_eps(p: Problem, t: int = 0, seed: int = 0) -> np.ndarray:
    """Full permittivity map (ny, nx) with the design block drawn for iteration t."""
    eps = base_eps(p)
    i0, i1, j0, j1 = p.design
    eps[j0:j1, i0:i1] = design_values(p, t, seed)
    return eps


def design_index(p: Problem) -> np.ndarray:
    """Linear grid indices n = i + nx*j of the design block, row-major."""
    i0, i1, j0, j1 = p.design
    jj, ii = np.meshgrid(np.arange(j0, j1), np.arange(i0, i1), indexing="ij")
    return (ii + p.nx * jj).reshape(-1)


def _profile(p: Problem, kind: str) -> np.ndarray:
    """Source profile along y on a single column, zero inside the y-PML."""
    j = np.arange(p.ny, dtype=np.float64)
    jc = (p.ny - 1) / 2.0
    inside = (j >= p.npml) & (j < p.ny - p.npml)
    if kind == "line":
        prof = np.ones(p.ny)
    elif kind == "gauss":
        prof = np.exp(-((j - jc) / p.width_cells) ** 2)
    elif kind == "alt_gauss":
        prof = np.sign(j - jc) * np.exp(-((j - jc) / p.width_cells) ** 2)
    else:
        raise ValueError(kind)
    return np.where(inside, prof, 0.0)


def sources(p: Problem) -> np.ndarray:
    """Right-hand sides b, shape (nsys, nrhs, N) complex128 (b = J)."""
    b = np.zeros((p.nsys, p.nrhs, p.ny, p.nx), dtype=np.complex128)
    for r, kind in enumerate(p.src_profiles):
        b[:, r, :, p.src_col] = _profile(p, kind)
    return b.reshape(p.nsys, p.nrhs, p.N)


def objective_vector(p: Problem) -> np.ndarray:
    """Mode-overlap vector c (N,) complex128: Gaussian across the output column."""
    c = np.zeros((p.ny, p.nx), dtype=np.complex128)
    c[:, p.obj_col] = _profile(p, "gauss")
    return c.reshape(p.N)


def fd_pixels(p: Problem, count: int = 32, seed: int = 0) -> np.ndarray:
    """Design pixels (linear grid indices) for finite-difference gradient checks."""
    rng = np.random.default_rng([seed, 99])
    idx = design_index(p)
    return np.sort(rng.choice(idx, size=min(count, idx.size), replace=False))


def random_complex(shape, seed: int) -> np.ndarray:
    """Seeded complex normal array, for reciprocity and parity tests."""
    rng = np.random.default_rng([seed, 7])
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
