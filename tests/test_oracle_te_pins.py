"""Pins of the oracle's TE (Hz) variant against what the mathematics and the
physics fix, independent of the oracle's own code paths:

  reduction   with a uniform permittivity the TE operator is exactly the TM
              operator divided by eps (PML included)
  symmetry    S A_TE is complex symmetric (S = diag(sx_c sy_c)) for any eps
  solves      the banded LU against LAPACK on the dense matrix, forward and
              transposed
  gradient    the face-by-face adjoint gradient against central differences
              of F, on pixels in the interior, on the grid edge and in a
              corner, two wavelengths x two sources
  physics     the reflection of a guided y-mode at a permittivity step,
              from a 2D solve with PML: equal to the exact solution of the
              discrete equations of the two cells at the step (two unknowns,
              R and T), close to the continuum Fresnel coefficient of an Hz
              field (k/eps continuous across the step) and far from that of
              an Ez field (k continuous), and closer to the continuum the
              finer the grid
Each planted mistake (on the CPU, in a copy of an oracle function) fails a pin.
"""
import numpy as np
import pytest

from oracle import fdfd_oracle as o


def _eps(ny, nx, seed):
    return np.random.default_rng([seed, 17]).uniform(2.085, 12.11, size=(ny, nx))


def test_uniform_eps_reduces_to_tm_over_eps():
    nx, ny, eps0 = 11, 9, 4.7
    eps = np.full((ny, nx), eps0)
    for om in (0.25, 0.6):
        te = o.dense_matrix(o.operator_coefficients_te(nx, ny, 3, 2, om, eps))
        tm = o.dense_matrix(o.operator_coefficients(nx, ny, 3, 2, om, eps))
        assert np.abs(te - tm / eps0).max() <= 1e-15 * np.abs(tm).max()


@pytest.mark.parametrize("npml", [(0, 0), (3, 2)])
def test_symmetrised_te_operator_is_symmetric(npml):
    nx, ny = 10, 8
    eps = _eps(ny, nx, 1)
    om = 0.4
    A = o.dense_matrix(o.operator_coefficients_te(nx, ny, npml[0], npml[1], om, eps))
    S = o.symmetrizer(nx, ny, npml[0], npml[1], om)
    SA = S[:, None] * A
    assert np.abs(SA - SA.T).max() <= 1e-15 * np.abs(SA).max()
    if npml == (0, 0):
        assert np.abs(A - A.T).max() <= 1e-15 * np.abs(A).max()
    else:  # the PML makes A itself non-symmetric
        assert np.abs(A - A.T).max() > 1e-3 * np.abs(A).max()


def test_band_solves_match_lapack():
    nx, ny = 9, 8
    eps = _eps(ny, nx, 2)
    coef = o.operator_coefficients_te(nx, ny, 2, 2, 0.5, eps)
    A = o.dense_matrix(coef)
    lu = o.BandLU(o.band_matrix(coef))
    b = np.random.default_rng([2, 5]).standard_normal((2, nx * ny)) + 1j
    for tr in (False, True):
        x = lu.solve(b, transpose=tr)
        want = np.linalg.solve(A.T if tr else A, b.T).T
        assert np.abs(x - want).max() <= 1e-12 * np.abs(want).max()


def _fd_problem():
    nx, ny, npml = 16, 13, 3
    eps = _eps(ny, nx, 3)
    omegas = np.array([0.45, 0.52])
    b = np.zeros((2, 2, ny, nx), dtype=np.complex128)
    b[:, 0, 2:11, 4] = 1.0
    b[:, 1, 6, 7] = 1.0 - 0.5j
    c = np.zeros((ny, nx), dtype=np.complex128)
    c[3:10, 11] = np.exp(-((np.arange(3, 10) - 6.0) / 2.0) ** 2)
    return nx, ny, npml, eps, omegas, b.reshape(2, 2, -1), c.reshape(-1)


def _F(nx, ny, npml, eps, omegas, b, c, pol="te"):
    return float(o.design_iteration(nx, ny, npml, omegas, eps, b, c=c, pol=pol)["F"].sum())


def test_gradient_matches_central_differences():
    nx, ny, npml, eps, omegas, b, c = _fd_problem()
    g = o.design_iteration(nx, ny, npml, omegas, eps, b, c=c, pol="te")["grad"].sum(axis=0)
    # h = 1e-3: the truncation error (h^2) is ~1e-9 relative here, while
    # smaller steps lose digits to cancellation on the small edge derivatives
    h = 1e-3
    # interior, next to the sources, the grid edge and a corner
    for (j, i) in ((6, 8), (4, 5), (0, 7), (ny - 1, nx - 1), (6, 0), (9, 12)):
        ep, em = eps.copy(), eps.copy()
        ep[j, i] += h
        em[j, i] -= h
        fd = (_F(nx, ny, npml, ep, omegas, b, c) - _F(nx, ny, npml, em, omegas, b, c)) / (2 * h)
        an = g[j * nx + i]
        assert abs(an - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (j, i, an, fd)


# -- physics: reflection at a permittivity step ----------------------------------

def _mode(ny):
    v = np.sin(np.pi * (np.arange(ny) + 1) / (ny + 1))
    kappa = 2.0 - 2.0 * np.cos(np.pi / (ny + 1))   # -D_yy eigenvalue of v, Dirichlet walls
    return v, kappa


def _step_reflection_2d(omega, eps1, eps2, scale=1, pol="te", coef_fn=None):
    """R of the lowest mode of a guide along y (Dirichlet walls in x, PML at
    both ends in y) at the step between rows j0 - 1 and j0, from a 2D solve
    (the banded oracle's band is nx wide): the mode amplitude between source
    and step is fitted to A e^{ik j} + B e^{-ik j} and
    R = B e^{-ik c} / (A e^{ik c}), c = j0 - 1/2.  scale refines the grid
    (omega / scale, every length in cells times scale)."""
    nx, ny, npml, j0 = 16 * scale - 1, 480 * scale, 60 * scale, 240 * scale
    eps = np.full((ny, nx), eps1)
    eps[j0:, :] = eps2
    v, kappa = _mode(nx)
    coef = (coef_fn or o.operator)(pol, nx, ny, 0, npml, omega, eps)
    b = np.zeros((ny, nx), dtype=np.complex128)
    b[npml + 20 * scale, :] = v
    x = o.BandLU(o.band_matrix(coef)).solve(b.reshape(-1)).reshape(ny, nx)
    amp = (x * v[None, :]).sum(axis=1) / (v ** 2).sum()
    # discrete wavenumber in medium 1: 2 cos k = 2 + kappa - omega^2 eps1
    k1 = np.arccos(1.0 + (kappa - omega ** 2 * eps1) / 2.0)
    j1, j2 = j0 - 90 * scale, j0 - 45 * scale
    M = np.array([[np.exp(1j * k1 * j1), np.exp(-1j * k1 * j1)], [np.exp(1j * k1 * j2), np.exp(-1j * k1 * j2)]])
    A, B = np.linalg.solve(M, amp[[j1, j2]])
    ctr = j0 - 0.5
    return B * np.exp(-1j * k1 * ctr) / (A * np.exp(1j * k1 * ctr))


def _step_reflection_exact(omega, eps1, eps2, ny=15):
    """The same R from the discrete TE equations of the two cells at the step
    (h_i = e^{ik1 i} + R e^{-ik1 i} up to cell i0 - 1, T e^{ik2 i} from i0;
    the face between them carries (eps1 + eps2) / 2), with i0 = 0."""
    _, kappa = _mode(ny)
    k1 = np.arccos(1.0 + (kappa - omega ** 2 * eps1) / 2.0)
    k2 = np.arccos(1.0 + (kappa - omega ** 2 * eps2) / 2.0)
    em = 0.5 * (eps1 + eps2)
    inc = lambda i: np.exp(1j * k1 * i)
    ref = lambda i: np.exp(-1j * k1 * i)
    tr = lambda i: np.exp(1j * k2 * i)
    # cell -1 (medium 1):  (h0 - h-1)/em - (h-1 - h-2)/eps1 + (omega^2 - kappa/eps1) h-1 = 0
    # cell  0 (medium 2):  (h1 - h0)/eps2 - (h0 - h-1)/em + (omega^2 - kappa/eps2) h0 = 0
    d1 = omega ** 2 - kappa / eps1
    d2 = omega ** 2 - kappa / eps2
    row1 = lambda f: -f(-1) / em - (f(-1) - f(-2)) / eps1 + d1 * f(-1)
    row2 = lambda f: f(-1) / em
    M = np.array([[row1(ref), tr(0) / em],
                  [row2(ref), (tr(1) - tr(0)) / eps2 - tr(0) / em + d2 * tr(0)]])
    rhs = -np.array([row1(inc), row2(inc)])
    R, _ = np.linalg.solve(M, rhs)
    return R * np.exp(1j * k1)   # referred to the step's plane, between cells -1 and 0


def _fresnel(omega, eps1, eps2, ny=15):
    """Continuum reflection of the mode at a step: Hz (k/eps continuous) and Ez
    (k continuous), with the continuum wavenumbers of the same guide."""
    ky = np.pi / (ny + 1)
    k1 = np.sqrt(omega ** 2 * eps1 - ky ** 2)
    k2 = np.sqrt(omega ** 2 * eps2 - ky ** 2)
    te = (k1 / eps1 - k2 / eps2) / (k1 / eps1 + k2 / eps2)
    tm = (k1 - k2) / (k1 + k2)
    return te, tm


def test_step_reflection_is_that_of_an_hz_field():
    eps1, eps2 = 2.085, 12.11
    errs = []
    for scale in (1, 2):
        omega, width = 0.2 / scale, 16 * scale - 1
        r2d = _step_reflection_2d(omega, eps1, eps2, scale=scale)
        rex = _step_reflection_exact(omega, eps1, eps2, ny=width)
        te, tm = _fresnel(omega, eps1, eps2, ny=width)
        assert abs(r2d - rex) < 1e-5, (omega, r2d, rex)        # PML reflection level
        assert abs(r2d - te) < 0.03, (omega, r2d, te)
        assert abs(r2d - tm) > 0.5, (omega, r2d, tm)           # Ez: the opposite sign here
        errs.append(abs(r2d - te))
    assert errs[1] < errs[0] / 3                                # second order in the cell size


# -- planted mistakes ---------------------------------------------------------------

def test_planted_eps_outside_the_derivative_fails_the_reflection_pin():
    """Permittivity multiplying the whole Laplacian row instead of sitting on
    the faces (the TM-like placement) gives the wrong interface condition."""
    def bad(pol, nx, ny, px, py, om, eps):
        coef = o.operator_coefficients(nx, ny, px, py, om, np.ones_like(eps))
        e = np.asarray(eps, dtype=np.float64)
        out = {k: coef[k] / e for k in ("xm", "xp", "ym", "yp")}
        out["diag"] = om ** 2 - (out["xm"] + out["xp"] + out["ym"] + out["yp"])
        out.update(nx=nx, ny=ny)
        return out
    r = _step_reflection_2d(0.2, 2.085, 12.11, coef_fn=bad)
    assert abs(r - _step_reflection_exact(0.2, 2.085, 12.11)) > 1e-2


def test_planted_full_weight_on_interior_faces_fails_central_differences():
    nx, ny, npml, eps, omegas, b, c = _fd_problem()
    out = o.design_iteration(nx, ny, npml, omegas, eps, b, c=c, pol="te")
    coef = o.operator_coefficients_te(nx, ny, npml, npml, omegas[0], eps)
    good = o.gradient_te(coef, eps, out["x"][0], out["lam"][0]).sum(axis=0)
    # the same faces with weight 1 for both cells (a dropped 1/2)
    ex, ey = o.face_permittivity(eps)
    bad = good.copy().reshape(ny, nx)
    X, L = out["x"][0].reshape(2, ny, nx), out["lam"][0].reshape(2, ny, nx)
    ap, aq = coef["xp"][:, :-1], coef["xm"][:, 1:]
    t = -(ap * L[:, :, :-1] * (X[:, :, 1:] - X[:, :, :-1]) + aq * L[:, :, 1:] * (X[:, :, :-1] - X[:, :, 1:])) / ex[:, 1:nx]
    g = (-2.0 * np.real(t)).sum(axis=0)
    bad[:, :-1] += 0.5 * g
    bad[:, 1:] += 0.5 * g
    h, (j, i) = 1e-5, (6, 8)
    ep, em = eps.copy(), eps.copy()
    ep[j, i] += h
    em[j, i] -= h
    fd0 = (_F(nx, ny, npml, ep, omegas[:1], b[:1], c) - _F(nx, ny, npml, em, omegas[:1], b[:1], c)) / (2 * h)
    assert abs(good[j * nx + i] - fd0) <= 1e-6 * abs(fd0)
    assert abs(bad[j, i] - fd0) > 1e-3 * abs(fd0)


def test_planted_edge_face_halved_fails_central_differences():
    """A grid-edge face given half its cell's permittivity in the operator
    (an interior-face rule applied at the edge) no longer matches the
    gradient's edge terms."""
    nx, ny, npml, eps, omegas, b, c = _fd_problem()
    orig = o.face_permittivity

    def halved(e):
        ex, ey = orig(e)
        ex = ex.copy()
        ex[:, 0] *= 0.5
        return ex, ey
    o.face_permittivity = halved
    try:
        g = o.design_iteration(nx, ny, npml, omegas, eps, b, c=c, pol="te")["grad"].sum(axis=0)
        h, (j, i) = 1e-5, (6, 0)
        ep, em = eps.copy(), eps.copy()
        ep[j, i] += h
        em[j, i] -= h
        fd = (_F(nx, ny, npml, ep, omegas, b, c) - _F(nx, ny, npml, em, omegas, b, c)) / (2 * h)
    finally:
        o.face_permittivity = orig
    assert abs(g[j * nx + i] - fd) > 1e-3 * abs(fd)
