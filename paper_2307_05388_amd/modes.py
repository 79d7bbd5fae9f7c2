"""Waveguide port modes for the inverse-design loop (paper Sec. IV: the mode
multiplexer is driven by the TE0, TE1 and TE2 modes of its input guide).

The modes of a straight guide along x are the transverse eigenvectors of the
same discretisation as the 2D operator: on one grid column with permittivity
eps_j (j = 0 .. ny-1, Dirichlet E = 0 outside),
    E_{j+1} - 2 E_j + E_{j-1} + omega^2 eps_j E_j = beta^2 E_j,
a real symmetric tridiagonal eigenproblem.  Guided modes are the eigenvectors
with the largest beta^2 (above omega^2 eps_cladding); mode k has k nodes.
This prepares source and overlap vectors once per wavelength on the host; it
is not part of the solve.
"""
from __future__ import annotations

import numpy as np


def column_modes(eps_col, omega, nmodes):
    """The nmodes modes with the largest beta^2 of one grid column.

    eps_col: (ny,) permittivity along the column.  Returns (beta2, profiles)
    with profiles (nmodes, ny), each of unit 2-norm, sign fixed so that its
    first nonzero lobe is positive, in decreasing beta^2 (mode 0 first)."""
    eps_col = np.asarray(eps_col, dtype=np.float64)
    n = eps_col.size
    main = omega ** 2 * eps_col - 2.0
    off = np.ones(n - 1)
    T = np.diag(main) + np.diag(off, 1) + np.diag(off, -1)
    w, v = np.linalg.eigh(T)
    order = np.argsort(w)[::-1][:nmodes]
    beta2 = w[order]
    prof = v[:, order].T.copy()
    for k in range(prof.shape[0]):
        nz = np.nonzero(np.abs(prof[k]) > 1e-6 * np.abs(prof[k]).max())[0]
        if prof[k, nz[0]] < 0:
            prof[k] = -prof[k]
    return beta2, prof


def guided_count(beta2, omega, eps_clad):
    """How many of the modes are guided (beta^2 above the cladding's light line
    of the same discretisation, omega^2 eps_clad - 4 sin^2(0) = omega^2 eps_clad)."""
    return int(np.sum(np.asarray(beta2) > omega ** 2 * eps_clad))
