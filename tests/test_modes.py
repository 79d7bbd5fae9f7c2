"""Pins of the port-mode solver (modes.column_modes): the discrete Dirichlet
eigenpairs of a homogeneous column in closed form, the parity and node count
of the modes of a symmetric guide, orthonormality, and the guided count of a
guide below and above the cut-off."""
import numpy as np
import pytest

from paper_2307_05388_amd.modes import column_modes, guided_count


@pytest.mark.parametrize("n,eps,omega", [(20, 2.085, 0.3), (57, 12.11, 0.1621467)])
def test_homogeneous_column_closed_form(n, eps, omega):
    beta2, prof = column_modes(np.full(n, eps), omega, 4)
    k = np.arange(1, 5)
    want = omega ** 2 * eps - 4.0 * np.sin(np.pi * k / (2 * (n + 1))) ** 2
    assert np.allclose(beta2, want, atol=1e-13)
    j = np.arange(n)
    for i, kk in enumerate(k):
        v = np.sin(np.pi * kk * (j + 1) / (n + 1))
        v /= np.linalg.norm(v)
        assert abs(abs(np.dot(prof[i], v)) - 1.0) < 1e-12


def test_symmetric_guide_parity_and_nodes():
    col = np.full(101, 2.085)
    col[41:60] = 12.11          # centred, odd width: symmetric about row 50
    beta2, prof = column_modes(col, 0.16, 3)
    for m in range(3):
        assert np.allclose(prof[m][::-1], (-1) ** m * prof[m], atol=1e-10)
        big = prof[m][np.abs(prof[m]) > 1e-3 * np.abs(prof[m]).max()]
        assert np.count_nonzero(np.diff(np.sign(big))) == m
    assert np.allclose(prof @ prof.T, np.eye(3), atol=1e-12)
    assert np.all(np.diff(beta2) < 0)


def test_guided_count_cut_off():
    om = 2 * np.pi * 40 / 1550.0
    narrow = np.full(160, 2.085)
    narrow[78:83] = 12.11       # 200 nm at 40 nm cells: single mode
    wide = np.full(160, 2.085)
    wide[71:89] = 12.11         # 720 nm: three guided modes
    assert guided_count(column_modes(narrow, om, 3)[0], om, 2.085) == 1
    assert guided_count(column_modes(wide, om, 4)[0], om, 2.085) == 3
