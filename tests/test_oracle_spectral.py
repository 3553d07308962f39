"""Pins for oracle.spectral: closed-form sine eigenpairs of the FD stiffness matrix
(Section 3.2 eq. Sy, Section 4.2) against hand-derived values, a Jacobi eigensolver
and the defining identities."""

import math
import os

import numpy as np
import pytest

from oracle import spectral

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_stiffness_entries():
    s = spectral.stiffness_matrix(4)
    h2 = (1.0 / 5) ** 2
    assert s[0, 0] == pytest.approx(2 / h2)
    assert s[0, 1] == pytest.approx(-1 / h2)
    assert s[1, 0] == pytest.approx(-1 / h2)
    assert s[0, 2] == 0.0
    assert np.allclose(s, s.T)


def test_eigenpairs_match_hand_derived_n3():
    rows = np.loadtxt(os.path.join(GOLDEN, "eig_n3.txt"))
    t, lam = spectral.sine_eigenpairs(3)
    np.testing.assert_allclose(lam, rows[:, 0], rtol=1e-15)
    for k in range(3):
        v = rows[k, 1:]
        col = t[:, k]
        sign = np.sign(col @ v)
        np.testing.assert_allclose(sign * col, v, atol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 7, 31, 63, 255])
def test_eigen_identities(n):
    s = spectral.stiffness_matrix(n)
    t, lam = spectral.sine_eigenpairs(n)
    assert np.array_equal(t, t.T)  # exactly symmetric by integer reduction
    scale = lam.max()
    assert np.abs(s @ t - t * lam).max() / scale <= 1e-14
    assert np.abs(t.T @ t - np.eye(n)).max() <= 1e-14
    assert np.all(np.diff(lam) > 0)


@pytest.mark.parametrize("n", [5, 16, 31])
def test_closed_form_vs_jacobi(n):
    s = spectral.stiffness_matrix(n)
    lam_j, v = spectral.jacobi_eigh(s)
    t, lam = spectral.sine_eigenpairs(n)
    np.testing.assert_allclose(lam_j, lam, rtol=1e-13)
    for k in range(n):
        sign = math.copysign(1.0, float(v[:, k] @ t[:, k]))
        np.testing.assert_allclose(sign * v[:, k], t[:, k], atol=1e-12)


def test_jacobi_against_library_on_random_symmetric():
    a = np.random.default_rng(3).standard_normal((9, 9))
    a = a + a.T
    lam_j, v = spectral.jacobi_eigh(a)
    np.testing.assert_allclose(lam_j, np.linalg.eigvalsh(a), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(a @ v, v * lam_j, atol=1e-11)


def test_mass_weighted_diagonalisation_identity_mass():
    """Section 4.2 with M = I reproduces the closed-form spectrum."""
    n = 12
    t, lam, tinv = spectral.diagonalize(spectral.stiffness_matrix(n), np.ones(n))
    np.testing.assert_allclose(lam, spectral.sine_eigenpairs(n)[1], rtol=1e-13)
    np.testing.assert_allclose(tinv @ t, np.eye(n), atol=1e-13)


def test_mass_weighted_diagonalisation_general_mass():
    """H = M^-1 S = T Lambda T^-1 for a diagonal SPD M (Section 4.2)."""
    n = 10
    m = np.random.default_rng(5).uniform(0.5, 2.0, n)
    s = spectral.stiffness_matrix(n)
    t, lam, tinv = spectral.diagonalize(s, m)
    h = s / m[:, None]
    np.testing.assert_allclose(t @ np.diag(lam) @ tinv, h, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(tinv @ t, np.eye(n), atol=1e-13)
