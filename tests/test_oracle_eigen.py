"""Pins of the nonlinear-eigenproblem oracle (oracle/eigen.py; Section 4.4,
eqs. system_qusi and system_normal; Section 6.3 Example 2, eq. ex3d2).

Independent references: the closed-form ground state of the discrete
Laplacian (sine products, eigenvalue sum_a 4 h_a^-2 sin^2(pi/(2(n_a+1))));
the constant eigenfunction of a Neumann problem with a constant potential,
whose eigenvalue is c + b / |Omega| exactly; first-order perturbation theory
in the cubic coefficient; and scipy's root finder on the eigenpair equations
(A_h U + f(U) = lam U, <U, U>_M = 1) with lam as an unknown.
"""

import math

import numpy as np
import pytest
import scipy.optimize

import synth
from oracle import eigen as eg


def sine_ground_state(shape, length):
    """Normalised (h^d-weighted) product of sin(pi i/(n+1)) and its eigenvalue."""
    u = np.ones(shape)
    lam = 0.0
    hvol = 1.0
    for ax, n in enumerate(shape):
        h = length / (n + 1)
        hvol *= h
        s = np.sin(math.pi * np.arange(1, n + 1) / (n + 1))
        bshape = [1] * len(shape)
        bshape[ax] = n
        u = u * s.reshape(bshape)
        lam += 4.0 / (h * h) * math.sin(math.pi / (2 * (n + 1))) ** 2
    return u / math.sqrt(hvol * float(np.sum(u * u))), lam


@pytest.mark.parametrize("shape,length", [((9, 11), 1.0), ((7, 8, 9), 16.0)])
def test_linear_problem_finds_the_closed_form_ground_state(shape, length):
    """b = 0, no potential, fixed beta > 0: the step is inverse iteration,
    which converges to the lowest eigenpair of A_h."""
    rng = np.random.default_rng(1)
    u0 = np.abs(rng.standard_normal(shape)) + 1.0
    out = eg.eigen_solve(u0, "dirichlet", length, cub=0.0, beta=1.0 / length ** 2,
                         rtol=1e-12, max_iter=5000)
    assert out["converged"]
    u_ref, lam_ref = sine_ground_state(shape, length)
    assert out["lam"] == pytest.approx(lam_ref, rel=1e-11)
    u = out["u"] * np.sign(out["u"].sum())
    assert np.abs(u - u_ref).max() <= 1e-9 * np.abs(u_ref).max()


@pytest.mark.parametrize("shape,length", [((6, 9), 2.0), ((5, 6, 7), 3.0)])
def test_neumann_constant_state_with_constant_potential(shape, length):
    """With Neumann data and V = c the constant u = |Omega|^-1/2 solves
    -Lap u + b u^3 + c u = lam u with lam = c + b / |Omega| (|Omega| = L^d:
    the trapezoid weights integrate constants exactly)."""
    b, c = 3.0, 2.5
    vol = length ** len(shape)
    rng = np.random.default_rng(2)
    u0 = 1.0 + 0.05 * rng.standard_normal(shape)
    pot = np.full(shape, c)
    out = eg.eigen_solve(u0, "neumann", length, cub=b, pot=pot, rtol=1e-12, max_iter=2000)
    assert out["converged"]
    assert out["lam"] == pytest.approx(c + b / vol, rel=1e-11)
    np.testing.assert_allclose(out["u"], 1.0 / math.sqrt(vol), rtol=1e-9)


def test_first_order_perturbation_in_the_cubic_coefficient():
    """lam(b) = lam(0) + b <u0^3, u0>_M + O(b^2) for the linear ground state u0
    (Dirichlet): the slope pins the cubic term and the h^d-weighted norm."""
    shape, length = (7, 9), 2.0
    u_ref, lam0 = sine_ground_state(shape, length)
    hvol = (length / 8) * (length / 10)
    s4 = hvol * float(np.sum(u_ref ** 4))
    errs = []
    for b in (0.02, 0.04):
        out = eg.eigen_solve(u_ref, "dirichlet", length, cub=b, beta=1.0, rtol=1e-13,
                             max_iter=5000)
        assert out["converged"]
        errs.append(abs((out["lam"] - lam0) / b - s4))
    assert errs[0] <= 1e-2 * s4
    assert 1.5 < errs[1] / errs[0] < 2.5  # the remainder is O(b)


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_fixed_point_solves_the_eigenpair_equations(bc):
    """Section 6.3 Example 2's nonlinearity and potential on a tiny grid: the
    midpoint iteration's (U, lam) is the root that scipy's Powell hybrid
    method finds for (A_h U + f(U) - lam U, <U, U>_M - 1) from a rough start."""
    n, length = 5, 16.0
    v, u0 = synth.schrodinger_3d(n)
    out = eg.eigen_solve(u0, bc, length, cub=1600.0, pot=v, rtol=1e-13, max_iter=5000)
    assert out["converged"]
    w = eg.mass_weights(u0.shape, bc, length)
    shape = u0.shape

    def eqs(z):
        u, lam = z[:-1].reshape(shape), z[-1]
        r = eg.apply_laplacian(u, bc, length) + 1600.0 * u ** 3 + v * u - lam * u
        return np.concatenate([r.ravel(), [float(np.sum(w * u * u)) - 1.0]])

    start = np.concatenate([(out["u"] * (1.0 + 0.01 * np.cos(np.arange(u0.size)).reshape(shape))).ravel(),
                            [out["lam"] * 1.01]])
    sol = scipy.optimize.root(eqs, start, method="hybr", options={"xtol": 1e-14})
    assert sol.success, sol.message
    assert sol.x[-1] == pytest.approx(out["lam"], rel=1e-10)
    np.testing.assert_allclose(sol.x[:-1].reshape(shape), out["u"], atol=1e-9 * np.abs(out["u"]).max())


def test_midpoint_and_fixed_shift_reach_the_same_eigenpair():
    """The shift changes the path, not the fixed point (Section 6.3 Example 2
    at 15^3; the midpoint takes 440 solves, beta = 200 takes 544, while fixed
    shifts of 60 or 100 drift to another state and do not converge)."""
    v, u0 = synth.schrodinger_3d(15)
    a = eg.eigen_solve(u0, "dirichlet", 16.0, cub=1600.0, pot=v, rtol=1e-11, max_iter=3000)
    b = eg.eigen_solve(u0, "dirichlet", 16.0, cub=1600.0, pot=v, beta=200.0, rtol=1e-11,
                       max_iter=6000)
    assert a["converged"] and b["converged"]
    assert a["lam"] == pytest.approx(b["lam"], rel=1e-10)
    np.testing.assert_allclose(a["u"], b["u"], atol=1e-8 * np.abs(a["u"]).max())
