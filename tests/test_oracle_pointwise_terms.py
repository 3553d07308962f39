"""Pins of the oracle's general pointwise term lambda U + q U^2 + b U^3 + V U
(the model of Section 2 with f(x, u) = b u^3 + q u^2 + V(x) u - f_src;
Section 6.3, Example 1, eq. ex3d1 has lambda = b = 10 and a potential V;
Section 6.2, Example 2, eq. 2dex has q = -1), for both boundary types.

Each pin goes through something other than the oracle's own formulas: the
continuous manufactured solution (truncation error O(h^2)), central
differences of the residual (the Jacobian diagonal), scipy's root finder (the
fixed point of the quasi-Newton loop) and mesh refinement of the discrete
solution.
"""

import numpy as np
import pytest
import scipy.optimize

import synth
from oracle import neumann as nm
from oracle import operators as ops
from oracle import qn as oqn

A = B = 10.0


def _max_residual(n):
    u, f, v = synth.neumann_potential_3d(n, A, B)
    hs = nm.spacing(u.shape)
    return float(np.abs(nm.residual_cubic(u, f, hs, A, B, v)).max())


def test_e7_exact_solution_residual_is_second_order():
    """Sampled exact solution of eq. ex3d1: the discrete residual is the
    stencil's truncation error only, O(h^2) up to and including the boundary
    nodes (u is even about each face, so the mirrored ghost node is exact to
    O(h^2) too).  A dropped V, lambda or wrong b leaves an O(1) residual."""
    errs = [_max_residual(n) for n in (9, 17, 33)]
    for coarse, fine in zip(errs, errs[1:]):
        assert 3.5 < coarse / fine < 4.5, errs
    u, f, v = synth.neumann_potential_3d(17, A, B)
    hs = nm.spacing(u.shape)
    assert np.abs(nm.residual_cubic(u, f, hs, A, B, None)).max() > 10 * errs[1]
    assert np.abs(nm.residual_cubic(u, f, hs, A, 1.0, v)).max() > 10 * errs[1]
    assert np.abs(nm.residual_cubic(u, f, hs, 0.0, B, v)).max() > 10 * errs[1]


def _fd_diagonal(res, u, eps=1e-4):
    """d R_i / d U_i by central differences, one point at a time."""
    d = np.empty(u.size)
    flat = u.ravel()
    for i in range(u.size):
        up, um = flat.copy(), flat.copy()
        up[i] += eps
        um[i] -= eps
        d[i] = (res(up.reshape(u.shape)).ravel()[i] - res(um.reshape(u.shape)).ravel()[i]) / (2 * eps)
    return d.reshape(u.shape)


@pytest.mark.parametrize("bc,quad", [("dirichlet", 0.0), ("neumann", 0.0),
                                     ("dirichlet", -1.3), ("neumann", 0.8)])
def test_jacobian_diagonal_matches_central_differences(bc, quad):
    """fu = 3 b U^2 + 2 q U + lambda + V is the diagonal of dF^h/dU minus
    diag(A_h): for a cubic in U_i the central difference is exact up to b eps^2."""
    rng = np.random.default_rng(11)
    shape = (4, 5, 6)
    u = rng.standard_normal(shape)
    f = rng.standard_normal(shape)
    v = rng.uniform(0.0, 50.0, shape)
    lin, cub = 0.7, 2.5
    if bc == "dirichlet":
        res = lambda w: ops.residual_cubic(w, f, lin, cub, v, quad)
        adiag = ops.assemble_laplacian(shape).diagonal().reshape(shape)
        fu = ops.fu_cubic(u, lin, cub, v, quad)
    else:
        hs = nm.spacing(shape)
        res = lambda w: nm.residual_cubic(w, f, hs, lin, cub, v, quad)
        adiag = nm.assemble_laplacian(shape, hs).diagonal().reshape(shape)
        fu = nm.fu_cubic(u, lin, cub, v, quad)
    d = _fd_diagonal(res, u) - adiag
    np.testing.assert_allclose(d, fu, rtol=1e-7, atol=1e-7 * np.abs(adiag).max())


def _root(res, u0):
    sol = scipy.optimize.root(lambda x: res(x.reshape(u0.shape)).ravel(), u0.ravel(),
                              method="hybr", options={"xtol": 1e-14})
    assert sol.success, sol.message
    return sol.x.reshape(u0.shape)


def test_e7_quasi_newton_fixed_point_is_the_root():
    """The midpoint quasi-Newton loop from U_0 = 0 converges to the discrete
    solution that scipy's Powell hybrid method finds from the sampled exact
    solution (finite-difference Jacobian of the residual, no fu involved)."""
    u, f, v = synth.neumann_potential_3d(5, A, B)
    hs = nm.spacing(u.shape)
    root = _root(lambda w: nm.residual_cubic(w, f, hs, A, B, v), u)
    out = nm.qn_solve(f, hs, lin=A, cub=B, pot=v, rtol=1e-13, max_iter=500)
    assert out["converged"]
    assert np.linalg.norm(out["u"] - root) <= 1e-10 * np.linalg.norm(root)


def test_dirichlet_quasi_newton_with_pointwise_terms_is_the_root():
    """Same for Dirichlet data with lambda, b and V (random positive V)."""
    rng = np.random.default_rng(5)
    shape = (5, 6, 7)
    v = rng.uniform(0.0, 20.0, shape)
    f = 50.0 * rng.standard_normal(shape)
    res = lambda w: ops.residual_cubic(w, f, 1.5, 3.0, v)
    out = oqn.qn_solve(oqn.CUBIC, f[None], midpoint=True, rtol=1e-13, max_iter=500,
                       lin=1.5, cub=3.0, pot=v)
    assert out["converged"]
    root = _root(res, out["u"][0] + 0.01)
    assert np.linalg.norm(out["u"][0] - root) <= 1e-10 * np.linalg.norm(root)
    newton = oqn.newton_solve(oqn.CUBIC, f[None], lin=1.5, cub=3.0, pot=v)
    assert np.linalg.norm(newton[0] - root) <= 1e-10 * np.linalg.norm(root)


def test_e7_discrete_solution_converges_second_order():
    """The converged discrete solution approaches the exact one at O(h^2)."""
    errs = []
    for n in (9, 17, 33):
        u, f, v = synth.neumann_potential_3d(n, A, B)
        hs = nm.spacing(u.shape)
        out = nm.qn_solve(f, hs, lin=A, cub=B, pot=v, rtol=1e-12, max_iter=500)
        assert out["converged"]
        errs.append(float(np.abs(out["u"] - u).max()))
    for coarse, fine in zip(errs, errs[1:]):
        assert 3.3 < coarse / fine < 4.7, errs


def test_polynomial_perturbation_is_normalised_and_seeded():
    """Section 6.2 / 6.3 perturbation: max |p| = 1 over the nodes, a degree-4
    polynomial per variable (its fifth differences along x vanish), and the
    seed fixes it."""
    p = synth.polynomial_perturbation(12, 3, 7)
    assert abs(np.abs(p).max() - 1.0) < 1e-15
    assert np.abs(np.diff(p, n=5, axis=2)).max() < 1e-10
    np.testing.assert_array_equal(p, synth.polynomial_perturbation(12, 3, 7))
    assert not np.array_equal(p, synth.polynomial_perturbation(12, 3, 8))


def test_quadratic_term_manufactured_residual_is_second_order():
    """-Lap u - u^2 = f (the nonlinearity of Section 6.2, Example 2, eq. 2dex)
    with u = sin(pi x) sin(2 pi y) on (0, 1)^2, Dirichlet data: the residual of
    the sampled exact solution is the O(h^2) truncation error; a dropped or
    sign-flipped quadratic term leaves an O(1) residual."""
    errs = []
    for n in (15, 31, 63):
        x = synth.grid_coords(n)
        u = np.sin(2 * np.pi * x)[:, None] * np.sin(np.pi * x)[None, :]
        f = 5 * np.pi ** 2 * u - u * u
        errs.append(float(np.abs(ops.residual_cubic(u, f, 0.0, 0.0, None, -1.0)).max()))
        if n == 31:
            assert np.abs(ops.residual_cubic(u, f, 0.0, 0.0, None, 0.0)).max() > 0.5
            assert np.abs(ops.residual_cubic(u, f, 0.0, 0.0, None, 1.0)).max() > 0.5
    for coarse, fine in zip(errs, errs[1:]):
        assert 3.5 < coarse / fine < 4.5, errs
