"""Pins of the spectral element oracle (oracle/sem.py; Section 3.1 and the
remark on Gauss-Lobatto integration; Section 4.2).

Independent references: exactness of the (k+1)-point Gauss-Lobatto rule up
to degree 2k-1; H U = -u'' at the nodes for polynomials the space holds
(both boundary types); the continuous eigenvalues (m pi / L)^2, approached at
order 2k; a direct solve of the assembled Kronecker operator; and the
convergence order of the discrete solution of a manufactured problem.
"""

import math

import numpy as np
import pytest

from oracle import sem


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_gauss_lobatto_rule_is_exact_to_degree_2k_minus_1(k):
    x, w = sem.gauss_lobatto(k)
    assert x[0] == -1.0 and x[-1] == 1.0
    np.testing.assert_allclose(x, -x[::-1], atol=1e-15)
    for p in range(2 * k):
        exact = 2.0 / (p + 1) if p % 2 == 0 else 0.0
        assert abs(float(np.sum(w * x ** p)) - exact) <= 1e-14
    # and not beyond: degree 2k is integrated with an error (k >= 1)
    assert abs(float(np.sum(w * x ** (2 * k))) - 2.0 / (2 * k + 1)) > 1e-6


@pytest.mark.parametrize("k,elements", [(2, 3), (3, 4), (4, 2)])
def test_h_is_minus_second_derivative_on_polynomials(k, elements):
    """For u in the space with homogeneous data, (S U)_i = int -u'' psi_i is
    integrated exactly and lumped at node i, so H U = -u'' at the nodes."""
    length = 2.0
    x, m, h, *_ = sem.axis_operator(elements, k, length, "dirichlet")
    u = x * (length - x)
    np.testing.assert_allclose(h @ u, 2.0, rtol=0, atol=1e-11)
    if k >= 3:
        x, m, h, *_ = sem.axis_operator(elements, k, length, "neumann")
        u = x * x * (3 * length - 2 * x)  # u'(0) = u'(L) = 0
        np.testing.assert_allclose(h @ u, -(6 * length - 12 * x), rtol=0, atol=1e-10)


@pytest.mark.parametrize("bc,k", [("dirichlet", 2), ("dirichlet", 3), ("neumann", 2)])
def test_low_eigenvalues_converge_at_order_2k(bc, k):
    length = 1.0
    errs = []
    for e in (4, 8):
        lam = sem.axis_operator(e, k, length, bc)[4]
        modes = np.arange(1, 4) if bc == "dirichlet" else np.arange(0, 3)
        exact = (modes * math.pi / length) ** 2
        errs.append(np.abs(lam[:3] - exact)[modes > 0].max())
    assert errs[0] / errs[1] > 0.6 * 2 ** (2 * k), errs


@pytest.mark.parametrize("bc,shape,k", [("dirichlet", (5, 7), 2), ("neumann", (7, 10), 3),
                                        ("dirichlet", (3, 5, 7), 2)])
def test_tensor_solve_matches_a_direct_solve(bc, shape, k):
    """T Lam T^-1 on every axis against the assembled sum of Kronecker
    products of H (C order: the last axis is innermost)."""
    rng = np.random.default_rng(3)
    ops_ = []
    for n in shape:
        e = (n + 1) // k if bc == "dirichlet" else (n - 1) // k
        ops_.append(sem.axis_operator(e, k, 1.5, bc))
        assert len(ops_[-1][0]) == n
    r = rng.standard_normal(shape)
    a = np.zeros((r.size, r.size))
    for ax, op in enumerate(ops_):
        mats = [np.eye(n) for n in shape]
        mats[ax] = op[2]
        term = mats[0]
        for mm in mats[1:]:
            term = np.kron(term, mm)
        a += term
    x_ref = np.linalg.solve(2.0 * a + 0.7 * np.eye(r.size), r.ravel()).reshape(shape)
    np.testing.assert_allclose(sem.fdm_solve(r, ops_, 0.7, 2.0), x_ref, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("k", [2, 3])
def test_manufactured_solution_converges_at_high_order(k):
    """-Lap u + u^3 = f on (0, 1)^2, u = sin(pi x) sin(2 pi y), Dirichlet:
    the nodal error of the converged discrete solution falls at least like
    h^(k + 1/2) (Q^k: h^(k+1) expected)."""
    errs = []
    for e in (4, 8):
        op = sem.axis_operator(e, k, 1.0, "dirichlet")
        x = op[0]
        u = np.sin(2 * math.pi * x)[:, None] * np.sin(math.pi * x)[None, :]
        f = 5 * math.pi ** 2 * u + u ** 3
        out = sem.qn_solve(f, [op, op], rtol=1e-13, max_iter=100)
        assert out["converged"]
        errs.append(float(np.abs(out["u"] - u).max()))
    assert errs[0] / errs[1] > 2 ** (k + 0.5), errs
