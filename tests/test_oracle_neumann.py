"""Pins for oracle.neumann (homogeneous Neumann data, Section 3.2): the cosine
eigenpairs against the stiffness matrix and against the diagonal-mass route of
Section 4.2, the mirrored stencil against the assembled Kronecker sum, the
tensor-product solve (Section 4.1) against a direct solve, and the
quasi-Newton iteration (Section 4) against a discrete manufactured solution and
second-order convergence."""

import numpy as np
import pytest

import synth
from oracle import neumann as nm
from oracle.spectral import diagonalize


@pytest.mark.parametrize("n", [2, 3, 9, 64, 65])
def test_cosine_eigenpairs_diagonalise_the_stiffness_matrix(n):
    h = 2.0 / (n - 1)
    t, lam, tinv = nm.cosine_eigenpairs(n, h)
    s = nm.stiffness(n, h)
    scale = np.abs(lam).max() + 1.0
    assert np.abs(s @ t - t * lam[None, :]).max() <= 1e-13 * scale
    assert np.abs(tinv @ t - np.eye(n)).max() <= 1e-13
    assert lam[0] == 0.0 and np.all(np.diff(lam) > 0)


@pytest.mark.parametrize("n", [5, 12, 33])
def test_cosine_modes_match_the_diagonal_mass_route(n):
    """S = W^-1 K with K = W S symmetric: the Section 4.2 route (symmetric
    M^-1/2 K M^-1/2 with M = W) gives the same eigenvalues, and its T columns are
    the cosine modes up to scale and sign."""
    h = 2.0 / (n - 1)
    s = nm.stiffness(n, h)
    w = nm.weights(n)
    k = w[:, None] * s
    assert np.abs(k - k.T).max() <= 1e-12 * np.abs(k).max()
    t2, lam2, tinv2 = diagonalize(k, w)
    t, lam, _ = nm.cosine_eigenpairs(n, h)
    assert np.allclose(lam2, lam, rtol=1e-12, atol=1e-9)
    for c in range(n):
        a, b = t[:, c], t2[:, c]
        ratio = np.dot(a, b) / np.dot(b, b)
        assert np.abs(a - ratio * b).max() <= 1e-10 * np.abs(a).max()


@pytest.mark.parametrize("shape", [(7, 9), (2, 5), (5, 6, 7)])
def test_mirrored_stencil_equals_the_assembled_operator(shape):
    rng = np.random.default_rng(3)
    u = rng.standard_normal(shape)
    hs = tuple(0.1 + 0.05 * i for i in range(len(shape)))
    a = nm.assemble_laplacian(shape, hs)
    assert np.allclose(nm.apply_laplacian(u, hs).ravel(), a @ u.ravel(), rtol=1e-13, atol=1e-10)
    assert np.abs(nm.apply_laplacian(np.ones(shape), hs)).max() <= 1e-10  # constants: no flux


def test_weighted_self_adjointness():
    """With the trapezoid weights the operator is symmetric: <W A u, v> = <u, W A v>
    (the factor 2 of the ghost rows is what makes this hold)."""
    shape = (6, 8)
    hs = nm.spacing(shape)
    rng = np.random.default_rng(4)
    u, v = rng.standard_normal(shape), rng.standard_normal(shape)
    w = nm.weights(shape[0])[:, None] * nm.weights(shape[1])[None, :]
    lhs = np.sum(w * nm.apply_laplacian(u, hs) * v)
    rhs = np.sum(u * w * nm.apply_laplacian(v, hs))
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("shape,shift,scale", [((9, 13), 0.5, 2.0), ((17, 17), 1.0, 1.0),
                                               ((5, 6, 7), 1.0, 1.0), ((2, 3, 4), 0.25, 1.5)])
def test_fdm_solve_matches_direct_solve(shape, shift, scale):
    rng = np.random.default_rng(5)
    r = rng.standard_normal(shape)
    hs = nm.spacing(shape)
    x = nm.fdm_solve(r, hs, shift, scale)
    ref = nm.direct_solve(r, hs, shift, scale)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= 1e-12


def test_qn_recovers_a_discrete_manufactured_solution():
    n = 33
    hs = nm.spacing((n, n))
    u_ex, _ = synth.neumann_2d(n)
    f = nm.apply_laplacian(u_ex, hs) + u_ex + u_ex ** 3  # U* = u_ex exactly
    res = nm.qn_solve(f, hs, lin=1.0)
    assert res["converged"]
    assert np.abs(res["u"] - u_ex).max() <= 1e-8


@pytest.mark.parametrize("gen,sizes", [(synth.neumann_2d, (17, 33, 65)),
                                       (synth.neumann_3d, (9, 17, 33))])
def test_second_order_convergence(gen, sizes):
    errs, its = [], []
    for n in sizes:
        u_ex, f = gen(n)
        hs = nm.spacing(u_ex.shape)
        res = nm.qn_solve(f, hs, lin=1.0)
        assert res["converged"]
        errs.append(np.abs(res["u"] - u_ex).max())
        its.append(res["iters"])
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.6 and 3.7 < r2 < 4.3, errs
    assert max(its) - min(its) <= 2, its  # mesh-independent iteration counts
