"""Pins for oracle.grayscott (Section 6.2, eq. 2dgrayeq): the discrete
operator against the assembled Kronecker sum, the reaction Jacobian against
central differences, the block eigenvalues against LAPACK, the per-component
solve against a dense direct solve, the damped step, and the roots the
iteration reaches against closed-form constant states and dense Newton."""

import math

import numpy as np
import pytest

from oracle import grayscott as gs
from oracle import neumann as nm

P = gs.PAPER_PARAMS
# a parameter set with non-trivial constant states: rho > 4 (mu + rho)^2
Q = {"da": 2.5e-4, "ds": 5e-4, "rho": 0.05, "mu": 0.01}


def _spot(n, amp=0.25, radius=0.1):
    x = np.linspace(0.0, 1.0, n)
    X, Y = np.meshgrid(x, x)
    m = ((X - 0.5) ** 2 + (Y - 0.5) ** 2 < radius ** 2).astype(float)
    return np.stack([amp * m, 1.0 - 0.5 * m])


def test_trivial_state_is_an_exact_root():
    n = 33
    u = np.stack([np.zeros((n, n)), np.ones((n, n))])
    r = gs.residual(u, gs.source((n, n), P["rho"]), (gs.spacing(n),) * 2, **P)
    assert np.all(r == 0.0)
    out = gs.qn_solve(u, n, **P)
    assert out["iters"] == 0 and out["converged"]


def test_residual_against_the_assembled_operator():
    n = 9
    rng = np.random.default_rng(0)
    u = rng.uniform(0.0, 1.0, (2, n, n))
    f = gs.source((n, n), P["rho"])
    hs = (gs.spacing(n),) * 2
    lap = nm.assemble_laplacian((n, n), hs)
    a, s = u[0].ravel(), u[1].ravel()
    k = P["mu"] + P["rho"]
    want_a = P["da"] * (lap @ a) - s * a * a + k * a
    want_s = P["ds"] * (lap @ s) + s * a * a + P["rho"] * s - P["rho"]
    r = gs.residual(u, f, hs, **P)
    assert np.allclose(r[0].ravel(), want_a, rtol=1e-13, atol=1e-15)
    assert np.allclose(r[1].ravel(), want_s, rtol=1e-13, atol=1e-15)


def test_block_entries_are_the_reaction_jacobian():
    """Central differences of the residual at one node: the diagonal of the
    Jacobian minus the diffusion part is the 2 x 2 block of that node."""
    n = 7
    rng = np.random.default_rng(1)
    u = rng.uniform(0.1, 0.9, (2, n, n))
    f = gs.source((n, n), P["rho"])
    hs = (gs.spacing(n),) * 2
    lap = nm.assemble_laplacian((n, n), hs).toarray()
    blk = gs.block_entries(u, P["rho"], P["mu"])
    j, i = 3, 2
    idx = j * n + i
    eps = 1e-6
    for comp in range(2):
        up, dn = u.copy(), u.copy()
        up[comp, j, i] += eps
        dn[comp, j, i] -= eps
        col = (gs.residual(up, f, hs, **P) - gs.residual(dn, f, hs, **P))[:, j, i] / (2 * eps)
        diffusion = (P["da"], P["ds"])
        num = col - np.array([diffusion[0] * lap[idx, idx] if comp == 0 else 0.0,
                              diffusion[1] * lap[idx, idx] if comp == 1 else 0.0])
        want = (np.array([blk[0][j, i], blk[2][j, i]]) if comp == 0
                else np.array([blk[1][j, i], blk[3][j, i]]))
        assert np.allclose(num, want, rtol=1e-6, atol=1e-8)


def test_block_eigenvalues_against_lapack():
    rng = np.random.default_rng(2)
    u = rng.uniform(0.0, 1.0, (2, 20, 20))
    a, b, c, d = gs.block_entries(u, P["rho"], P["mu"])
    lm, lp = gs.block_eigs(u, P["rho"], P["mu"])
    n_complex = 0
    for idx in np.ndindex(a.shape):
        ev = np.linalg.eigvals(np.array([[a[idx], b[idx]], [c[idx], d[idx]]]))
        re = np.sort(ev.real)
        if abs(ev.imag).max() > 0:
            n_complex += 1
        assert lm[idx] == pytest.approx(re[0], rel=1e-12, abs=1e-14)
        assert lp[idx] == pytest.approx(re[1], rel=1e-12, abs=1e-14)
    assert 0 < n_complex < a.size  # both branches of the rule are exercised


def test_component_solve_against_a_dense_direct_solve():
    n = 12
    rng = np.random.default_rng(3)
    r = rng.standard_normal((2, n, n))
    hs = (gs.spacing(n),) * 2
    x = gs.solve(r, hs, (P["da"], P["ds"]), 0.03)
    for c, dc in enumerate((P["da"], P["ds"])):
        ref = nm.direct_solve(r[c], hs, 0.03, scale=dc)
        assert np.linalg.norm(x[c] - ref) <= 1e-12 * np.linalg.norm(ref)


def test_the_damped_step():
    n = 17
    u0 = _spot(n, radius=0.3)
    hs = (gs.spacing(n),) * 2
    f = gs.source((n, n), P["rho"])
    one = gs.qn_solve(u0, n, **P, tau=0.1, max_iter=1, rtol=0.0)
    b = gs.midpoint_shift(u0, P["rho"], P["mu"])
    step = gs.solve(gs.residual(u0, f, hs, **P), hs, (P["da"], P["ds"]), b)
    assert np.array_equal(one["u"], u0 - 0.1 * step)
    assert one["beta"] == [b]


@pytest.mark.parametrize("which", [1, 2])
def test_constant_states_closed_form(which):
    """For rho > 4 (mu + rho)^2 the constant states with S A = mu + rho are
    exact roots of the discrete system."""
    states = gs.homogeneous_states(Q["rho"], Q["mu"])
    assert len(states) == 3
    a, s = states[which]
    assert s * a == pytest.approx(Q["mu"] + Q["rho"], rel=1e-14)
    n = 11
    u = np.stack([np.full((n, n), a), np.full((n, n), s)])
    r = gs.residual(u, gs.source((n, n), Q["rho"]), (gs.spacing(n),) * 2, **Q)
    assert np.abs(r).max() <= 1e-15


def test_iteration_reaches_the_dense_newton_root_from_a_perturbed_constant_state():
    """Started near the upper constant state, the damped iteration and dense
    Newton converge to the same root, which is that constant state."""
    n = 9
    a, s = gs.homogeneous_states(Q["rho"], Q["mu"])[2]
    rng = np.random.default_rng(4)
    u0 = np.stack([np.full((n, n), a), np.full((n, n), s)]) * (1 + 0.02 * rng.standard_normal((2, n, n)))
    newton = gs.newton_solve(u0, n, **Q)
    out = gs.qn_solve(u0, n, **Q, tau=0.1, rtol=1e-12, max_iter=20000)
    assert out["converged"], out["relres"][-3:]
    assert np.abs(out["u"] - newton).max() <= 1e-9
    assert np.abs(newton[0] - a).max() <= 1e-10 and np.abs(newton[1] - s).max() <= 1e-10


def test_paper_parameters_spot_start_reaches_the_trivial_state():
    """With the paper's parameters, a spot start decays: the damped iteration
    and dense Newton from it both end at (0, 1) (the paper's eight
    non-trivial states need its initial guesses, which it shows only as
    figures)."""
    n = 9
    u0 = _spot(n, radius=0.3)
    out = gs.qn_solve(u0, n, **P, tau=0.1, rtol=1e-10)
    assert out["converged"]
    assert np.abs(out["u"][0]).max() <= 1e-9 and np.abs(out["u"][1] - 1.0).max() <= 1e-9
    newton = gs.newton_solve(out["u"], n, **P)
    assert np.abs(newton - out["u"]).max() <= 1e-9


def test_undamped_and_damped_iterations_share_the_root_and_the_damped_one_is_slower():
    n = 9
    a, s = gs.homogeneous_states(Q["rho"], Q["mu"])[2]
    rng = np.random.default_rng(5)
    u0 = np.stack([np.full((n, n), a), np.full((n, n), s)]) * (1 + 0.02 * rng.standard_normal((2, n, n)))
    full = gs.qn_solve(u0, n, **Q, tau=1.0, rtol=1e-11)
    damped = gs.qn_solve(u0, n, **Q, tau=0.1, rtol=1e-11)
    assert full["converged"] and damped["converged"]
    assert np.abs(full["u"] - damped["u"]).max() <= 1e-9
    assert damped["iters"] > 3 * full["iters"]
