"""Pins for oracle.tensor.fdm_solve (Section 4.1, eq. fin_inverse) against
direct solves, and for oracle.qn (Section 4, eq. identity-method) against dense
Newton (eq. newton), discrete manufactured solutions, second-order convergence,
mesh independence and the contraction bound of Section 5 (eq. norm_ratio)."""

import math

import numpy as np
import pytest

import synth
from oracle import operators as ops
from oracle import qn, tensor
from oracle.spectral import sine_eigenpairs


@pytest.mark.parametrize("shape,shift,scale", [
    ((15, 15), 0.0, 1.0), ((63, 63), 1.0, 1.0), ((9, 13), 3.5, 2.0),
    ((7, 7, 7), 0.1007, 1.0), ((15, 15, 15), 0.0, 1.0), ((5, 9, 6), -10.0, 1.5),
])
def test_fdm_solve_equals_direct_solve(shape, shift, scale):
    r = synth.random_field(shape, 21)
    x_t = tensor.fdm_solve(r, shift, scale)
    x_d = tensor.direct_solve(r, shift, scale)
    assert np.linalg.norm(x_t - x_d) / np.linalg.norm(x_d) <= 1e-13


def test_fdm_solve_inverts_operator():
    shape = (31, 31, 31)
    x = synth.random_field(shape, 5)
    r = 1.7 * ops.apply_laplacian(x) + 0.3 * x
    got = tensor.fdm_solve(r, 0.3, 1.7)
    assert np.linalg.norm(got - x) / np.linalg.norm(x) <= 1e-12


def test_denominator_smallest_entry():
    lam = sine_eigenpairs(10)[1]
    d = tensor.spectral_denominator((10, 10, 10), 0.5, 2.0)
    assert d[0, 0, 0] == pytest.approx(2.0 * 3 * lam[0] + 0.5)
    assert d[9, 0, 3] == pytest.approx(2.0 * (lam[9] + lam[0] + lam[3]) + 0.5)


def test_config1_iterations_and_second_order():
    errs = []
    for n in (15, 31, 63):
        ue, f = synth.manufactured_c1(n)
        res = qn.qn_solve(qn.CUBIC, f[None], beta=1.0, rtol=1e-10)
        assert res["converged"]
        assert res["iters"] == 8
        errs.append(np.abs(res["u"][0] - ue).max())
    assert 3.8 < errs[0] / errs[1] < 4.2
    assert 3.8 < errs[1] / errs[2] < 4.2


def test_one_dimensional_example_of_section6():
    """Section 6.1 Ex. 1: -u'' + u^3 = pi^2 sin(pi x) + sin^3(pi x), u = sin(pi x)."""
    errs = []
    for n in (63, 127):
        x = synth.grid_coords(n)
        ue = np.sin(math.pi * x)
        f = math.pi ** 2 * ue + ue ** 3
        res = qn.qn_solve(qn.CUBIC, f[None], midpoint=True)
        assert res["converged"]
        errs.append(np.abs(res["u"][0] - ue).max())
    assert 3.8 < errs[0] / errs[1] < 4.2


@pytest.mark.parametrize("shape,kind", [((15, 15), qn.CUBIC), ((6, 7, 5), qn.CUBIC),
                                        ((9, 11), qn.SYSTEM)])
def test_fixed_point_equals_dense_newton(shape, kind):
    ncomp = 2 if kind == qn.SYSTEM else 1
    f = 20.0 * synth.random_field((ncomp,) + shape, 17)
    un = qn.newton_solve(kind, f)
    res = qn.qn_solve(kind, f, midpoint=True, rtol=1e-13, max_iter=400)
    assert res["converged"]
    assert np.linalg.norm(res["u"] - un) / np.linalg.norm(un) <= 1e-12


@pytest.mark.parametrize("kind,shape", [(qn.CUBIC, (31, 31, 31)), (qn.QUASILINEAR, (15, 15, 15)),
                                        (qn.SYSTEM, (31, 31))])
def test_discrete_manufactured_solution_is_recovered(kind, shape):
    ncomp = 2 if kind == qn.SYSTEM else 1
    amp = 0.3 if kind == qn.QUASILINEAR else 1.5
    ue = amp * synth.random_field((ncomp,) + shape, 3)
    # F := (A_h u_e + N_h(u_e)) with the source removed, so F^h(u_e) = 0 exactly
    f = qn.residual(kind, ue, np.zeros_like(ue))
    rtol = 1e-12
    res = qn.qn_solve(kind, f, midpoint=(kind != qn.QUASILINEAR), rtol=rtol, max_iter=500)
    assert res["converged"]
    # |U - u_e| <= |J^-1| |R| <= rtol |F| / lam_min(J), and lam_min(J) >= lam_min(A_h) - 1
    lam_min = sum(sine_eigenpairs(n)[1][0] for n in shape) - 1.0
    bound = 2.0 * rtol * np.linalg.norm(f) / lam_min
    assert np.linalg.norm(res["u"] - ue) <= bound


def test_contraction_bound_holds():
    """Error ratio per iteration <= g(beta) of eq. norm_ratio plus O(|e|)."""
    n = 31
    ue, f = synth.manufactured_c1(n)
    ustar = qn.qn_solve(qn.CUBIC, f[None], beta=1.0, rtol=1e-14, max_iter=100)["u"]
    lam_min = 2 * sine_eigenpairs(n)[1][0]
    u = np.zeros_like(ustar)
    prev = np.linalg.norm(u - ustar)
    for _ in range(5):
        fu = ops.fu_cubic(u[0])
        r = qn.residual(qn.CUBIC, u, f[None])
        beta = 0.5 * (fu.min() + fu.max())
        u = u - tensor.fdm_solve(r[0], beta)[None]
        e = np.linalg.norm(u - ustar)
        g = qn.contraction_bound(float(fu.min()), float(fu.max()), lam_min, beta)
        assert e / prev <= g + 0.05
        prev = e


def test_midpoint_rule_is_min_max_midpoint():
    u = synth.random_field((1, 8, 8), 4)
    c, b = qn.shift_rule(qn.CUBIC, u, 0.0, True)
    vals = sorted(3.0 * float(t) ** 2 for t in u.ravel())
    assert c == 1.0
    assert b == pytest.approx(0.5 * (vals[0] + vals[-1]), rel=1e-15)


def test_quasilinear_mesh_independent_iterations():
    its = []
    for n in (15, 31):
        _, f = synth.manufactured_c3(n, 2.0)
        res = qn.qn_solve(qn.QUASILINEAR, f[None])
        assert res["converged"]
        its.append(res["iters"])
    assert abs(its[0] - its[1]) <= 1


def test_quasilinear_second_order_convergence():
    errs = []
    for n in (15, 31):
        ue, f = synth.manufactured_c3(n, 1.0)
        res = qn.qn_solve(qn.QUASILINEAR, f[None])
        errs.append(np.abs(res["u"][0] - ue).max())
    assert 3.6 < errs[0] / errs[1] < 4.4


def test_config2_iterations():
    ue, f = synth.manufactured_c2(31)
    res = qn.qn_solve(qn.CUBIC, f[None], beta=0.1007)
    assert res["converged"] and res["iters"] == 4


def test_config2_beta_sweep():
    """The fixed shift of the 3D cubic workload: the oracle's sweep over
    beta in {0, b_mid, 2 b_mid, 5 b_mid}, b_mid = 1.5 max(U*^2) (the midpoint
    of f_u = 3u^2 at the exact solution, Section 4), recorded at 63^3.  The
    fixed beta = 0.1007 is b_mid and needs no more iterations than any other
    point of the sweep."""
    ue, f = synth.manufactured_c2(63)
    b_mid = 1.5 * float(np.max(ue ** 2))
    assert b_mid == pytest.approx(0.1007, abs=5e-4)
    sweep = {}
    for b in (0.0, b_mid, 2.0 * b_mid, 5.0 * b_mid):
        res = qn.qn_solve(qn.CUBIC, f[None], beta=b)
        assert res["converged"]
        sweep[round(b, 4)] = res["iters"]
    print("beta sweep (beta: iterations):", sweep)
    assert list(sweep.values()) == [4, 4, 5, 6]
    fixed = qn.qn_solve(qn.CUBIC, f[None], beta=0.1007)
    assert fixed["iters"] == min(sweep.values())
