"""The shift rules compared in the paper's tables (Section 6.2, Tables
results2d1 and results2d_space; Section 6.3, Tables results3D and
results3D_mesh): beta_k = (min + max)/2 of the Jacobian diagonal (the
proposed midpoint), min + max, max and min.  The tables show the midpoint
needing the fewest iterations, min + max and max about twice as many, and min
the most; the oracle reproduces that ordering on the same problems from the
same kind of start, which pins its shift rules (a swapped min/max or a missing
factor 1/2 reorders them)."""

import numpy as np
import pytest

import synth
from oracle import neumann as nm


def _iters(u_ex, f, hs, rule, **kw):
    u_star = nm.qn_solve(f, hs, rtol=1e-13, max_iter=500, **kw)["u"]
    shape = f.shape
    p = synth.polynomial_perturbation(shape[0], len(shape), 0)
    out = nm.qn_solve(f, hs, u0=u_star + 0.1 * p, rule=rule, max_iter=2000, **kw)
    assert out["converged"], rule
    return out["iters"]


def test_rule_ordering_2d_eq_ex2d1():
    u_ex, f = synth.neumann_2d(65)
    hs = nm.spacing(f.shape)
    it = {r: _iters(u_ex, f, hs, r, lin=1.0) for r in ("mid", "sum", "max", "min")}
    assert it["mid"] < it["sum"] and it["mid"] < it["max"] and it["max"] < it["min"], it
    assert 1.4 < it["sum"] / it["mid"] < 2.6 and 1.4 < it["max"] / it["mid"] < 2.6, it


def test_rule_ordering_3d_eq_ex3d1():
    u_ex, f, v = synth.neumann_potential_3d(17)
    hs = nm.spacing(f.shape)
    it = {r: _iters(u_ex, f, hs, r, lin=10.0, cub=10.0, pot=v) for r in ("mid", "sum", "max")}
    assert it["mid"] < it["max"] < it["sum"], it
    assert 1.4 < it["sum"] / it["mid"] < 2.6, it


def test_shift_of_values():
    fu = np.array([2.0, 5.0, 3.0])
    assert nm.shift_of("mid", fu, 0) == 3.5 and nm.shift_of("sum", fu, 0) == 7.0
    assert nm.shift_of("max", fu, 0) == 5.0 and nm.shift_of("min", fu, 0) == 2.0
    assert nm.shift_of("fixed", fu, 9.0) == 9.0


def test_dirichlet_rule_shifts_match_pointwise_jacobian_blocks():
    """The Dirichlet oracle's shift rules against the Jacobian blocks built
    node by node: the cubic diagonal 3 u^2 + lin (a 1x1 block) and the
    system's [[3u^2, -1], [-1, 3v^2]] (Section 4.3), eigenvalues by LAPACK's
    symmetric solver; each rule is the named function of their range."""
    from oracle import qn as oqn
    rng = np.random.default_rng(21)
    u = rng.standard_normal((2, 5, 6))
    eig = np.array([np.linalg.eigvalsh(np.array([[3 * a * a, -1.0], [-1.0, 3 * b * b]]))
                    for a, b in zip(u[0].ravel(), u[1].ravel())])
    lo, hi = eig[:, 0].min(), eig[:, 1].max()
    d = 3 * u[0] ** 2 + 0.7
    want = {"mid": (0.5 * (lo + hi), 0.5 * (d.min() + d.max())), "max": (hi, d.max()),
            "sum": (lo + hi, d.min() + d.max()), "min": (lo, d.min())}
    for rule, (w_sys, w_cub) in want.items():
        assert oqn.shift_rule(oqn.SYSTEM, u, 0.0, False, rule=rule)[1] == pytest.approx(w_sys, rel=1e-14)
        assert oqn.shift_rule(oqn.CUBIC, u[:1], 0.0, False, lin=0.7, rule=rule)[1] == \
            pytest.approx(w_cub, rel=1e-14)
    # no rule: the midpoint flag, else the fixed beta
    assert oqn.shift_rule(oqn.CUBIC, u[:1], 2.5, False, lin=0.7)[1] == 2.5
    assert oqn.shift_rule(oqn.CUBIC, u[:1], 2.5, True, lin=0.7)[1] == pytest.approx(want["mid"][1])


@pytest.mark.parametrize("rule", ["max", "sum", "min"])
def test_dirichlet_rules_reach_the_dense_newton_root(rule):
    """Every rule's iteration (Dirichlet data, cubic problem and system)
    converges to the root that dense Newton's method finds."""
    from oracle import qn as oqn
    rng = np.random.default_rng(1)
    for kind, c in ((oqn.CUBIC, 1), (oqn.SYSTEM, 2)):
        f = 30.0 * rng.standard_normal((c, 6, 7))
        root = oqn.newton_solve(kind, f)
        out = oqn.qn_solve(kind, f, rule=rule, rtol=1e-13, max_iter=500)
        assert out["converged"]
        assert np.linalg.norm(out["u"] - root) <= 1e-11 * np.linalg.norm(root)
