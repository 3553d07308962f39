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
