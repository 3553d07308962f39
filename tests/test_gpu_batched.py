"""GPU tests of the batched solver: every instance of a mixed batch (uneven
sizes, scalar and 2-component) matches the single-instance solver and the CPU
oracle; tile shapes and graph length do not change results; a diverging
instance does not disturb the others."""

import numpy as np
import pytest
import torch

import synth
from oracle import qn as oqn
from oracle.spectral import sine_eigenpairs
from paper_2502_03611_amd import Solver
from paper_2502_03611_amd.batched import BatchedSolver
from parity_rules import counts_agree, rel_l2

pytestmark = pytest.mark.gpu

SIZES = [15, 31, 63, 15, 100, 33, 63, 31, 17, 63, 127, 15]
NCOMP = [1, 2, 1, 1, 2, 1, 2, 1, 2, 1, 2, 2]


def sources(sizes, ncomp, seed0=4000000):
    out = []
    for i, (n, c) in enumerate(zip(sizes, ncomp)):
        rng = np.random.default_rng(seed0 + i)
        out.append(20.0 * np.stack([synth.gaussian_random_field(n, 0.1, rng) for _ in range(c)]))
    return out


def build(prec, sizes=SIZES, ncomp=NCOMP):
    b = BatchedSolver(sizes, ncomp, precision=prec, beta_mode="midpoint")
    F = b.pool()
    srcs = sources(sizes, ncomp)
    for i, f in enumerate(srcs):
        b.fill(F, i, f)
    return b, F, srcs


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batched_matches_single_instance_and_oracle(prec):
    print(f"batched {prec}", flush=True)
    b, F, srcs = build(prec)
    U = b.pool()
    status, res = b.iterate(U, F, rtol=1e-10, max_iter=100, graph_iters=3)
    assert status == 0, res
    for i, f in enumerate(srcs):
        n, c = SIZES[i], NCOMP[i]
        kind = "system" if c == 2 else "cubic"
        s = Solver((n, n), kind, beta_mode="midpoint", precision=prec)
        u1 = torch.zeros((c, n, n), dtype=torch.float64, device="cuda")
        st = s.iterate(u1, torch.from_numpy(f).cuda(), rtol=1e-10, max_iter=100)
        ub = b.view(U, i).cpu().numpy()
        assert res[i]["iters"] == st["iters"], (i, res[i], st)
        assert np.linalg.norm(ub - u1.cpu().numpy()) <= 1e-12 * np.linalg.norm(ub)
        ref = oqn.qn_solve(oqn.SYSTEM if c == 2 else oqn.CUBIC, f, midpoint=True, rtol=1e-10)
        assert abs(res[i]["iters"] - ref["iters"]) <= (0 if prec == "fp64" else 1)
        # both stopped at relres <= 1e-10: |U_b - U_o| <= 2 rtol |F| / lam_min(J)
        lam = 2 * sine_eigenpairs(n)[1][0] - (1.0 if c == 2 else 0.0)
        assert np.linalg.norm(ub - ref["u"]) <= 2e-10 * np.linalg.norm(f) / lam


@pytest.mark.parametrize("rule", ["max", "sum", "min"])
def test_batched_shift_rules_dirichlet_mixed_batch(rule):
    """The table's other shift rules on the mixed Dirichlet batch (scalar and
    2-component instances, FP64), each instance under the same rule:
    iteration counts agree with the oracle's and the single-problem solver's
    (equal, or one apart only when the deciding relres lies within 0.1 % of
    rtol); after exactly K = 4 solves (rtol = 0) every instance is within 1e-12
    of the oracle's U_4 and of the single-problem solver's."""
    print(f"batched dirichlet rule {rule}", flush=True)
    k = 4
    b = BatchedSolver(SIZES, NCOMP, precision="fp64", beta_mode=rule)
    F = b.pool()
    srcs = sources(SIZES, NCOMP)
    for i, f in enumerate(srcs):
        b.fill(F, i, f)
    U = b.pool()
    status, res = b.iterate(U, F, rtol=1e-10, max_iter=300, graph_iters=3)
    assert status == 0, res
    Uk = b.pool()
    statusk, resk = b.iterate(Uk, F, rtol=0.0, max_iter=k, graph_iters=3)
    assert statusk == 3 and all(r["iters"] == k for r in resk)
    for i, f in enumerate(srcs):
        n, c = SIZES[i], NCOMP[i]
        kind = "system" if c == 2 else "cubic"
        okind = oqn.SYSTEM if c == 2 else oqn.CUBIC
        ref = oqn.qn_solve(okind, f, rule=rule, rtol=1e-10, max_iter=300)
        assert ref["converged"]
        assert counts_agree(res[i]["iters"], ref), (i, res[i], ref["iters"], ref["relres"][-2:])
        s = Solver((n, n), kind, beta_mode=rule, precision="fp64")
        u1 = torch.zeros((c, n, n), dtype=torch.float64, device="cuda")
        st = s.iterate(u1, torch.from_numpy(f).cuda(), rtol=1e-10, max_iter=300)
        assert counts_agree(st["iters"], ref), (i, st, ref["iters"])
        assert counts_agree(res[i]["iters"], {"iters": st["iters"], "relres": ref["relres"]})
        refk = oqn.qn_solve(okind, f, rule=rule, rtol=0.0, max_iter=k)
        ubk = b.view(Uk, i).cpu().numpy()
        assert rel_l2(ubk, refk["u"]) <= 1e-12, (i, rel_l2(ubk, refk["u"]))
        u1k = torch.zeros((c, n, n), dtype=torch.float64, device="cuda")
        s.iterate(u1k, torch.from_numpy(f).cuda(), rtol=0.0, max_iter=k)
        assert rel_l2(ubk, u1k.cpu().numpy()) <= 1e-12


def test_tiles_and_graph_length_do_not_change_results():
    b, F, _ = build("fp32")
    U1 = b.pool()
    b.iterate(U1, F, rtol=1e-10, max_iter=100, graph_iters=1)
    b.autotune()
    print("classes", b.classes(), flush=True)
    U2 = b.pool()
    b.iterate(U2, F, rtol=1e-10, max_iter=100, graph_iters=5)
    assert torch.equal(U1, U2)


def test_diverging_instance_is_isolated():
    b, F, _ = build("fp32")
    U1 = b.pool()
    _, r1 = b.iterate(U1, F, rtol=1e-10, max_iter=100)
    bad = 3
    b.view(F, bad)[0, 2, 2] = float("nan")
    U2 = b.pool()
    status, r2 = b.iterate(U2, F, rtol=1e-10, max_iter=100)
    assert status == 4 and r2[bad]["status"] == 4
    for i in range(len(SIZES)):
        if i != bad:
            assert r2[i] == r1[i]
            assert torch.equal(b.view(U1, i), b.view(U2, i))


def test_max_iter_reported_per_instance():
    b, F, _ = build("fp64")
    U = b.pool()
    status, res = b.iterate(U, F, rtol=1e-10, max_iter=2, graph_iters=4)
    assert status == 3
    assert all(r["iters"] <= 2 for r in res)
    assert any(r["status"] == 3 for r in res)


NEU_SIZES = [17, 33, 40, 64, 17, 33, 129, 40]


@pytest.mark.parametrize("prec,mode,beta", [("fp64", "midpoint", 0.0), ("fp32", "midpoint", 0.0),
                                            ("fp64", "fixed", 3.0), ("fp64", "max", 0.0),
                                            ("fp64", "sum", 0.0), ("fp64", "min", 0.0)])
def test_batched_neumann_matches_single_instance_and_oracle(prec, mode, beta):
    """Section 6.2, Example 1 (eq. ex2d1): -Lap u + u + u^3 = f on [-1, 1]^2
    with zero normal derivative, every instance started from the sampled
    exact solution plus 0.1 times its own seeded degree-4 polynomial (the
    paper's perturbed starts, here one batch instead of one solve each), under
    each shift rule of the paper's table.  Against the single-problem solver: equal counts and iterates to 1e-12;
    against the oracle: equal counts (FP64) and the rtol bound."""
    from oracle import neumann as nm
    print(f"batched neumann {prec} {mode}", flush=True)
    b = BatchedSolver(NEU_SIZES, [1] * len(NEU_SIZES), precision=prec, beta_mode=mode, beta=beta,
                      boundary="neumann", length=2.0, lin=1.0)
    U, F = b.pool(), b.pool()
    starts, srcs = [], []
    for i, n in enumerate(NEU_SIZES):
        u, f = synth.neumann_2d(n)
        u0 = u + 0.1 * synth.polynomial_perturbation(n, 2, i)
        starts.append(u0)
        srcs.append(f)
        b.fill(U, i, u0[None])
        b.fill(F, i, f[None])
    status, res = b.iterate(U, F, rtol=1e-10, max_iter=200, graph_iters=4)
    assert status == 0, res
    for i, n in enumerate(NEU_SIZES):
        ub = b.view(U, i).cpu().numpy()[0]
        s = Solver((n, n), "cubic", boundary="neumann", length=2.0, lin=1.0, beta_mode=mode,
                   beta=beta, precision=prec)
        u1 = torch.from_numpy(starts[i][None].copy()).cuda()
        st = s.iterate(u1, torch.from_numpy(srcs[i][None].copy()).cuda(), rtol=1e-10, max_iter=200)
        assert res[i]["iters"] == st["iters"], (i, res[i], st)
        assert np.linalg.norm(ub - u1.cpu().numpy()[0]) <= 1e-12 * np.linalg.norm(ub)
        ref = nm.qn_solve(srcs[i], nm.spacing((n, n)), lin=1.0, u0=starts[i], beta=beta,
                          midpoint=mode == "midpoint", rtol=1e-10, max_iter=200,
                          rule=mode if mode in ("max", "sum", "min") else None)
        assert ref["converged"]
        assert abs(res[i]["iters"] - ref["iters"]) <= (0 if prec == "fp64" else 1), (i, res[i])
        # both stopped at relres <= 1e-10 and the Jacobian is >= lin = 1:
        # |U_b - U_o| <= 2 rtol |F| / 1
        assert np.linalg.norm(ub - ref["u"]) <= 2e-10 * np.linalg.norm(srcs[i])


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 3e-6), ("bf16x3", 4e-5)])
def test_batched_fdm_solve_every_instance(prec, tol):
    """qnb_fdm_solve: X_i = (scale A_h + shift I)^-1 R_i for every instance of
    a mixed pool (scalar and 2-component, uneven sizes), against the oracle's
    tensor-product solve; X may alias R."""
    from oracle import tensor as otensor
    b = BatchedSolver(SIZES, NCOMP, precision=prec, beta_mode="midpoint")
    R = b.pool()
    rng = np.random.default_rng(77)
    rs = []
    for i, (n, c) in enumerate(zip(SIZES, NCOMP)):
        r = rng.standard_normal((c, n, n))
        rs.append(r)
        b.fill(R, i, r)
    X = b.fdm_solve(R, 1.5, 0.25)
    b.fdm_solve(R, 1.5, 0.25, X=R)
    assert torch.equal(X, R)
    for i, r in enumerate(rs):
        x = b.view(X, i).cpu().numpy()
        for c in range(r.shape[0]):
            ref = otensor.fdm_solve(r[c], 0.25, 1.5)
            assert rel_l2(x[c], ref) <= tol, (i, c)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_batched_step_size_in_every_precision(prec):
    """step = 1/2 halves every instance's first correction, in the update
    epilogue of each transform precision the batch offers."""
    print(f"batched step {prec}", flush=True)
    sizes, ncomp = [31, 64, 17, 100], [1, 2, 2, 1]
    srcs = sources(sizes, ncomp)
    out = []
    for step in (1.0, 0.5):
        b = BatchedSolver(sizes, ncomp, precision=prec, beta_mode="midpoint", step=step)
        F, U = b.pool(), b.pool()
        for i, f in enumerate(srcs):
            b.fill(F, i, f)
        b.iterate(U, F, rtol=0.0, max_iter=1, graph_iters=1)
        out.append([b.view(U, i).cpu().numpy() for i in range(len(sizes))])
    for full, half in zip(*out):
        assert np.linalg.norm(full) > 0
        assert np.linalg.norm(half - 0.5 * full) <= 1e-14 * np.linalg.norm(full)
