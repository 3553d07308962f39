"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle on
the same seeded inputs.  Tolerances (FP64):
  residual  ||R_gpu - R_ora|| / (||A_h U|| + ||N(U)|| + ||F||) <= 1e-13
            (near convergence R is pure cancellation, so it is measured against
            the size of the terms that cancel);
  solve     ||X_gpu - X_ora|| / ||X_ora|| <= 1e-12;
  iterate   equal iteration counts to rtol 1e-10, then exactly K solves on both
            sides: ||U_gpu - U_ora|| / ||U_ora|| <= 1e-12.
"""

import math

import numpy as np
import pytest
import torch

import synth
from oracle import operators as ops
from oracle import qn as oqn
from oracle import tensor as otensor
from paper_2502_03611_amd import Solver, QN_OK, QN_ERR_NOT_CONVERGED, QN_ERR_DIVERGED, QN_ERR_INVALID
from paper_2502_03611_amd._binding import QNError

pytestmark = pytest.mark.gpu

KIND = {"cubic": oqn.CUBIC, "system": oqn.SYSTEM, "quasilinear": oqn.QUASILINEAR}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def term_scale(kind, u):
    lap = sum(np.linalg.norm(ops.apply_laplacian(u[c])) for c in range(u.shape[0]))
    nl = float(np.linalg.norm(u ** 3)) if kind != "quasilinear" else float(
        np.linalg.norm(ops.residual_quasilinear(u[0], np.zeros_like(u[0]))))
    return lap + nl


@pytest.mark.parametrize("kind,shape", [
    ("cubic", (37, 45, 70)), ("cubic", (1, 1, 1)), ("cubic", (5, 1, 9)), ("cubic", (63, 63)),
    ("cubic", (100, 37)), ("cubic", (1, 1)), ("system", (17, 19, 23)), ("system", (45, 70)),
    ("quasilinear", (33, 20, 65)), ("quasilinear", (50, 61)),
    # 3D tile widths 256 and 512 (two tiles across x at 1000), 256-wide tiles
    # of 512-thread workgroups (two components), and a column tile over 64
    # thin z-slabs (slab boundaries every 3 planes)
    ("cubic", (6, 5, 250)), ("quasilinear", (4, 7, 500)), ("cubic", (3, 4, 1000)),
    ("system", (5, 6, 500)), ("quasilinear", (130, 3, 60)),
])
def test_residual_parity(kind, shape):
    print(f"residual {kind} {shape}", flush=True)
    ncomp = 2 if kind == "system" else 1
    u = synth.random_field((ncomp,) + shape, 101)
    f = synth.random_field((ncomp,) + shape, 102, scale=10.0)
    s = Solver(shape, kind, beta=0.0)
    red = torch.zeros(4, dtype=torch.float64, device="cuda")
    r = host(s.residual(dev(u), dev(f), red=red))
    ref = oqn.residual(KIND[kind], u, f)
    scale = term_scale(kind, u) + float(np.linalg.norm(f))
    assert np.linalg.norm(r - ref) / scale <= 1e-13
    red = red.cpu().numpy()
    if kind == "cubic":
        mu = ops.fu_cubic(u[0])
        lo, hi = mu.min(), mu.max()
    elif kind == "system":
        lm, lp = ops.system_jacobian_eigs(u[0], u[1])
        lo, hi = lm.min(), lp.max()
    else:
        a = ops.coeff_quasilinear(u[0])
        lo, hi = a.min(), a.max()
    assert red[0] == pytest.approx(float(np.sum(ref * ref)), rel=1e-12)
    assert red[1] == pytest.approx(lo, rel=1e-14, abs=1e-15)
    assert red[2] == pytest.approx(hi, rel=1e-14)
    assert red[3] == pytest.approx(float(np.sum(f * f)), rel=1e-13)


@pytest.mark.parametrize("shape,scale,shift", [
    ((63, 63), 1.0, 1.0), ((100, 37), 2.0, 0.5), ((1, 1), 1.0, 0.0), ((7, 300), 1.0, 3.0),
    ((31, 31, 31), 1.0, 0.1007), ((17, 40, 65), 1.5, 2.0), ((3, 5, 2), 1.0, 0.0),
    ((64, 64, 64), 1.0, -10.0),
])
def test_fdm_solve_parity_fp64(shape, scale, shift):
    print(f"fdm fp64 {shape}", flush=True)
    r = synth.random_field((1,) + shape, 7)
    s = Solver(shape, "cubic")
    x = host(s.fdm_solve(dev(r), scale, shift))
    ref = otensor.fdm_solve(r[0], shift, scale)
    assert rel(x[0], ref) <= 1e-12


def test_fdm_solve_two_components_and_alias():
    shape = (33, 33, 33)
    r = synth.random_field((2,) + shape, 8)
    s = Solver(shape, "system")
    t = dev(r)
    s.fdm_solve(t, 1.0, 0.3, X=t)  # X aliases R
    x = host(t)
    for c in range(2):
        assert rel(x[c], otensor.fdm_solve(r[c], 0.3)) <= 1e-12


def test_fdm_solve_smooth_rhs():
    shape = (63, 63, 63)
    _, f = synth.manufactured_c2(63)
    s = Solver(shape, "cubic")
    x = host(s.fdm_solve(dev(f[None]), 1.0, 0.0))
    assert rel(x[0], otensor.fdm_solve(f, 0.0)) <= 1e-12


def test_fdm_solve_max_size_2d():
    shape = (4096, 4096)
    r = synth.random_field((1,) + shape, 9)
    s = Solver(shape, "cubic")
    x = host(s.fdm_solve(dev(r), 1.0, 1.0))
    assert rel(x[0], otensor.fdm_solve(r[0], 1.0)) <= 1e-12


# Reduced-precision solve bounds against the FP64 solve (six chained mode
# products, contractions of at most 70 terms here): FP32 about
# sqrt(K) 2^-24 sqrt(6) = 1.2e-6, hence 3e-6; bf16x3 carries the split error
# sqrt(6) 2^-16 = 3.7e-5 (the oracle's own split-bf16 solve lands at 1.1e-5);
# bf16x6 drops only terms below 2^-24 and is bounded like FP32.
@pytest.mark.parametrize("prec,tol", [("fp32", 3e-6), ("bf16x3", 4e-5), ("bf16x6", 3e-6)])
@pytest.mark.parametrize("shape", [(63, 63), (31, 31, 31), (40, 50, 70), (40, 45, 33), (64, 98, 20)])
def test_fdm_solve_reduced_precision(prec, tol, shape):
    print(f"fdm {prec} {shape}", flush=True)
    r = synth.random_field((1,) + shape, 10)
    s = Solver(shape, "cubic", precision=prec)
    x = host(s.fdm_solve(dev(r), 1.0, 0.5))
    err = rel(x[0], otensor.fdm_solve(r[0], 0.5))
    print(f"  {prec} {shape} rel err {err:.3e}", flush=True)
    assert err <= tol


@pytest.mark.parametrize("kind,shape", [("quasilinear", (40, 45, 33)), ("system", (36, 64, 63)),
                                        ("quasilinear", (64, 127, 128))])
def test_bf16x3_solve_from_an_input_folded_along_x(kind, shape):
    """3D bf16x3 solvers of the quasi-linear and 2-component problems whose
    extents allow it take every forward product folded by mode parity, the x
    product from an input written folded along x (here by the copy of the
    caller's right-hand side): the solve stays within the split error bound of
    the FP64 oracle's, per component."""
    print(f"x-folded fdm {kind} {shape}", flush=True)
    ncomp = 2 if kind == "system" else 1
    r = synth.random_field((ncomp,) + shape, 12)
    s = Solver(shape, kind, beta=1.0, precision="bf16x3")
    x = host(s.fdm_solve(dev(r), 1.3, 0.7))
    for c in range(ncomp):
        err = rel(x[c], otensor.fdm_solve(r[c], 0.7, 1.3))
        print(f"  component {c}: rel err {err:.3e}", flush=True)
        assert err <= 4e-5


@pytest.mark.parametrize("prec,parts", [("bf16x3", 2), ("bf16x6", 3)])
@pytest.mark.parametrize("shape,scale,shift", [((63, 63), 1.0, 0.5), ((31, 31, 31), 1.7, 0.0),
                                               ((40, 50, 70), 1.0, 2.0)])
def test_split_bf16_solve_matches_the_split_oracle(prec, parts, shape, scale, shift):
    """The split-bf16 solve against the oracle's own split-bf16 solve (the same
    part products in the same product order, summed exactly, FP32 storage
    between products): they differ only by the matrix cores' FP32
    accumulation, at most K 2^-24 relative per product for K-term sums (K <= 96
    here, six chained products), measured 0.8e-6 to 4e-6; the bound 1e-5 is
    about 200 times below what a lost or doubled part product (2^-9 relative)
    does to the result, and 4 times below the split error itself."""
    from oracle import splitbf16 as osb
    print(f"split oracle {prec} {shape}", flush=True)
    r = synth.random_field((1,) + shape, 11)
    s = Solver(shape, "cubic", precision=prec)
    x = host(s.fdm_solve(dev(r), scale, shift))
    ref = osb.split_fdm_solve(r[0], shift, parts, scale=scale)
    err = rel(x[0], ref)
    print(f"  {prec} {shape}: rel diff vs split oracle {err:.3e}, vs FP64 oracle "
          f"{rel(x[0], otensor.fdm_solve(r[0], shift, scale)):.3e}", flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("kind,shape,beta,mode", [
    ("cubic", (63, 63), 1.0, "fixed"), ("quasilinear", (31, 33, 35), 0.0, "fixed"),
    ("system", (40, 45), 0.0, "midpoint"), ("quasilinear", (40, 45, 33), 0.0, "fixed"),
    ("system", (63, 45, 20), 0.0, "midpoint"),
])
def test_reduced_precision_iterate_reaches_the_fp64_solution(prec, kind, shape, beta, mode):
    """Transforms in reduced precision with the FP64 residual and update: the
    outer iteration refines to the same 1e-10 relative residual; the result
    agrees with the FP64 oracle's converged U to <= 1e-9 relative L2 and takes
    at most 10% more iterations."""
    print(f"mixed iterate {prec} {kind} {shape}", flush=True)
    ncomp = 2 if kind == "system" else 1
    f = synth.random_field((ncomp,) + shape, 31, scale=30.0)
    ref = oqn.qn_solve(KIND[kind], f, beta=beta, midpoint=(mode == "midpoint"), rtol=1e-10,
                       max_iter=300)
    s = Solver(shape, kind, beta=beta, beta_mode=mode, precision=prec)
    u = torch.zeros((ncomp,) + shape, dtype=torch.float64, device="cuda")
    st = s.iterate(u, dev(f), rtol=1e-10, max_iter=300)
    assert st["status"] == QN_OK, st
    assert st["relres"] <= 1e-10
    assert st["iters"] <= math.ceil(1.1 * ref["iters"]), (st["iters"], ref["iters"])
    err = rel(host(u), ref["u"])
    print(f"  iters {st['iters']} (oracle {ref['iters']}), rel err {err:.2e}", flush=True)
    assert err <= 1e-9


def run_both(kind, f, shape, beta=0.0, beta_mode="fixed", rtol=1e-10, max_iter=300):
    ncomp = f.shape[0]
    s = Solver(shape, kind, beta=beta, beta_mode=beta_mode)
    u = torch.zeros((ncomp,) + shape, dtype=torch.float64, device="cuda")
    st = s.iterate(u, dev(f), rtol=rtol, max_iter=max_iter)
    ref = oqn.qn_solve(KIND[kind], f, beta=beta, midpoint=(beta_mode == "midpoint"), rtol=rtol,
                       max_iter=max_iter)
    return s, st, host(u), ref


def check_iterate_parity(kind, f, shape, beta=0.0, beta_mode="fixed"):
    s, st, u, ref = run_both(kind, f, shape, beta, beta_mode)
    assert st["status"] == QN_OK, st
    k = ref["iters"]
    if st["iters"] != k:
        # allowed only when the deciding residual sits within 0.1% of the tolerance
        deciding = ref["relres"][min(st["iters"], k)]
        assert abs(st["iters"] - k) == 1 and abs(deciding / 1e-10 - 1) < 1e-3, (st, ref["relres"])
    # exactly K solves on both sides
    s2 = Solver(shape, kind, beta=beta, beta_mode=beta_mode)
    ug = torch.zeros((f.shape[0],) + shape, dtype=torch.float64, device="cuda")
    st2 = s2.iterate(ug, dev(f), rtol=0.0, max_iter=k)
    assert st2["status"] == QN_ERR_NOT_CONVERGED and st2["iters"] == k
    assert rel(host(ug), ref["u"]) <= 1e-12
    return st, ref


def test_iterate_config1_fixed_beta():
    ue, f = synth.manufactured_c1(63)
    st, ref = check_iterate_parity("cubic", f[None], (63, 63), beta=1.0)
    assert ref["iters"] == 8 and st["iters"] == 8


def test_iterate_config1_midpoint():
    ue, f = synth.manufactured_c1(63)
    check_iterate_parity("cubic", f[None], (63, 63), beta_mode="midpoint")


def test_iterate_system_2d():
    rng = np.random.default_rng(4000001)
    f = np.stack([synth.gaussian_random_field(63, 0.1, rng) for _ in range(2)])
    check_iterate_parity("system", f, (63, 63), beta_mode="midpoint")


def test_iterate_system_3d_ragged():
    f = 30.0 * synth.random_field((2, 9, 17, 33), 5)
    check_iterate_parity("system", f, (9, 17, 33), beta_mode="midpoint")


def test_iterate_quasilinear_3d():
    _, f = synth.manufactured_c3(31, synth.amplitude_c3(0))
    check_iterate_parity("quasilinear", f[None], (31, 31, 31))


def test_iterate_config2_full_size():
    """3D -Lap u + u^3 = f at 255^3, beta = 0.1007 (midpoint at the exact solution)."""
    print("config2 255^3", flush=True)
    ue, f = synth.manufactured_c2(255)
    st, ref = check_iterate_parity("cubic", f[None], (255, 255, 255), beta=0.1007)
    assert st["iters"] == ref["iters"] == 4


def test_fdm_solve_full_size_511_property():
    """At 511^3: solve (A_h + s I) X = R for R built by the oracle stencil from a
    seeded X_true; the GPU solve must return X_true."""
    print("fdm 511^3 property", flush=True)
    n = 511
    xt = synth.random_field((n, n, n), 12)
    r = ops.apply_laplacian(xt)
    r += 0.5 * xt
    s = Solver((n, n, n), "cubic")
    x = host(s.fdm_solve(dev(r[None]), 1.0, 0.5))
    del r
    assert rel(x[0], xt) <= 1e-12


def test_quasilinear_full_size_511_converges_second_order():
    """511^3 quasi-linear FP64: converges to 1e-10, with the iteration count of
    the oracle at 63^3 (mesh independence) and the O(h^2) discretisation error
    predicted from the oracle's 63^3 error."""
    print("quasilinear 511^3", flush=True)
    amp = synth.amplitude_c3(0)
    ue63, f63 = synth.manufactured_c3(63, amp)
    ref = oqn.qn_solve(oqn.QUASILINEAR, f63[None])
    e63 = float(np.abs(ref["u"][0] - ue63).max())
    n = 511
    ue, f = synth.manufactured_c3(n, amp)
    s = Solver((n, n, n), "quasilinear")
    u = torch.zeros((1, n, n, n), dtype=torch.float64, device="cuda")
    st = s.iterate(u, dev(f[None]), rtol=1e-10, max_iter=400)
    assert st["status"] == QN_OK, st
    assert abs(st["iters"] - ref["iters"]) <= 1
    err = float(np.abs(host(u)[0] - ue).max())
    pred = e63 * (64.0 / 512.0) ** 2
    assert 0.5 * pred <= err <= 1.5 * pred


def test_divergence_flagged_on_nan_source():
    ue, f = synth.manufactured_c1(31)
    f[3, 4] = float("nan")
    s = Solver((31, 31), "cubic", beta=1.0)
    u = torch.zeros((1, 31, 31), dtype=torch.float64, device="cuda")
    st = s.iterate(u, dev(f[None]))
    assert st["status"] == QN_ERR_DIVERGED


@pytest.mark.parametrize("kind,shape", [("cubic", (31, 33)), ("system", (17, 19, 23)),
                                        ("quasilinear", (20, 24, 28))])
def test_max_iter_zero_reports_the_initial_residual(kind, shape):
    """max_iter = 0: no solve, U untouched, relres = relres0 = ||F^h(U_0)|| / ||F||."""
    ncomp = 2 if kind == "system" else 1
    u0 = synth.random_field((ncomp,) + shape, 401, scale=0.5)
    f = synth.random_field((ncomp,) + shape, 402, scale=10.0)
    s = Solver(shape, kind, beta=0.0 if kind == "quasilinear" else 1.0)
    u = dev(u0)
    st = s.iterate(u, dev(f), rtol=1e-10, max_iter=0)
    assert st["status"] == QN_ERR_NOT_CONVERGED and st["iters"] == 0
    assert torch.equal(u, dev(u0))
    expect = np.linalg.norm(oqn.residual(KIND[kind], u0, f)) / np.linalg.norm(f)
    assert st["relres"] == pytest.approx(expect, rel=1e-10)
    assert st["relres0"] == st["relres"]


@pytest.mark.parametrize("kind,shape", [("cubic", (63, 63)), ("system", (20, 30, 25)),
                                        ("quasilinear", (33, 20, 31))])
def test_exact_discrete_solution_needs_no_solve(kind, shape):
    """Source built from a discrete field (F := A_h U* + N_h(U*)): starting at U*,
    the first residual already meets the tolerance."""
    ncomp = 2 if kind == "system" else 1
    ue = synth.random_field((ncomp,) + shape, 403, scale=0.5)
    f = oqn.residual(KIND[kind], ue, np.zeros_like(ue))
    s = Solver(shape, kind, beta=0.0 if kind == "quasilinear" else 1.0)
    u = dev(ue)
    st = s.iterate(u, dev(f), rtol=1e-10, max_iter=50)
    assert st["status"] == QN_OK and st["iters"] == 0 and st["relres"] <= 1e-10
    assert torch.equal(u, dev(ue))


def test_tolerance_met_at_the_start_and_zero_source():
    ue, f = synth.manufactured_c1(31)
    s = Solver((31, 31), "cubic", beta=1.0)
    u = torch.zeros((1, 31, 31), dtype=torch.float64, device="cuda")
    st = s.iterate(u, dev(f[None]), rtol=1.0, max_iter=10)  # relres(U_0 = 0) = 1
    assert st["status"] == QN_OK and st["iters"] == 0 and float(u.abs().max()) == 0.0
    with pytest.raises(QNError) as err:
        s.iterate(u, torch.zeros_like(u), rtol=1e-10, max_iter=10)
    assert err.value.status == QN_ERR_INVALID


def test_max_iter_leaves_last_iterate_and_resume_is_bitwise():
    ue, f = synth.manufactured_c1(63)
    s = Solver((63, 63), "cubic", beta=1.0)
    fa = dev(f[None])
    ua = torch.zeros((1, 63, 63), dtype=torch.float64, device="cuda")
    st = s.iterate(ua, fa, rtol=1e-10, max_iter=3)
    assert st["status"] == QN_ERR_NOT_CONVERGED and st["iters"] == 3
    st = s.iterate(ua, fa, rtol=0.0, max_iter=2)
    ub = torch.zeros_like(ua)
    s.iterate(ub, fa, rtol=0.0, max_iter=5)
    assert torch.equal(ua, ub)


def test_deterministic_bitwise():
    _, f = synth.manufactured_c3(31, 1.3)
    outs = []
    for _ in range(2):
        s = Solver((31, 31, 31), "quasilinear")
        u = torch.zeros((1, 31, 31, 31), dtype=torch.float64, device="cuda")
        s.iterate(u, dev(f[None]), rtol=0.0, max_iter=6)
        outs.append(host(u))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("shape,prec,kind", [((255, 255), "fp64", "cubic"), ((63, 63), "fp32", "cubic"),
                                             ((40, 70, 130), "fp64", "cubic"),
                                             ((40, 45, 33), "bf16x3", "cubic"),
                                             ((64, 127, 125), "bf16x3", "cubic"),
                                             ((64, 127, 125), "bf16x3", "quasilinear")])
def test_every_admissible_tile_gives_the_same_bits(shape, prec, kind):
    """Each launch of the solve is pinned in turn to every instantiated tile
    (plain, paired, deep-staged) that qn_set_tile accepts; every solve returns
    the bits of the default one.  Shapes that are not admissible are refused."""
    print(f"all tiles {shape} {prec} {kind}", flush=True)
    f = dev(synth.random_field((1,) + shape, 302, scale=20.0))
    ref = Solver(shape, kind, beta=1.0, precision=prec)
    want = ref.fdm_solve(f, scale=1.5, shift=0.25)
    s = Solver(shape, kind, beta=1.0, precision=prec)
    default = s.tiles()
    tried = 0
    for i, (kind, axis, _, _) in enumerate(default):
        base = kind & 3
        for flags in (0, 4, 32, 36, 64):
            for tm in (32, 64, 128):
                for tn in (32, 64, 128):
                    try:
                        s.set_tile(i, (base + flags, axis, tm, tn))
                    except QNError:
                        continue
                    tried += 1
                    assert s.tiles()[i] == (base + flags, axis, tm, tn)
                    got = s.fdm_solve(f, scale=1.5, shift=0.25)
                    assert torch.equal(got, want), (i, base + flags, tm, tn)
        s.set_tile(i, default[i])
    assert tried > len(default)
    with pytest.raises(QNError):
        s.set_tile(0, (3, 0, 32, 32))  # wrong kind for launch 0
    with pytest.raises(QNError):
        s.set_tile(0, (0, 0, 48, 32))  # not an instantiated shape


@pytest.mark.parametrize("kind,shape,prec", [
    ("cubic", (37, 45, 70), "fp64"), ("system", (31, 64, 97), "fp64"),
    ("quasilinear", (65, 33), "fp64"), ("cubic", (40, 50, 70), "fp32"),
    ("cubic", (40, 50, 70), "bf16x3"), ("system", (33, 60), "bf16x6"),
    ("cubic", (40, 45, 33), "bf16x3"), ("system", (36, 64, 63), "bf16x3"),
])
def test_autotuned_tiles_give_bitwise_identical_solves(kind, shape, prec):
    """The tile shape changes the work split, never the arithmetic order: an
    autotuned solver returns the same bits as the default one, and every chosen
    tile divides its launch's extents."""
    print(f"autotune {kind} {shape} {prec}", flush=True)
    ncomp = 2 if kind == "system" else 1
    f = dev(synth.random_field((ncomp,) + shape, 301, scale=20.0))
    beta = 0.0 if kind == "quasilinear" else 1.0
    ref = Solver(shape, kind, beta=beta, precision=prec)
    tuned = Solver(shape, kind, beta=beta, precision=prec)
    tuned.autotune()
    dense = prec.startswith("bf16")
    for kid, axis, tm, tn in tuned.tiles():
        n = list(reversed(shape))[axis]
        if dense:  # unfolded: tiles divide the padded extent P (and the row count)
            p = 32 * math.ceil(n / 32)
            assert (p % tm == 0) if kid % 4 in (1, 2) else (p % tn == 0), (kid, axis, tm, tn)
        else:
            bk = 32 * math.ceil(math.ceil(n / 2) / 32)
            assert bk % (tm if kid % 4 in (1, 2) else tn) == 0, (kid, axis, tm, tn)
    ua, ub = ref.empty().zero_(), tuned.empty().zero_()
    sa = ref.iterate(ua, f, rtol=0.0, max_iter=3)
    sb = tuned.iterate(ub, f, rtol=0.0, max_iter=3)
    assert sa["iters"] == sb["iters"] == 3
    assert torch.equal(ua, ub)
    xa = ref.fdm_solve(f, scale=1.5, shift=0.25)
    xb = tuned.fdm_solve(f, scale=1.5, shift=0.25)
    assert torch.equal(xa, xb)


def test_mfma_probe_is_plausible():
    """The matrix-core probe reaches a dense rate between 30 % and 110 % of the
    published peaks (FP64 78.6, FP32 157.3, bf16 2500 TFLOP/s)."""
    from paper_2502_03611_amd._binding import probe_mfma
    for prec, peak in (("fp64", 78.6), ("fp32", 157.3), ("bf16x3", 2500.0)):
        v = probe_mfma(prec)
        print(f"mfma probe {prec}: {v:.1f} TFLOP/s", flush=True)
        assert 0.3 * peak <= v <= 1.1 * peak, (prec, v)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("kind,shape", [("cubic", (45, 70)), ("system", (17, 19, 23)),
                                        ("system", (63, 45, 20))])
def test_step_size_scales_the_correction_in_every_precision(prec, kind, shape):
    """U_1 = U_0 - step dU: with step 1/2 the first update is half the undamped
    one (dU is the same bits, so the two differ by the rounding of the
    subtraction only), in the update epilogue of every transform precision."""
    print(f"step {kind} {shape} {prec}", flush=True)
    ncomp = 2 if kind == "system" else 1
    u0 = synth.random_field((ncomp,) + shape, 7)
    f = dev(synth.random_field((ncomp,) + shape, 8, scale=10.0))
    ua, ub = dev(u0), dev(u0)
    Solver(shape, kind, beta=1.0, precision=prec).iterate(ua, f, rtol=0.0, max_iter=1)
    Solver(shape, kind, beta=1.0, precision=prec, step=0.5).iterate(ub, f, rtol=0.0, max_iter=1)
    d_full, d_half = host(ua) - u0, host(ub) - u0
    assert np.linalg.norm(d_full) > 0
    assert np.linalg.norm(d_half - 0.5 * d_full) <= 1e-14 * (np.linalg.norm(d_full) + np.linalg.norm(u0))
