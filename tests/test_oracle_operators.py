"""Pins for oracle.operators and oracle.tensor.mode_product: stencils against the
assembled Kronecker sum (eqs. A_definition_2D/3D), exactness on quadratics, the
vec/Kronecker identity of Section 3.1 (eq. vec-property), the quasi-linear flux
form against explicit face loops and the continuous operator, and the 2x2
block eigenvalues of Section 4.3 (eq. eigenvalues) against hand values and a
library eigensolver."""

import math
import os

import numpy as np
import pytest

import synth
from oracle import operators as ops
from oracle import tensor

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("shape", [(9,), (7, 11), (5, 6, 8), (4, 4, 4)])
def test_stencil_equals_assembled_kronecker_sum(shape):
    u = synth.random_field(shape, 11)
    a = ops.assemble_laplacian(shape)
    ref = (a @ u.ravel()).reshape(shape)
    got = ops.apply_laplacian(u)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_laplacian_exact_on_quadratics():
    """Central differences are exact for u = x(1-x) y(1-y) z(1-z), which is zero
    on the boundary: -Lap u = 2[y(1-y)z(1-z) + x(1-x)z(1-z) + x(1-x)y(1-y)]."""
    n = 9
    z, y, x = np.meshgrid(*[synth.grid_coords(n)] * 3, indexing="ij")
    qx, qy, qz = x * (1 - x), y * (1 - y), z * (1 - z)
    u = qx * qy * qz
    expect = 2.0 * (qy * qz + qx * qz + qx * qy)
    np.testing.assert_allclose(ops.apply_laplacian(u), expect, rtol=1e-12, atol=1e-12)


def test_vec_kronecker_identity_column_major():
    """vec(A X B^T) = (B (x) A) vec(X), vec = column stacking (Section 3.1)."""
    rng = np.random.default_rng(0)
    a, b, x = rng.standard_normal((4, 4)), rng.standard_normal((3, 3)), rng.standard_normal((4, 3))
    lhs = (a @ x @ b.T).ravel(order="F")
    rhs = np.kron(b, a) @ x.ravel(order="F")
    np.testing.assert_allclose(lhs, rhs, rtol=1e-13)
    # The same object in this package's layout: X stored as (ny, nx) C-order is
    # X^T, and kron_apply([B, A]) is (B (x) A) on its C-order ravel.
    got = tensor.kron_apply([b, a], x.T.copy())
    np.testing.assert_allclose(got, (a @ x @ b.T).T, rtol=1e-13)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mode_product_matches_explicit_kronecker(axis):
    rng = np.random.default_rng(axis)
    shape = (3, 4, 5)
    x = rng.standard_normal(shape)
    m = rng.standard_normal((shape[axis], shape[axis]))
    mats = [np.eye(n) for n in shape]
    mats[axis] = m
    np.testing.assert_allclose(tensor.mode_product(x, m, axis),
                               tensor.kron_apply(mats, x), rtol=1e-12, atol=1e-13)


def test_three_mode_products_equal_paper_3d_form():
    """(C (x) B (x) A) vec(X) with A on x, B on y, C on z (Section 4.1)."""
    rng = np.random.default_rng(9)
    x = rng.standard_normal((3, 4, 5))  # (z, y, x)
    a, b, c = (rng.standard_normal((k, k)) for k in (5, 4, 3))
    y = tensor.mode_product(tensor.mode_product(tensor.mode_product(x, a, 2), b, 1), c, 0)
    np.testing.assert_allclose(y, tensor.kron_apply([c, b, a], x), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("shape", [(4, 5), (3, 4, 3)])
def test_quasilinear_vectorised_equals_face_loops(shape):
    u = synth.random_field(shape, 2)
    f = synth.random_field(shape, 3)
    np.testing.assert_allclose(ops.residual_quasilinear(u, f),
                               ops.residual_quasilinear_loops(u, f), rtol=1e-13, atol=1e-10)


def test_quasilinear_reduces_to_laplacian_for_small_u():
    """a(u) = 1 + u^2 -> 1: L(U)U = A_h U + O(|U|^3)."""
    u = 1e-5 * synth.random_field((6, 7, 5), 4)
    lin = ops.apply_laplacian(u)
    got = ops.residual_quasilinear(u, np.zeros_like(u))
    assert np.abs(got - lin).max() <= 1e-9 * np.abs(lin).max()


def test_quasilinear_consistency_second_order():
    """L(u_ex) u_ex - f_ex = O(h^2) for the manufactured smooth solution."""
    errs = []
    for n in (15, 31):
        ue, f = synth.manufactured_c3(n, 1.5)
        errs.append(np.abs(ops.residual_quasilinear(ue, f)).max())
    assert 3.6 < errs[0] / errs[1] < 4.4


def test_quasilinear_symmetric_form():
    """Discrete integration by parts: <V, L(U)U> = sum_faces a_f dU dV / h^2,
    boundary faces included (U = V = 0 outside)."""
    shape = (4, 5, 6)
    u = synth.random_field(shape, 7)
    v = synth.random_field(shape, 8)
    lhs = float(np.sum(v * ops.residual_quasilinear(u, np.zeros_like(u))))
    hs = ops.spacing(shape)
    rhs = 0.0
    for ax in range(3):
        pad = [(0, 0)] * 3
        pad[ax] = (1, 1)
        up, vp = np.pad(u, pad), np.pad(v, pad)
        ap = 1.0 + up * up
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        af = 0.5 * (ap[tuple(lo)] + ap[tuple(hi)])
        rhs += float(np.sum(af * (up[tuple(hi)] - up[tuple(lo)]) * (vp[tuple(hi)] - vp[tuple(lo)]))) / hs[ax] ** 2
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_cubic_residual_second_order_consistency():
    errs = []
    for n in (31, 63):
        ue, f = synth.manufactured_c1(n)
        errs.append(np.abs(ops.residual_cubic(ue, f)).max())
    assert 3.6 < errs[0] / errs[1] < 4.4


def test_system_eigs_hand_values():
    rows = np.loadtxt(os.path.join(GOLDEN, "system_eigs.txt"))
    lm, lp = ops.system_jacobian_eigs(rows[:, 0], rows[:, 1])
    np.testing.assert_allclose(lm, rows[:, 2], rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(lp, rows[:, 3], rtol=1e-14)


def test_system_eigs_against_library():
    u = synth.random_field((50,), 1)
    v = synth.random_field((50,), 2)
    lm, lp = ops.system_jacobian_eigs(u, v)
    for i in range(50):
        blk = np.array([[3 * u[i] ** 2, -1.0], [-1.0, 3 * v[i] ** 2]])
        e = np.linalg.eigvalsh(blk)
        assert lm[i] == pytest.approx(e[0], rel=1e-12, abs=1e-12)
        assert lp[i] == pytest.approx(e[1], rel=1e-12)


def test_system_residual_block_structure():
    """F^h(U,V) = blockdiag(A_h, A_h)(U,V) + N_h (Section 4.3)."""
    shape = (6, 5)
    u, v = synth.random_field(shape, 1), synth.random_field(shape, 2)
    f1, f2 = synth.random_field(shape, 3), synth.random_field(shape, 4)
    a = ops.assemble_laplacian(shape)
    r1, r2 = ops.residual_system(u, v, f1, f2)
    np.testing.assert_allclose(r1.ravel(), a @ u.ravel() + u.ravel() ** 3 - v.ravel() - f1.ravel(), atol=1e-10)
    np.testing.assert_allclose(r2.ravel(), a @ v.ravel() + v.ravel() ** 3 - u.ravel() - f2.ravel(), atol=1e-10)


def test_manufactured_c2_source_matches_finite_difference_of_exact():
    """Independent check of the analytic RHS used as input: the discrete
    residual of u_exact is O(h^2) against it."""
    errs = []
    for n in (15, 31):
        ue, f = synth.manufactured_c2(n)
        errs.append(np.abs(ops.residual_cubic(ue, f)).max() / math.sqrt(n))
    assert errs[1] < errs[0]
