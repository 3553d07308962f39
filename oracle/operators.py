"""Discrete residuals F^h(U) = A_h vec(U) + N_h(U) (oracle; test-only).

Arrays are C-order (.., ny, nx), x fastest = the paper's vec order.  Homogeneous
Dirichlet data: the unknowns are the interior nodes, h_a = 1/(n_a+1) per axis,
and the boundary values (zero) drop out of the near-boundary rows (Section 3.2,
the F_h cases for Dirichlet data, all of whose boundary terms vanish here).

Problems (the paper's model is -Lap u + lambda u + f(x,u) = 0, Section 2
eq. main-pde; here lambda = 0):
* cubic: f(x, u) = u^3 - f_src(x), so N_h(U) = U^3 - F.
* system (Section 4.3, eq. system): f = u^3 - v - f1, g = v^3 - u - f2.
* quasi-linear -div((1+u^2) grad u) = f_src, in conservative flux form with
  arithmetic-mean face coefficients.  The paper has no divergence-form
  example (its model in Section 2 is semilinear), so this discretisation is a
  reading: the standard second-order conservative scheme.
"""

import numpy as np
import scipy.sparse as sp

from .spectral import stiffness_matrix


def spacing(shape):
    """h per axis, in array-axis order (.., y, x)."""
    return tuple(1.0 / (n + 1) for n in shape)


def apply_laplacian(u):
    """A_h vec(U) by the central-difference stencil (Section 3.2 eq. fdm-discrete),
    U zero outside the interior.  Works for 1, 2 or 3 dimensions."""
    hs = spacing(u.shape)
    out = np.zeros_like(u)
    for ax, h in enumerate(hs):
        pad = [(0, 0)] * u.ndim
        pad[ax] = (1, 1)
        up = np.pad(u, pad)
        lo = np.take(up, np.arange(0, u.shape[ax]), axis=ax)
        hi = np.take(up, np.arange(2, u.shape[ax] + 2), axis=ax)
        out += (2.0 * u - lo - hi) / (h * h)
    return out


def assemble_laplacian(shape):
    """Sparse A_h as the Kronecker sum of 1D stiffness matrices
    (eqs. A_definition_2D / A_definition_3D with lambda = 0, H = S since M = I).

    For shape (.., ny, nx) acting on the C-order ravel: the last axis (x) is
    the innermost Kronecker factor, e.g. 3D: I_z (x) I_y (x) S_x + I_z (x) S_y
    (x) I_x + S_z (x) I_y (x) I_x.
    """
    d = len(shape)
    total = None
    for ax in range(d):
        factors = [sp.identity(n, format="csr") for n in shape]
        factors[ax] = sp.csr_matrix(stiffness_matrix(shape[ax]))
        term = factors[0]
        for f in factors[1:]:
            term = sp.kron(term, f, format="csr")
        total = term if total is None else total + term
    return total.tocsr()


def residual_cubic(u, f, lin=0.0, cub=1.0, pot=None, quad=0.0):
    """F^h(U) = A_h U + lin U + quad U^2 + cub U^3 + V U - F (Section 4 eq. F_u
    with the model of Section 2: lambda = lin, f(x, u) = cub u^3 + quad u^2 +
    V(x) u - f_src(x); pot = V sampled on the grid, None = 0)."""
    r = apply_laplacian(u) + lin * u + quad * u ** 2 + cub * u ** 3 - f
    return r if pot is None else r + pot * u


def fu_cubic(u, lin=0.0, cub=1.0, pot=None, quad=0.0):
    """Diagonal of the Jacobian (N_h)_U of the pointwise part:
    3 cub U^2 + 2 quad U + lin + V."""
    d = 3.0 * cub * u * u + 2.0 * quad * u + lin
    return d if pot is None else d + pot


def residual_system(u, v, f1, f2):
    """Block residual of Section 4.3 (eq. system) with lambda_1 = lambda_2 = 0,
    f(x,u,v) = u^3 - v - f1 and g(x,u,v) = v^3 - u - f2.  Returns (R1, R2)."""
    r1 = apply_laplacian(u) + u ** 3 - v - f1
    r2 = apply_laplacian(v) + v ** 3 - u - f2
    return r1, r2


def system_jacobian_eigs(u, v):
    """Per-point eigenvalues of the 2x2 block DN_h (Section 4.3, eq. eigenvalues).

    Entries: (N1)_U = 3u^2, (N1)_V = -1, (N2)_U = -1, (N2)_V = 3v^2, so
    lam_+- = (a + d +- sqrt((a - d)^2 + 4 b c)) / 2.  Returns (lam_minus, lam_plus).
    """
    a = 3.0 * u * u
    d = 3.0 * v * v
    b = -1.0
    c = -1.0
    disc = np.sqrt((a - d) ** 2 + 4.0 * b * c)
    return 0.5 * (a + d - disc), 0.5 * (a + d + disc)


def coeff_quasilinear(u):
    """a(u) = 1 + u^2."""
    return 1.0 + u * u


def residual_quasilinear(u, f):
    """R = L(U) U - F with the conservative flux form
    (L(U)U)_i = sum_axes sum_{+-} a_{i+-1/2} (U_i - U_{i+-1}) / h^2,
    a_{i+-1/2} = (a(U_i) + a(U_{i+-1})) / 2, and U = 0 (a = 1) on the boundary."""
    hs = spacing(u.shape)
    a = coeff_quasilinear(u)
    out = np.zeros_like(u)
    for ax, h in enumerate(hs):
        pad = [(0, 0)] * u.ndim
        pad[ax] = (1, 1)
        up = np.pad(u, pad)
        ap = np.pad(a, pad, constant_values=1.0)
        for off in (0, 2):
            un = np.take(up, np.arange(off, u.shape[ax] + off), axis=ax)
            an = np.take(ap, np.arange(off, u.shape[ax] + off), axis=ax)
            out += 0.5 * (a + an) * (u - un) / (h * h)
    return out - f


def residual_quasilinear_loops(u, f):
    """Same operator as residual_quasilinear, by explicit loops over faces.

    Each interior face between node p and neighbour q (q may be a boundary
    node with value 0) contributes a_f (U_p - U_q) / h^2 to row p.  Tiny N only.
    """
    hs = spacing(u.shape)
    out = -np.array(f, dtype=np.float64, copy=True)
    shape = u.shape
    for p in np.ndindex(*shape):
        up = u[p]
        ap = 1.0 + up * up
        acc = 0.0
        for ax in range(u.ndim):
            h = hs[ax]
            for step in (-1, 1):
                q = list(p)
                q[ax] += step
                if 0 <= q[ax] < shape[ax]:
                    uq = u[tuple(q)]
                else:
                    uq = 0.0
                aq = 1.0 + uq * uq
                acc += 0.5 * (ap + aq) * (up - uq) / (h * h)
        out[p] += acc
    return out
