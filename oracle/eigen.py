"""Nonlinear eigenproblem by the quasi-Newton iteration with normalisation
(oracle; test-only).

Section 4.4 (eqs. Eigenvalue_p, system_qusi, system_normal): find u and the
eigenvalue lam with -Lap u + f(u) = lam u.  The eigenvalue is expressed
through u as a Rayleigh quotient in the mass inner product,

    lam_n = <A_h U_n + f(U_n), U_n>_M / <U_n, U_n>_M,

the residual is F^h(U_n) = A_h U_n + N_h(U_n) with N_h(U_n) = f(U_n) - lam_n U_n,
one step is U~ = U_n - (A_h + beta_n I)^-1 F^h(U_n), and the next iterate is
U~ normalised, U_{n+1} = U~ / sqrt(<U~, U~>_M); the start is normalised too.

Here f(u) = b u^3 + (lin + V(x)) u (Section 6.3, Example 2, eq. ex3d2:
b = alpha = 1600, lin = 0, a potential V, Dirichlet data on (-8, 8)^3), on
finite-difference grids with homogeneous Dirichlet or Neumann data.  Readings
(the paper leaves these open):
* M is the lumped finite-difference mass h^d (W (x) W (x) W): W = I for
  Dirichlet data, W = diag(1/2, 1, .., 1, 1/2) (trapezoid weights) for Neumann
  data, so <1, 1>_M is the domain's volume and ||U||_M approximates the L2 norm.
* beta_n: the midpoint rule of Section 4 applied to the diagonal of
  (N_h)_U = diag(f'(U_n)) - lam_n I with lam_n held fixed:
  beta_n = (min f'(U_n) + max f'(U_n)) / 2 - lam_n, f'(u) = 3 b u^2 + lin + V;
  or a fixed beta.
* Stop when ||F^h(U_n)||_M / |lam_n| <= rtol (||U_n||_M = 1).
Dirichlet data on a cube of side L: A_h = L^-2 A_h(unit cube), h = L/(n+1).
Pinned in tests/test_oracle_eigen.py.
"""

import math

import numpy as np

from . import neumann as nm
from . import operators as ops
from .tensor import fdm_solve as dirichlet_fdm_solve


def spacing(shape, bc, length):
    """h per axis (array-axis order)."""
    if bc == "neumann":
        return nm.spacing(shape, length)
    return tuple(length / (n + 1) for n in shape)


def mass_weights(shape, bc, length):
    """Diagonal of M = h^d (W (x) .. (x) W) on the grid, array shape."""
    hs = spacing(shape, bc, length)
    w = np.full(shape, float(np.prod(hs)))
    if bc == "neumann":
        for ax, n in enumerate(shape):
            bshape = [1] * len(shape)
            bshape[ax] = n
            w = w * nm.weights(n).reshape(bshape)
    return w


def apply_laplacian(u, bc, length):
    """A_h U with homogeneous Dirichlet (side L) or Neumann data."""
    if bc == "neumann":
        return nm.apply_laplacian(u, spacing(u.shape, bc, length))
    return ops.apply_laplacian(u) / (length * length)


def solve(r, shift, bc, length):
    """(A_h + shift I)^-1 R by the tensor-product formula (Section 4.1)."""
    if bc == "neumann":
        return nm.fdm_solve(r, spacing(r.shape, bc, length), shift)
    return dirichlet_fdm_solve(r, shift, 1.0 / (length * length))


def f_term(u, cub, lin, pot):
    v = lin * u + cub * u ** 3
    return v if pot is None else v + pot * u


def f_prime(u, cub, lin, pot):
    d = 3.0 * cub * u * u + lin
    return d if pot is None else d + pot


def rayleigh(u, bc, length, cub, lin, pot):
    """lam = <A_h U + f(U), U>_M / <U, U>_M."""
    w = mass_weights(u.shape, bc, length)
    g = apply_laplacian(u, bc, length) + f_term(u, cub, lin, pot)
    return float(np.sum(w * g * u)) / float(np.sum(w * u * u))


def residual(u, lam, bc, length, cub, lin, pot):
    """F^h(U) = A_h U + f(U) - lam U."""
    return apply_laplacian(u, bc, length) + f_term(u, cub, lin, pot) - lam * u


def normalise(u, bc, length):
    w = mass_weights(u.shape, bc, length)
    return u / math.sqrt(float(np.sum(w * u * u)))


def eigen_solve(u0, bc="dirichlet", length=1.0, cub=1.0, lin=0.0, pot=None, beta=None,
                rtol=1e-10, max_iter=2000):
    """The iteration of Section 4.4 from U_0 (normalised first).  beta = None
    takes the midpoint rule, a number a fixed shift.  Returns dict(u (the last
    normalised iterate), lam, iters (solves), relres (history), beta (per
    solve), converged)."""
    w = mass_weights(u0.shape, bc, length)
    u = normalise(np.asarray(u0, dtype=np.float64), bc, length)
    hist, betas = [], []
    k = 0
    lam = float("nan")
    while True:
        lam = rayleigh(u, bc, length, cub, lin, pot)
        r = residual(u, lam, bc, length, cub, lin, pot)
        rel = math.sqrt(float(np.sum(w * r * r))) / abs(lam)
        hist.append(rel)
        if rel <= rtol or k >= max_iter or not math.isfinite(rel):
            break
        if beta is None:
            fp = f_prime(u, cub, lin, pot)
            b = 0.5 * (float(fp.min()) + float(fp.max())) - lam
        else:
            b = float(beta)
        betas.append(b)
        u = normalise(u - solve(r, b, bc, length), bc, length)
        k += 1
    return {"u": u, "lam": lam, "iters": k, "relres": hist, "beta": betas,
            "converged": hist[-1] <= rtol}
