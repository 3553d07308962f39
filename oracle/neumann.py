"""Finite differences with homogeneous Neumann data (oracle; test-only).

Section 3.2 (the Neumann case): the unknowns are all nodes x_0 .. x_{n-1} of
[a, b] (boundary nodes included), h = (b - a) / (n - 1), and the ghost node
outside each end equals its mirror image (zero normal derivative), which turns
the first and last rows of the 1D stiffness matrix into h^-2 (2, -2) and
h^-2 (-2, 2); the boundary data terms of the paper's F_h vanish for
homogeneous data.  H = S is not symmetric, but S = W^-1 K with K symmetric and
W = diag(1/2, 1, .., 1, 1/2), which is the diagonal-mass form H = M^-1 S of
Section 4.2; its eigenpairs are the cosine modes

    T[j, k] = cos(j k pi / (n - 1)),  lam_k = (4 / h^2) sin^2(k pi / (2 (n - 1))),

j, k = 0 .. n-1 (the arguments reduced as integers, j k mod 2 (n - 1)), with
T^-1 = diag(1 / c_k) T^T W, c_k = sum_j W_jj T[j, k]^2 = (n - 1) / 2, or n - 1
for k = 0 and k = n - 1.  lam_0 = 0 (constants), so a solve needs a positive
shift.

Problem (the paper's model -Lap u + lambda u + f(x, u) = 0 of Section 2 with
f(x, u) = b u^3 + V(x) u - f_src(x), b = 1 and V = 0 unless given; the 3D
example of Section 6.3 has lambda = b = 10 and a potential V):
F^h(U) = A_h U + lambda U + b U^3 + V U - F, Jacobian diagonal
f_u = 3 b U^2 + lambda + V.  The tensor-product solve of Section 4.1
(eq. fin_inverse) applies T^-1 along every axis, divides by
scale (lam_i + lam_j (+ lam_k)) + shift and applies T; the quasi-Newton loop
is the one of Section 4 (eq. identity-method) with the midpoint shift.
Pinned in tests/test_oracle_neumann.py.
"""

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .tensor import mode_product


def spacing(shape, length=2.0):
    """h per axis (array-axis order) for nodes on an interval of the given length."""
    return tuple(length / (n - 1) for n in shape)


def stiffness(n, h):
    """Dense 1D ghost-point stiffness matrix of order n (n >= 2)."""
    s = np.zeros((n, n))
    idx = np.arange(n)
    s[idx, idx] = 2.0
    s[idx[:-1], idx[:-1] + 1] = -1.0
    s[idx[:-1] + 1, idx[:-1]] = -1.0
    s[0, 1] = -2.0
    s[n - 1, n - 2] = -2.0
    return s / (h * h)


def weights(n):
    """Diagonal of W (trapezoid weights): 1/2 at both ends, 1 inside."""
    w = np.ones(n)
    w[0] = w[-1] = 0.5
    return w


def cosine_eigenpairs(n, h):
    """(T, lam, Tinv) of stiffness(n, h) in closed form, lam increasing."""
    m = n - 1
    j = np.arange(n, dtype=np.int64)
    red = np.outer(j, j) % (2 * m)
    t = np.cos(math.pi * red.astype(np.float64) / m)
    lam = (4.0 / (h * h)) * np.sin(math.pi * j.astype(np.float64) / (2 * m)) ** 2
    c = np.full(n, m / 2.0)
    c[0] = c[-1] = float(m)
    tinv = (t.T * weights(n)[None, :]) / c[:, None]
    return t, lam, tinv


def apply_laplacian(u, hs):
    """A_h vec(U) by the mirrored central-difference stencil (ghost node =
    mirror image of the first interior neighbour); 2 or 3 dimensions."""
    out = np.zeros_like(u)
    for ax, h in enumerate(hs):
        n = u.shape[ax]
        lo_idx = np.concatenate([[1], np.arange(0, n - 1)])
        hi_idx = np.concatenate([np.arange(1, n), [n - 2]])
        lo = np.take(u, lo_idx, axis=ax)
        hi = np.take(u, hi_idx, axis=ax)
        out += (2.0 * u - lo - hi) / (h * h)
    return out


def assemble_laplacian(shape, hs):
    """Sparse A_h as the Kronecker sum of the 1D ghost-point matrices (x innermost)."""
    total = None
    for ax in range(len(shape)):
        factors = [sp.identity(n, format="csr") for n in shape]
        factors[ax] = sp.csr_matrix(stiffness(shape[ax], hs[ax]))
        term = factors[0]
        for f in factors[1:]:
            term = sp.kron(term, f, format="csr")
        total = term if total is None else total + term
    return total


def residual_cubic(u, f, hs, lin=0.0, cub=1.0, pot=None, quad=0.0):
    """F^h(U) = A_h U + lin U + quad U^2 + cub U^3 + V U - F (pot = V on the
    nodes, None = 0)."""
    r = apply_laplacian(u, hs) + lin * u + quad * u ** 2 + cub * u ** 3 - f
    return r if pot is None else r + pot * u


def fu_cubic(u, lin=0.0, cub=1.0, pot=None, quad=0.0):
    """Jacobian diagonal of the pointwise part: 3 cub U^2 + 2 quad U + lin + V."""
    d = 3.0 * cub * u * u + 2.0 * quad * u + lin
    return d if pot is None else d + pot


def fdm_solve(r, hs, shift, scale=1.0):
    """X = (scale A_h + shift I)^-1 R by eq. fin_inverse with the cosine modes."""
    eig = [cosine_eigenpairs(n, h) for n, h in zip(r.shape, hs)]
    y = r
    for ax, (_, _, tinv) in enumerate(eig):
        y = mode_product(y, tinv, ax)
    d = np.zeros(r.shape)
    for ax, (_, lam, _) in enumerate(eig):
        bshape = [1] * r.ndim
        bshape[ax] = r.shape[ax]
        d = d + lam.reshape(bshape)
    y = y / (scale * d + shift)
    for ax, (t, _, _) in enumerate(eig):
        y = mode_product(y, t, ax)
    return y


def direct_solve(r, hs, shift, scale=1.0):
    """X = (scale A_h + shift I)^-1 R by a direct solve of the assembled system."""
    a = assemble_laplacian(r.shape, hs) * scale + shift * sp.identity(r.size, format="csr")
    if r.size <= 4096:
        x = np.linalg.solve(a.toarray(), r.ravel())
    else:
        x = spla.spsolve(a.tocsc(), r.ravel())
    return np.asarray(x).reshape(r.shape)


def shift_of(rule, fu, beta):
    """beta_k by the rule: "mid" (min + max)/2, "max", "sum" (min + max), "min"
    of the Jacobian diagonal fu, or "fixed" (the rules compared in the tables
    of Sections 6.2-6.3)."""
    lo, hi = float(fu.min()), float(fu.max())
    return {"mid": 0.5 * (lo + hi), "max": hi, "sum": lo + hi, "min": lo, "fixed": beta}[rule]


def qn_solve(f, hs, lin=0.0, u0=None, beta=0.0, midpoint=True, rtol=1e-10, max_iter=200,
             solver=fdm_solve, cub=1.0, pot=None, rule=None, quad=0.0):
    """The quasi-Newton iteration for the cubic problem: R_k = F^h(U_k); stop
    when ||R_k|| / ||F|| <= rtol (or after max_iter solves); beta_k = the fixed
    beta or the midpoint of 3 cub U_k^2 + lin + V (rule: another shift rule of
    shift_of); U_{k+1} = U_k - (A_h + beta_k I)^-1 R_k.  f, u0, pot: arrays of the grid's shape.  Returns
    dict(u, iters, relres, beta)."""
    f = np.asarray(f, dtype=np.float64)
    u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.float64, copy=True)
    fnorm = math.sqrt(float(np.sum(f * f)))
    hist, betas = [], []
    k = 0
    while True:
        r = residual_cubic(u, f, hs, lin, cub, pot, quad)
        rel = math.sqrt(float(np.sum(r * r))) / fnorm
        hist.append(rel)
        if rel <= rtol or k >= max_iter or not math.isfinite(rel):
            break
        r_ = rule if rule is not None else ("mid" if midpoint else "fixed")
        b = shift_of(r_, fu_cubic(u, lin, cub, pot, quad), beta)
        betas.append(b)
        u = u - solver(r, hs, b)
        k += 1
    return {"u": u, "iters": k, "relres": hist, "beta": betas, "converged": hist[-1] <= rtol}
