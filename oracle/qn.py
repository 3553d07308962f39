"""The quasi-Newton iteration (oracle; test-only).

Section 4, eq. identity-method: vec(U_{n+1}) = vec(U_n) - [A_h + beta_n I]^-1
F^h(U_n), with the midpoint shift beta_n = (lam_max + lam_min)((N_h)_U(U_n)) / 2
(Section 4, and Theorem thm:convergence).  (N_h)_U is diagonal for a pointwise
nonlinearity (the remark after the theorem), so its extreme eigenvalues are the
min / max of f_u over the grid.  For the 2-component system the eigenvalues of
each 2x2 block (Section 4.3, eq. eigenvalues) are used: beta = (min lam_- +
max lam_+) / 2 over all points.

Stopping rule (the paper iterates "until the residual is sufficiently small"
without a number): relative Euclidean residual ||F^h(U_k)||_2 / ||F||_2 <= rtol,
with F the source term; the iteration count is the number of solves performed.

Quasi-linear problem: the Jacobian approximation is c_k A_h + beta I with
c_k = (min a(U_k) + max a(U_k)) / 2, a(u) = 1 + u^2, i.e. the midpoint idea
applied to the diffusion coefficient (a reading; the paper's theory covers the
semilinear case only).
"""

import math

import numpy as np

from . import operators as ops
from .tensor import fdm_solve, direct_solve

CUBIC = "cubic"
SYSTEM = "system"
QUASILINEAR = "quasilinear"


def residual(kind, u, f, lin=0.0, cub=1.0, pot=None, quad=0.0):
    """F^h(U) for the problem kind; u, f carry a leading component axis.
    lin, cub, pot: the cubic problem's linear coefficient, cubic coefficient
    and potential field (see operators.residual_cubic)."""
    if kind == CUBIC:
        return ops.residual_cubic(u[0], f[0], lin, cub, pot, quad)[None]
    if kind == SYSTEM:
        r1, r2 = ops.residual_system(u[0], u[1], f[0], f[1])
        return np.stack([r1, r2])
    if kind == QUASILINEAR:
        return ops.residual_quasilinear(u[0], f[0])[None]
    raise ValueError(kind)


def shift_rule(kind, u, beta, midpoint, lin=0.0, cub=1.0, pot=None, quad=0.0, rule=None):
    """Return (scale c_k, shift beta_k) of the Jacobian approximation.  The
    shift comes from the range [lo, hi] of the Jacobian diagonal (cubic) or of
    the 2x2 block eigenvalues (system, Section 4.3 eq. eigenvalues): its
    midpoint (Section 4), or by `rule` "max" (hi), "sum" (lo + hi), "min" (lo),
    the alternatives the tables of Sections 6.2-6.3 compare; else the fixed
    beta."""
    if kind == QUASILINEAR:
        a = ops.coeff_quasilinear(u[0])
        return 0.5 * (float(a.min()) + float(a.max())), beta
    if rule is None and not midpoint:
        return 1.0, beta
    if kind == CUBIC:
        fu = ops.fu_cubic(u[0], lin, cub, pot, quad)
        lo, hi = float(fu.min()), float(fu.max())
    else:
        lm, lp = ops.system_jacobian_eigs(u[0], u[1])
        lo, hi = float(lm.min()), float(lp.max())
    r = "mid" if rule is None else rule
    return 1.0, {"mid": 0.5 * (lo + hi), "max": hi, "sum": lo + hi, "min": lo}[r]


def qn_solve(kind, f, u0=None, beta=0.0, midpoint=False, rtol=1e-10,
             max_iter=200, solver=fdm_solve, lin=0.0, cub=1.0, pot=None, quad=0.0, rule=None):
    """Run the quasi-Newton iteration (shift: see shift_rule; rule overrides
    midpoint).

    f, u0: arrays of shape (ncomp, .., ny, nx).  Runs until relres <= rtol or
    max_iter solves.  Returns dict(u, iters, relres (history, one entry per
    residual evaluation), beta (per solve), scale (per solve), converged).
    """
    f = np.asarray(f, dtype=np.float64)
    u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.float64, copy=True)
    fnorm = math.sqrt(float(np.sum(f * f)))
    hist, betas, scales = [], [], []
    k = 0
    while True:
        r = residual(kind, u, f, lin, cub, pot, quad)
        rel = math.sqrt(float(np.sum(r * r))) / fnorm
        hist.append(rel)
        if rel <= rtol or k >= max_iter or not math.isfinite(rel):
            break
        c, b = shift_rule(kind, u, beta, midpoint, lin, cub, pot, quad, rule)
        betas.append(b)
        scales.append(c)
        for comp in range(u.shape[0]):
            u[comp] -= solver(r[comp], b, c)
        k += 1
    return {"u": u, "iters": k, "relres": hist, "beta": betas, "scale": scales,
            "converged": hist[-1] <= rtol}


def newton_solve(kind, f, u0=None, tol=1e-13, max_iter=30, lin=0.0, cub=1.0, pot=None):
    """Dense Newton's method (Section 4, eq. newton) for tiny grids: the
    Jacobian A_h + (N_h)_U is assembled and solved directly.  Used only to pin
    the fixed point of the quasi-Newton iteration."""
    f = np.asarray(f, dtype=np.float64)
    u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.float64, copy=True)
    shape = f.shape[1:]
    a = ops.assemble_laplacian(shape).toarray()
    n = a.shape[0]
    fnorm = math.sqrt(float(np.sum(f * f)))
    for _ in range(max_iter):
        r = residual(kind, u, f, lin, cub, pot)
        if math.sqrt(float(np.sum(r * r))) / fnorm <= tol:
            break
        if kind == CUBIC:
            jac = a + np.diag(ops.fu_cubic(u[0], lin, cub, pot).ravel())
            u[0] -= np.linalg.solve(jac, r[0].ravel()).reshape(shape)
        elif kind == SYSTEM:
            jac = np.zeros((2 * n, 2 * n))
            jac[:n, :n] = a + np.diag(3.0 * u[0].ravel() ** 2)
            jac[n:, n:] = a + np.diag(3.0 * u[1].ravel() ** 2)
            jac[:n, n:] = -np.eye(n)
            jac[n:, :n] = -np.eye(n)
            du = np.linalg.solve(jac, r.reshape(2 * n))
            u -= du.reshape(u.shape)
        else:
            raise ValueError(kind)
    return u


def contraction_bound(fu_min, fu_max, lam_min_a, beta):
    """g(beta) of the remark on the optimal beta (Section 5): the bound
    max_mu |beta - mu| / (lam_min(A_h) + beta) on the linear error-propagation
    factor (eq. norm_ratio)."""
    return max(abs(beta - fu_min), abs(beta - fu_max)) / (lam_min_a + beta)


__all__ = ["CUBIC", "SYSTEM", "QUASILINEAR", "residual", "shift_rule", "qn_solve",
           "newton_solve", "contraction_bound", "direct_solve", "fdm_solve"]
