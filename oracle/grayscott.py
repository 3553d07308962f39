"""The steady-state Gray-Scott system with the damped quasi-Newton iteration
(oracle; test-only).

Section 6.2 (eq. 2dgrayeq) on Omega = (0, 1)^2 with zero normal derivative:

    -D_A Lap A - S A^2 + (mu + rho) A = 0,
    -D_S Lap S + S A^2 - rho (1 - S) = 0.

Discretisation: finite differences with ghost nodes as in the Neumann case of
Section 3.2 (all n nodes per axis, h = 1 / (n - 1)).  Reading of the
splitting F^h = A_h U + N_h(U) (Section 4) for a system whose components
diffuse at different rates: A_h = blockdiag(D_A A, D_S A) with A the discrete
-Lap, and every reaction term, the linear ones included, in N_h; the constant
rho of the second equation is the source, F = (0, rho), so the stopping rule
||F^h(U) - F|| / ||F|| of the other problems applies:

    R = (D_A A A - S A^2 + (mu + rho) A,  D_S A S + S A^2 + rho S - rho).

The Jacobian of N_h is the 2 x 2 block per node of Section 4.3

    [[a, b], [c, d]] = [[-2 S A + mu + rho, -A^2], [2 S A, A^2 + rho]],

whose eigenvalues are eq. eigenvalues; b c = -2 S A^3 can make the
discriminant negative, and then both eigenvalues are read as their common
real part (a + d) / 2 (the shift is real).  beta_k is the midpoint
(min lam_- + max lam_+) / 2 over the nodes (Section 4), and the step of
Section 4 (eq. identity-method) is shortened by the step size tau the paper
uses for this example (0.1):

    U_{k+1} = U_k - tau (A_h + beta_k I)^-1 (F^h(U_k) - F),

the inverse applied per component, (D_c A + beta_k I)^-1, by the
tensor-product formula of Section 4.1 (eq. fin_inverse) with the cosine
modes.  lam_min(A) = 0, so the solve needs beta_k > 0.

Constant states solve the algebraic system alone (A of a constant is zero):
the trivial state (0, 1) always, and for rho > 4 (mu + rho)^2 the two states
with S A = mu + rho, (mu + rho) A^2 - rho A + rho (mu + rho) = 0.
"""

import math

import numpy as np

from . import neumann as nm

PAPER_PARAMS = {"da": 2.5e-4, "ds": 5e-4, "rho": 0.04, "mu": 0.065}  # Section 6.2


def spacing(n):
    """h of the n nodes per axis of [0, 1] (both ends included)."""
    return 1.0 / (n - 1)


def source(shape, rho):
    """F = (0, rho) on every node; shape (2, ny, nx)."""
    f = np.zeros((2,) + tuple(shape))
    f[1] = rho
    return f


def residual(u, f, hs, da, ds, rho, mu):
    """F^h(A, S) - F for u = (A, S), f = (F_A, F_S)."""
    a, s = u[0], u[1]
    sa2 = s * a * a
    ra = da * nm.apply_laplacian(a, hs) - sa2 + (mu + rho) * a - f[0]
    rs = ds * nm.apply_laplacian(s, hs) + sa2 + rho * s - f[1]
    return np.stack([ra, rs])


def block_entries(u, rho, mu):
    """a = (N1)_A, b = (N1)_S, c = (N2)_A, d = (N2)_S per node."""
    a, s = u[0], u[1]
    return -2.0 * s * a + mu + rho, -a * a, 2.0 * s * a, a * a + rho


def block_eigs(u, rho, mu):
    """(lam_-, lam_+) per node by eq. eigenvalues; a negative discriminant
    gives the common real part for both."""
    a, b, c, d = block_entries(u, rho, mu)
    disc = (a - d) ** 2 + 4.0 * b * c
    root = np.sqrt(np.maximum(disc, 0.0))
    return 0.5 * (a + d - root), 0.5 * (a + d + root)


def midpoint_shift(u, rho, mu):
    lm, lp = block_eigs(u, rho, mu)
    return 0.5 * (float(lm.min()) + float(lp.max()))


def solve(r, hs, diff, beta):
    """Per component c: (D_c A + beta I)^-1 R_c (eq. fin_inverse)."""
    return np.stack([nm.fdm_solve(r[c], hs, beta, scale=diff[c]) for c in range(2)])


def qn_solve(u0, n, da, ds, rho, mu, tau=0.1, beta=None, rtol=1e-10, max_iter=20000):
    """The damped iteration from u0 (shape (2, n, n)); beta = None: the
    midpoint shift, else that fixed shift.  Stops at ||F^h(U_k) - F|| / ||F||
    <= rtol, after max_iter solves, at a non-finite residual, or when the
    shift leaves A_h + beta_k I not positive definite (beta_k <= 0).  Returns
    dict(u, iters, relres (history), beta (per solve), converged, singular)."""
    hs = (spacing(n), spacing(n))
    f = source((n, n), rho)
    u = np.array(u0, dtype=np.float64, copy=True)
    fnorm = math.sqrt(float(np.sum(f * f)))
    hist, betas = [], []
    k = 0
    singular = False
    while True:
        r = residual(u, f, hs, da, ds, rho, mu)
        rel = math.sqrt(float(np.sum(r * r))) / fnorm
        hist.append(rel)
        if rel <= rtol or k >= max_iter or not math.isfinite(rel):
            break
        b = midpoint_shift(u, rho, mu) if beta is None else float(beta)
        if b <= 0.0:
            singular = True
            break
        betas.append(b)
        u = u - tau * solve(r, hs, (da, ds), b)
        k += 1
    return {"u": u, "iters": k, "relres": hist, "beta": betas,
            "converged": hist[-1] <= rtol, "singular": singular}


def homogeneous_states(rho, mu):
    """The spatially constant roots (A, S): (0, 1) and, when
    rho > 4 (mu + rho)^2, the two with S A = mu + rho."""
    out = [(0.0, 1.0)]
    k = mu + rho
    disc = rho * rho - 4.0 * rho * k * k
    if disc > 0.0:
        for sgn in (-1.0, 1.0):
            a = (rho + sgn * math.sqrt(disc)) / (2.0 * k)
            out.append((a, k / a))
    return out


def newton_solve(u0, n, da, ds, rho, mu, tol=1e-13, max_iter=50):
    """Dense Newton's method on the assembled system (tiny n only), to pin
    the roots the damped iteration reaches."""
    hs = (spacing(n), spacing(n))
    f = source((n, n), rho)
    lap = nm.assemble_laplacian((n, n), hs).toarray()
    m = n * n
    u = np.array(u0, dtype=np.float64, copy=True)
    fnorm = math.sqrt(float(np.sum(f * f)))
    for _ in range(max_iter):
        r = residual(u, f, hs, da, ds, rho, mu)
        if math.sqrt(float(np.sum(r * r))) / fnorm <= tol:
            break
        a, b, c, d = (x.ravel() for x in block_entries(u, rho, mu))
        jac = np.zeros((2 * m, 2 * m))
        jac[:m, :m] = da * lap + np.diag(a)
        jac[:m, m:] = np.diag(b)
        jac[m:, :m] = np.diag(c)
        jac[m:, m:] = ds * lap + np.diag(d)
        u = u - np.linalg.solve(jac, r.reshape(2 * m)).reshape(u.shape)
    return u
