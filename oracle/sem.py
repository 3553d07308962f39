"""Spectral element discretisation, Q^k with Gauss-Lobatto nodes (oracle;
test-only).

Section 3.1 (eqs. discrete-system, vectorized-system, final-system, and the
remark on the integration): per axis the interval of length L is cut into E
equal elements of order k; the nodes are the (k+1)-point Gauss-Lobatto
points of every element (shared at element ends), the basis the Lagrange
polynomials at those nodes, and every integral is taken by the same
Gauss-Lobatto rule.  Hence the mass matrix M is diagonal (its entries are the
quadrature weights summed over the elements that share the node), the
stiffness matrix S_ij = sum_e sum_q w_q psi_i'(x_q) psi_j'(x_q), and the
nonlinearity acts node by node: after multiplying by M^-1 the discrete
problem is A_h U + f(U) - F = 0 with A_h the Kronecker sum of H = M^-1 S.
Homogeneous Dirichlet data keep the E k - 1 interior nodes (the rows and
columns of the end nodes are removed); homogeneous Neumann data keep all
E k + 1 nodes (the boundary integral vanishes).

Section 4.2: H = M^-1/2 (M^-1/2 S M^-1/2) M^1/2 with a symmetric middle
factor, so H = T Lam T^-1 with T = M^-1/2 T~ (T~ orthonormal); here the pair
comes from scipy's generalised symmetric eigensolver S T = M T Lam
(T^T M T = I, so T^-1 = T^T M).  The solve and the quasi-Newton loop are
those of Sections 4 and 4.1.  Problem: -Lap u + lin u + quad u^2 + cub u^3 + V u = f.
Pinned in tests/test_oracle_sem.py.
"""

import math

import numpy as np
import scipy.linalg
from numpy.polynomial import legendre as leg

from .tensor import mode_product


def gauss_lobatto(k):
    """(k+1) Gauss-Lobatto nodes on [-1, 1] (ascending) and weights: the ends
    and the roots of P_k', weights 2 / (k (k+1) P_k(x)^2)."""
    ck = np.zeros(k + 1)
    ck[k] = 1.0
    inner = leg.legroots(leg.legder(ck)) if k > 1 else np.array([])
    x = np.concatenate([[-1.0], np.sort(inner), [1.0]])
    pk = leg.legval(x, ck)
    return x, 2.0 / (k * (k + 1) * pk * pk)


def lagrange_derivative(x):
    """D[q, p] = psi_p'(x_q) for the Lagrange basis at nodes x (direct formula)."""
    n = len(x)
    d = np.zeros((n, n))
    for p in range(n):
        for q in range(n):
            if p != q:
                num = 1.0
                for m in range(n):
                    if m != p and m != q:
                        num *= x[q] - x[m]
                den = 1.0
                for m in range(n):
                    if m != p:
                        den *= x[p] - x[m]
                d[q, p] = num / den
            else:
                d[q, p] = sum(1.0 / (x[p] - x[m]) for m in range(n) if m != p)
    return d


def nodes_and_matrices(elements, k, length, bc):
    """Global nodes (of the unknowns), lumped mass diagonal and stiffness
    matrix of one axis on [0, L] (Dirichlet: interior nodes; Neumann: all)."""
    xi, w = gauss_lobatto(k)
    dref = lagrange_derivative(xi)
    he = length / elements
    ntot = elements * k + 1
    x = np.zeros(ntot)
    m = np.zeros(ntot)
    s = np.zeros((ntot, ntot))
    jac = he / 2.0
    # element stiffness: sum_q w_q psi_p'(x_q) psi_r'(x_q) with d/dx = (2/he) d/dxi
    ke = (dref.T * w) @ dref / jac
    for e in range(elements):
        idx = e * k + np.arange(k + 1)
        x[idx] = e * he + (xi + 1.0) * jac
        m[idx] += w * jac
        s[np.ix_(idx, idx)] += ke
    if bc == "dirichlet":
        keep = np.arange(1, ntot - 1)
        return x[keep], m[keep], s[np.ix_(keep, keep)]
    return x, m, s


def axis_operator(elements, k, length, bc):
    """H = M^-1 S of one axis, and its eigen-decomposition (T, lam, T^-1)."""
    x, m, s = nodes_and_matrices(elements, k, length, bc)
    h = s / m[:, None]
    lam, t = scipy.linalg.eigh(s, np.diag(m))
    return x, m, h, t, lam, t.T * m[None, :]


def apply_a(u, ops_):
    """A_h U = sum over axes of H applied along that axis (array-axis order)."""
    out = np.zeros_like(u)
    for ax, op in enumerate(ops_):
        out += mode_product(u, op[2], ax)
    return out


def residual_cubic(u, f, ops_, lin=0.0, cub=1.0, pot=None, quad=0.0):
    r = apply_a(u, ops_) + lin * u + quad * u ** 2 + cub * u ** 3 - f
    return r if pot is None else r + pot * u


def fu_cubic(u, lin=0.0, cub=1.0, pot=None, quad=0.0):
    d = 3.0 * cub * u * u + 2.0 * quad * u + lin
    return d if pot is None else d + pot


def fdm_solve(r, ops_, shift, scale=1.0):
    """(scale A_h + shift I)^-1 R by the tensor-product formula (Section 4.1)."""
    y = r
    for ax, op in enumerate(ops_):
        y = mode_product(y, op[5], ax)
    d = np.zeros(r.shape)
    for ax, op in enumerate(ops_):
        bshape = [1] * r.ndim
        bshape[ax] = r.shape[ax]
        d = d + op[4].reshape(bshape)
    y = y / (scale * d + shift)
    for ax, op in enumerate(ops_):
        y = mode_product(y, op[3], ax)
    return y


def qn_solve(f, ops_, lin=0.0, cub=1.0, pot=None, u0=None, beta=0.0, midpoint=True,
             rtol=1e-10, max_iter=200, quad=0.0):
    """The quasi-Newton loop of Section 4 on the SEM operator: stop when
    ||R||_2 / ||F||_2 <= rtol; beta_k = midpoint of 3 cub U^2 + 2 quad U + lin + V
    or fixed."""
    u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.float64, copy=True)
    fnorm = math.sqrt(float(np.sum(f * f)))
    hist, betas = [], []
    k = 0
    while True:
        r = residual_cubic(u, f, ops_, lin, cub, pot, quad)
        rel = math.sqrt(float(np.sum(r * r))) / fnorm
        hist.append(rel)
        if rel <= rtol or k >= max_iter or not math.isfinite(rel):
            break
        if midpoint:
            fu = fu_cubic(u, lin, cub, pot, quad)
            b = 0.5 * (float(fu.min()) + float(fu.max()))
        else:
            b = beta
        betas.append(b)
        u = u - fdm_solve(r, ops_, b)
        k += 1
    return {"u": u, "iters": k, "relres": hist, "beta": betas, "converged": hist[-1] <= rtol}
