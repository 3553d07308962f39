"""1D stiffness matrices and their eigen-decompositions (oracle; test-only).

Section 3.2 (finite differences) gives, for homogeneous Dirichlet data on a
uniform grid, the interior stiffness matrix S = h^-2 tridiag(-1, 2, -1) with the
mass matrix M = I (eq. Sy and the bullet list before it).  Section 4.2 shows
that H = M^-1 S is diagonalised as H = T Lambda T^-1 with T = M^-1/2 T~, where
T~ diagonalises the symmetric M^-1/2 S M^-1/2.  For M = I this reduces to the
symmetric eigenproblem of S, whose eigenvectors are the discrete sine modes
(a textbook closed form that the paper does not print).
"""

import math

import numpy as np


def stiffness_matrix(n):
    """Dense S = h^-2 tridiag(-1, 2, -1) of order n, h = 1/(n+1) (Section 3.2)."""
    h = 1.0 / (n + 1)
    s = np.zeros((n, n))
    idx = np.arange(n)
    s[idx, idx] = 2.0
    s[idx[:-1], idx[:-1] + 1] = -1.0
    s[idx[:-1] + 1, idx[:-1]] = -1.0
    return s / (h * h)


def sine_eigenpairs(n):
    """Closed-form eigenpairs of stiffness_matrix(n).

    T[j, k] = sqrt(2/(n+1)) sin(j k pi/(n+1)), j, k = 1..n (orthonormal and
    symmetric, so T^-1 = T^T = T), lam[k] = (4/h^2) sin^2(k pi / (2(n+1))).
    The sine argument is reduced as an integer (j k mod 2(n+1)) before the
    multiplication by pi, so T is exactly symmetric.
    Returns (T, lam) with lam in increasing order.
    """
    m = n + 1
    j = np.arange(1, n + 1, dtype=np.int64)
    red = np.outer(j, j) % (2 * m)
    t = math.sqrt(2.0 / m) * np.sin(math.pi * red.astype(np.float64) / m)
    h = 1.0 / m
    lam = (4.0 / (h * h)) * np.sin(math.pi * j.astype(np.float64) / (2 * m)) ** 2
    return t, lam


def diagonalize(stiff, mass_diag):
    """Section 4.2: H = M^-1 S = T Lambda T^-1 for a diagonal SPD mass matrix.

    Forms the symmetric M^-1/2 S M^-1/2, diagonalises it (library symmetric
    eigensolver), and returns (T, lam, Tinv) with T = M^-1/2 T~ and
    Tinv = T~^T M^1/2.
    """
    mh = 1.0 / np.sqrt(mass_diag)
    sym = mh[:, None] * stiff * mh[None, :]
    lam, tt = np.linalg.eigh(sym)
    t = mh[:, None] * tt
    tinv = tt.T * np.sqrt(mass_diag)[None, :]
    return t, lam, tinv


def jacobi_eigh(a, tol=1e-15, max_sweeps=60):
    """Cyclic Jacobi eigenvalue algorithm for a symmetric matrix (textbook).

    Used only as an independent cross-check of the closed-form eigenpairs.
    Returns (lam, V) with eigenvalues ascending and eigenvectors in columns.
    """
    a = np.array(a, dtype=np.float64, copy=True)
    n = a.shape[0]
    v = np.eye(n)
    for _ in range(max_sweeps):
        off = math.sqrt(float(np.sum(np.tril(a, -1) ** 2)))
        if off <= tol * math.sqrt(float(np.sum(a * a))):
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = a[p, q]
                if apq == 0.0:
                    continue
                theta = (a[q, q] - a[p, p]) / (2.0 * apq)
                t = math.copysign(1.0, theta) / (abs(theta) + math.sqrt(theta * theta + 1.0))
                c = 1.0 / math.sqrt(t * t + 1.0)
                s = t * c
                ap = a[:, p].copy()
                aq = a[:, q].copy()
                a[:, p] = c * ap - s * aq
                a[:, q] = s * ap + c * aq
                ap = a[p, :].copy()
                aq = a[q, :].copy()
                a[p, :] = c * ap - s * aq
                a[q, :] = s * ap + c * aq
                vp = v[:, p].copy()
                vq = v[:, q].copy()
                v[:, p] = c * vp - s * vq
                v[:, q] = s * vp + c * vq
    lam = np.diag(a).copy()
    order = np.argsort(lam)
    return lam[order], v[:, order]
