"""Tensor-product inverse of (c A_h + shift I) and direct solves (oracle; test-only).

Section 4.1 (eq. fin_inverse): with H_a = T_a Lambda_a T_a^-1 per axis,
(A_h + beta I)^-1 R is obtained by transforming R with T_a^-1 along every
axis, dividing element-wise by Lambda_i + Lambda_j (+ Lambda_k) + beta, and
transforming back with T_a.  The 3D form applies the same mode products along
three axes (the tensor-product identity (C (x) B (x) A) vec(X) of Section 4.1).
For the finite-difference stiffness matrix T is the orthonormal symmetric sine
matrix, so T^-1 = T.

The scale c multiplies A_h (c = 1 gives the paper's operator; the quasi-linear
problem uses c_k, the midpoint of the coefficient a(U) = 1 + U^2).
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operators import assemble_laplacian
from .spectral import sine_eigenpairs


def mode_product(x, m, axis):
    """Y = X x_axis M: Y[.., i, ..] = sum_k M[i, k] X[.., k, ..] along `axis`."""
    y = np.tensordot(m, x, axes=([1], [axis]))
    return np.moveaxis(y, 0, axis)


def kron_apply(mats, x):
    """Explicit Kronecker matrix times vec(X), for pinning mode_product.

    mats are per array axis (.., y, x); the matrix is mats[0] (x) ... (x)
    mats[-1] acting on the C-order ravel (x innermost), i.e. the paper's
    (C (x) B (x) A) vec(X) with A acting on x.
    """
    k = mats[0]
    for m in mats[1:]:
        k = np.kron(k, m)
    return (k @ x.ravel()).reshape(x.shape)


def spectral_denominator(shape, shift, scale=1.0):
    """D[.., j, i] = scale * (lam_i + lam_j (+ lam_k)) + shift on the eigen-grid."""
    lams = [sine_eigenpairs(n)[1] for n in shape]
    d = np.zeros(shape)
    for ax, lam in enumerate(lams):
        bshape = [1] * len(shape)
        bshape[ax] = shape[ax]
        d = d + lam.reshape(bshape)
    return scale * d + shift


def fdm_solve(r, shift, scale=1.0):
    """X = (scale A_h + shift I)^-1 R by eq. fin_inverse (forward sine transforms
    along every axis, element-wise divide, inverse transforms)."""
    ts = [sine_eigenpairs(n)[0] for n in r.shape]
    y = r
    for ax, t in enumerate(ts):
        y = mode_product(y, t.T, ax)  # T^-1 = T^T
    y = y / spectral_denominator(r.shape, shift, scale)
    for ax, t in enumerate(ts):
        y = mode_product(y, t, ax)
    return y


def direct_solve(r, shift, scale=1.0):
    """X = (scale A_h + shift I)^-1 R by a direct solve of the assembled system
    (dense LU up to 4096 unknowns, sparse LU above)."""
    a = assemble_laplacian(r.shape) * scale + shift * sp.identity(r.size, format="csr")
    if r.size <= 4096:
        x = np.linalg.solve(a.toarray(), r.ravel())
    else:
        x = spla.spsolve(a.tocsc(), r.ravel())
    return np.asarray(x).reshape(r.shape)
