"""Reference of the split-bf16 products (oracle; test-only).

Not part of the paper: the reduced-precision transforms of the solver run
their mode products on bf16 matrix cores with each FP32 operand split into
bfloat16 parts (the method of Henry, Tang & Heinecke, "Leveraging the
bfloat16 artificial intelligence datatype for higher-precision computations",
ARITH 2019):

    x0 = bf16(x),  x1 = bf16(x - x0),  x2 = bf16(x - x0 - x1)   (round to nearest even)

and a product keeps the part products A_i B_j with i + j < NP:
NP = 2 ("bf16x3": A0B0 + A0B1 + A1B0) or NP = 3 ("bf16x6": the six pairs with
i + j < 3).  Here the part products are exact (bf16 x bf16 fits in FP64) and
summed in FP64, so this reference carries only the splitting and truncation
error of the method, not the FP32 accumulation of the matrix cores.
Pinned in tests/test_oracle_splitbf16.py by brute-force rounding and by the
error bound against the FP64 product.
"""

import numpy as np


def bf16_rne(x):
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as
    FP32.  Finite inputs only."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32)


def split(x, parts):
    """The bf16 parts of FP32 x (list of `parts` FP32 arrays holding bf16 values);
    the remainders are formed in FP32."""
    x = np.asarray(x, dtype=np.float32)
    out = []
    rem = x
    for _ in range(parts):
        p = bf16_rne(rem)
        out.append(p)
        rem = (rem - p).astype(np.float32)
    return out


def split_matmul(a, b, parts):
    """sum_{i + j < parts} A_i @ B_j in FP64 (A, B rounded to FP32 first)."""
    pa = split(a, parts)
    pb = split(b, parts)
    c = np.zeros((np.shape(a)[0], np.shape(b)[1]))
    for i in range(parts):
        for j in range(parts - i):
            c += pa[i].astype(np.float64) @ pb[j].astype(np.float64)
    return c


def split_mode_product(x, m, axis, parts):
    """Y = X x_axis M (Y[.., i, ..] = sum_k M[i, k] X[.., k, ..]) with every
    scalar product taken as the split-bf16 product of the FP32-rounded
    operands, summed exactly, the result rounded to FP32 (the storage of the
    reduced-precision transforms)."""
    xm = np.moveaxis(np.asarray(x), axis, 0)
    shp = xm.shape
    y = split_matmul(m, xm.reshape(shp[0], -1), parts)
    return np.moveaxis(y.astype(np.float32).reshape((m.shape[0],) + shp[1:]), 0, axis)


def split_fdm_solve(r, shift, parts, scale=1.0):
    """X = (scale A_h + shift I)^-1 R by the tensor-product formula (Section 4.1,
    eq. fin_inverse) with split-bf16 mode products: R rounded to FP32, the
    forward sine transform along every axis, the divide by scale (lam_i + lam_j
    (+ lam_k)) + shift in FP64 rounded to FP32, the inverse transforms.  Every
    product and the divide see FP32 inputs and store FP32 results; the only
    difference from the matrix cores is their FP32 accumulation order.
    Dirichlet finite differences (sine eigenvectors, T^-1 = T).

    In exact arithmetic the order of the mode products is immaterial; with a
    rounding after every product it is not (two orders differ by about the
    split error itself), so it is fixed here: the forward products from the
    x axis (the last array axis, the innermost Kronecker factor of the vec
    order) outwards, the inverse products in the reverse order."""
    from .spectral import sine_eigenpairs
    from .tensor import spectral_denominator

    ts = [sine_eigenpairs(n)[0] for n in r.shape]
    axes = list(range(r.ndim))
    y = np.asarray(r, dtype=np.float32)
    for ax in reversed(axes):
        y = split_mode_product(y, ts[ax].T, ax, parts)
    y = (y.astype(np.float64) / spectral_denominator(r.shape, shift, scale)).astype(np.float32)
    for ax in axes:
        y = split_mode_product(y, ts[ax], ax, parts)
    return y.astype(np.float64)
