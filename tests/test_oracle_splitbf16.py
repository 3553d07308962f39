"""Pins for oracle.splitbf16: round-to-nearest-even to bfloat16 against brute
force, the exactness of the parts, and the error of the split products
against the FP64 product (bounds from the splitting: each RNE step to an
8-bit significand leaves a remainder <= 2^-8 of its input)."""

import math

import numpy as np
import pytest

from oracle import splitbf16 as sb


def brute_bf16(x):
    """Nearest bfloat16 by enumerating the two neighbours on the bf16 grid."""
    out = np.empty_like(x)
    for i, v in enumerate(x):
        bits = int(np.float32(v).view(np.uint32))
        lo = np.uint32(bits & 0xFFFF0000).view(np.float32)
        hi = np.uint32((bits & 0xFFFF0000) + 0x10000).view(np.float32)
        dlo, dhi = abs(float(v) - float(lo)), abs(float(hi) - float(v))
        if dlo < dhi:
            out[i] = lo
        elif dhi < dlo:
            out[i] = hi
        else:  # tie: the even significand
            out[i] = lo if ((bits >> 16) & 1) == 0 else hi
    return out


def test_rne_matches_brute_force():
    rng = np.random.default_rng(0)
    x = np.concatenate([(rng.standard_normal(4000) * 10.0 ** rng.integers(-6, 6, 4000)).astype(np.float32),
                        # exact ties: bf16 grid value + half an ulp, both parities
                        (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32),
                        np.array([0.0, -0.0, 1.0, -3.5], np.float32)])
    assert np.array_equal(sb.bf16_rne(x).view(np.uint32), brute_bf16(x).view(np.uint32))


def test_parts_are_bf16_and_reconstruct():
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(10000) * 3.0).astype(np.float32)
    for parts, bound in ((2, 2.0 ** -16), (3, 2.0 ** -24)):
        p = sb.split(x, parts)
        for q in p:  # every part is representable in bf16: low 16 bits zero
            assert np.all(q.view(np.uint32) & 0xFFFF == 0)
        rec = sum(q.astype(np.float64) for q in p)
        err = np.abs(rec - x.astype(np.float64))
        assert np.all(err <= bound * np.abs(x.astype(np.float64)) * 1.0001)


@pytest.mark.parametrize("parts,coef", [(2, 3 * 2.0 ** -16), (3, 6 * 2.0 ** -24)])
def test_split_product_error_bound(parts, coef):
    """|C_split - A B| <= coef * (|A| |B|) entrywise: bf16x3 drops A1 B1 and the
    remainders below the two parts (each <= 2^-16 of an operand); bf16x6 drops
    the pairs with i + j >= 3 and the remainders below three parts (2^-24)."""
    rng = np.random.default_rng(2 + parts)
    a = rng.standard_normal((64, 512)).astype(np.float32)
    b = rng.standard_normal((512, 48)).astype(np.float32)
    a64, b64 = a.astype(np.float64), b.astype(np.float64)
    c = sb.split_matmul(a, b, parts)
    ref = a64 @ b64
    bound = coef * (np.abs(a64) @ np.abs(b64))
    assert np.all(np.abs(c - ref) <= bound)
    # and the split is not trivially exact: one part alone is far less accurate
    c1 = sb.split_matmul(a, b, 1)
    assert np.max(np.abs(c1 - ref) / bound) > 10.0


@pytest.mark.parametrize("shape", [(31, 31), (9, 12, 17)])
def test_split_solve_against_the_fp64_solve_and_a_direct_solve(shape):
    """The split-bf16 tensor-product solve carries the splitting error and
    nothing else: bf16x6 (three parts) is within FP32 storage error of the
    FP64 solve (and of a dense direct solve, which shares no step with it);
    bf16x3 (two parts) is within sqrt(6) 2^-16 of it but clearly not at FP32
    level; a one-part product (plain bf16) misses the bf16x3 bound."""
    from oracle import tensor as ot
    rng = np.random.default_rng(5)
    r = rng.standard_normal(shape)
    ref = ot.direct_solve(r, 0.7)
    assert np.linalg.norm(ot.fdm_solve(r, 0.7) - ref) <= 1e-13 * np.linalg.norm(ref)
    err = {p: np.linalg.norm(sb.split_fdm_solve(r, 0.7, p) - ref) / np.linalg.norm(ref)
           for p in (1, 2, 3)}
    assert err[3] <= 3e-7
    assert 3e-7 < err[2] <= math.sqrt(6) * 2.0 ** -16
    assert err[1] > 10 * math.sqrt(6) * 2.0 ** -16


def test_split_solve_scale_and_exact_modes():
    """A single sine mode: the FP64 solve returns it divided by its
    eigenvalue sum plus the shift; the split solve within its bound, and the
    scale multiplies the eigenvalue sum (not the shift)."""
    from oracle.spectral import sine_eigenpairs
    n = (15, 20)
    (ty, ly), (tx, lx) = sine_eigenpairs(n[0]), sine_eigenpairs(n[1])
    r = np.outer(ty[:, 2], tx[:, 5])
    for scale, shift in ((1.0, 0.0), (2.5, 3.0)):
        want = r / (scale * (ly[2] + lx[5]) + shift)
        got = sb.split_fdm_solve(r, shift, 2, scale=scale)
        assert np.linalg.norm(got - want) <= math.sqrt(6) * 2.0 ** -16 * np.linalg.norm(want)


def test_split_solve_product_order_matters_at_the_split_error_level():
    """With a rounding after every product the axis order changes the result
    by about the split error (so a reference must fix it), while in FP64 it
    does not."""
    from oracle import tensor as ot
    from oracle.spectral import sine_eigenpairs
    rng = np.random.default_rng(6)
    r = rng.standard_normal((21, 26))
    got = sb.split_fdm_solve(r, 0.3, 2)
    ty, tx = sine_eigenpairs(21)[0], sine_eigenpairs(26)[0]
    # the other order: y first forward, x first inverse
    y = np.asarray(r, dtype=np.float32)
    y = sb.split_mode_product(y, ty.T, 0, 2)
    y = sb.split_mode_product(y, tx.T, 1, 2)
    y = (y.astype(np.float64) / ot.spectral_denominator(r.shape, 0.3)).astype(np.float32)
    y = sb.split_mode_product(y, tx, 1, 2)
    y = sb.split_mode_product(y, ty, 0, 2).astype(np.float64)
    ref = ot.fdm_solve(r, 0.3)
    d = np.linalg.norm(y - got) / np.linalg.norm(ref)
    assert 1e-6 < d < math.sqrt(6) * 2.0 ** -16
