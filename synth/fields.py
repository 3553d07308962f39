"""Seeded input generators (no solver arithmetic; see package docstring)."""

import math

import numpy as np

# Per-side interior sizes of the batched workload (uneven instance mix).
BATCH_SIZES = (63, 127, 255, 511, 1023)


def grid_coords(n):
    """Interior node coordinates x_i = i/(n+1), i = 1..n, on (0, 1)."""
    return np.arange(1, n + 1, dtype=np.float64) / (n + 1)


def _mesh(shape):
    """Coordinate arrays for a C-order (.., ny, nx) grid, x fastest."""
    axes = [grid_coords(n) for n in shape]
    return np.meshgrid(*axes, indexing="ij")


def manufactured_c1(n):
    """2D -Lap u + u^3 = f, u = sin(pi x) sin(pi y) (1 + x y).

    Returns (u_exact, f) sampled on the n x n interior grid, shape (ny, nx).
    -Lap u = 2 pi^2 s_x s_y (1+xy) - 2 pi (y c_x s_y + x s_x c_y).
    """
    y, x = _mesh((n, n))
    sx, sy = np.sin(math.pi * x), np.sin(math.pi * y)
    cx, cy = np.cos(math.pi * x), np.cos(math.pi * y)
    u = sx * sy * (1.0 + x * y)
    mlap = 2.0 * math.pi ** 2 * sx * sy * (1.0 + x * y) - 2.0 * math.pi * (
        y * cx * sy + x * sx * cy)
    return u, mlap + u ** 3


def manufactured_c2(n):
    """3D -Lap u + u^3 = f, u = sin(pi x) sin(pi y) sin(pi z) exp(x+y+z)/e^3.

    Returns (u_exact, f), shape (nz, ny, nx).  With g(t) = sin(pi t) e^t,
    g'' = e^t ((1 - pi^2) sin(pi t) + 2 pi cos(pi t)).  The fields are
    separable, so the 1D factors are evaluated once and broadcast.
    """
    t = grid_coords(n)
    g = np.sin(math.pi * t) * np.exp(t - 1.0)
    g2 = np.exp(t - 1.0) * ((1.0 - math.pi ** 2) * np.sin(math.pi * t)
                             + 2.0 * math.pi * np.cos(math.pi * t))
    gz, gy, gx = g[:, None, None], g[None, :, None], g[None, None, :]
    u = gz * gy * gx
    lap = g2[:, None, None] * gy * gx + gz * g2[None, :, None] * gx + gz * gy * g2[None, None, :]
    return u, -lap + u ** 3


def amplitude_c3(seed):
    """Seeded amplitude A ~ U[0.5, 2] of the quasi-linear manufactured solution."""
    return float(np.random.default_rng(seed).uniform(0.5, 2.0))


def manufactured_c3(n, amplitude):
    """3D -div((1+u^2) grad u) = f with u = A sin(pi x) sin(pi y) sin(pi z).

    -div((1+u^2) grad u) = -(1+u^2) Lap u - 2 u |grad u|^2 and Lap u = -3 pi^2 u,
    so f = 3 pi^2 u (1+u^2) - 2 u |grad u|^2.  Returns (u_exact, f); the 1D
    factors are evaluated once and broadcast.
    """
    t = grid_coords(n)
    s1, c1 = np.sin(math.pi * t), np.cos(math.pi * t)
    sz, sy, sx = s1[:, None, None], s1[None, :, None], s1[None, None, :]
    cz, cy, cx = c1[:, None, None], c1[None, :, None], c1[None, None, :]
    u = amplitude * (sz * sy * sx)
    grad2 = (amplitude * math.pi) ** 2 * (
        (sz * sy * cx) ** 2 + (sz * cy * sx) ** 2 + (cz * sy * sx) ** 2)
    f = 3.0 * math.pi ** 2 * u * (1.0 + u * u) - 2.0 * u * grad2
    return u, f


def random_field(shape, seed, scale=1.0):
    """Seeded i.i.d. N(0, scale^2) float64 array of the given shape."""
    return scale * np.random.default_rng(seed).standard_normal(shape)


def _sine_synthesis_matrix(n):
    """B[i, k] = sin(k pi x_i): samples sine mode k at interior node i."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return np.sin(math.pi * np.outer(i, i) / (n + 1))


def gaussian_random_field(n, length_scale, rng):
    """Zero-boundary Gaussian random field on the n x n interior grid.

    A sine series f(x, y) = sum_{k,l} sqrt(s_k s_l) xi_{kl} sin(k pi x) sin(l pi y)
    with xi ~ N(0,1) i.i.d. and the squared-exponential spectral weight
    s_k = exp(-(length_scale k pi)^2 / 2), then scaled to unit empirical
    variance over the grid.  Shape (ny, nx).
    """
    k = np.arange(1, n + 1, dtype=np.float64)
    s = np.exp(-0.5 * (length_scale * k * math.pi) ** 2)
    w = np.sqrt(np.outer(s, s))
    xi = rng.standard_normal((n, n))
    b = _sine_synthesis_matrix(n)
    f = b @ (w * xi) @ b.T
    std = math.sqrt(float(np.mean(f * f)))
    return f / std if std > 0 else f


def batched_instance(i):
    """Instance i of the batched workload: 2D, N drawn from BATCH_SIZES.

    Even i: scalar -Lap u + u^3 = f.  Odd i: 2-component system with sources
    (f1, f2).  Sources are unit-variance GRFs with length scale 0.1.
    Returns dict(n, ncomp, f) with f of shape (ncomp, n, n).
    """
    rng = np.random.default_rng(4000000 + i)
    n = int(BATCH_SIZES[int(rng.integers(0, len(BATCH_SIZES)))])
    ncomp = 1 if i % 2 == 0 else 2
    f = np.stack([gaussian_random_field(n, 0.1, rng) for _ in range(ncomp)])
    return {"n": n, "ncomp": ncomp, "f": f}


def learned_guess_rhs(seed, n=255):
    """Source for the learned-initial-guess workload: GRF with a seeded length
    scale in [0.05, 0.3] and amplitude in [1, 50].  Shape (n, n)."""
    rng = np.random.default_rng(seed)
    ell = float(rng.uniform(0.05, 0.3))
    amp = float(rng.uniform(1.0, 50.0))
    return amp * gaussian_random_field(n, ell, rng)


def node_coords(n, a=-1.0, b=1.0):
    """All n nodes x_j = a + j (b - a)/(n - 1), j = 0..n-1 (boundary included)."""
    return a + (b - a) * np.arange(n, dtype=np.float64) / (n - 1)


def neumann_2d(n):
    """2D -Lap u + u^3 + u = f on [-1, 1]^2 with zero normal derivative,
    u = cos(pi x) cos(2 pi y): -Lap u = 5 pi^2 u.  Sampled on all n x n nodes
    (boundary included).  Returns (u_exact, f), shape (ny, nx)."""
    x = node_coords(n)
    u = np.cos(2.0 * math.pi * x)[:, None] * np.cos(math.pi * x)[None, :]
    return u, 5.0 * math.pi ** 2 * u + u ** 3 + u


def neumann_3d(n):
    """3D -Lap u + u^3 + u = f on [-1, 1]^3 with zero normal derivative,
    u = cos(pi x) + cos(pi y) + cos(pi z): -Lap u = pi^2 u.  All n^3 nodes.
    Returns (u_exact, f), shape (nz, ny, nx)."""
    c = np.cos(math.pi * node_coords(n))
    u = c[:, None, None] + c[None, :, None] + c[None, None, :]
    return u, math.pi ** 2 * u + u ** 3 + u


def neumann_potential_3d(n, a=10.0, b=10.0):
    """3D -Lap u + a u + b u^3 + V u = f on [-1, 1]^3 with zero normal
    derivative (Section 6.3, Example 1, eq. ex3d1): u = cos(pi x) + cos(pi y) +
    cos(pi z), -Lap u = pi^2 u, V = 100 (sin^2(pi x/4) + sin^2(pi y/4) +
    sin^2(pi z/4)) + x^2 + y^2 + z^2.  All n^3 nodes.  Returns (u_exact, f, V),
    shape (nz, ny, nx)."""
    x = node_coords(n)
    c = np.cos(math.pi * x)
    w = 100.0 * np.sin(math.pi * x / 4.0) ** 2 + x * x
    u = c[:, None, None] + c[None, :, None] + c[None, None, :]
    v = w[:, None, None] + w[None, :, None] + w[None, None, :]
    f = math.pi ** 2 * u + a * u + b * u ** 3 + v * u
    return u, f, v


def polynomial_coefficients(dim, seed, degree=4):
    """Coefficients a ~ U(-1, 1) of the perturbation polynomial, from
    default_rng(seed), shape (degree + 1,) * dim, indexed (x, y[, z]) exponents."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(degree + 1,) * dim)


def polynomial_perturbation(n, dim, seed, degree=4, coords=None):
    """Section 6.2 / 6.3 initial-guess perturbation p on the n^dim nodes with
    per-axis coordinates `coords` (default: all n nodes of [-1, 1]): sum of
    a_{i..} x^i y^j (z^k) over exponents 0..degree with coefficients
    a ~ U(-1, 1) from default_rng(seed), divided by its largest magnitude over
    the nodes (so max |p| = 1 on the grid).  Shape (ny, nx) or (nz, ny, nx);
    the coefficient array is indexed (x, y[, z]) exponents."""
    coef = polynomial_coefficients(dim, seed, degree)
    x = node_coords(n) if coords is None else np.asarray(coords, dtype=np.float64)
    powers = np.stack([x ** e for e in range(degree + 1)])  # (degree+1, n)
    if dim == 2:
        p = np.einsum("ij,iX,jY->YX", coef, powers, powers, optimize=True)
    else:  # one axis at a time: (k, Y, X) first, then the z-planes (no n^3 temporaries)
        kyx = np.einsum("ijk,iX,jY->kYX", coef, powers, powers, optimize=True)
        p = np.einsum("kZ,kYX->ZYX", powers, kyx, optimize=True)
    p /= max(float(p.max()), -float(p.min()))
    return p


def interior_coords(n, a, b):
    """Interior nodes x_i = a + i (b - a)/(n + 1), i = 1..n (Dirichlet grid on (a, b))."""
    return a + (b - a) * np.arange(1, n + 1, dtype=np.float64) / (n + 1)


def schrodinger_3d(n, half=8.0):
    """Section 6.3, Example 2 (eq. ex3d2) on the n^3 interior nodes of
    (-half, half)^3 with Dirichlet data: the potential V = 100 (sin^2(pi x/4) +
    sin^2(pi y/4) + sin^2(pi z/4)) + x^2 + y^2 + z^2 and a start
    exp(-|x|^2 / 2) (not normalised).  Returns (V, u_start), shape (nz, ny, nx)."""
    x = interior_coords(n, -half, half)
    w = 100.0 * np.sin(math.pi * x / 4.0) ** 2 + x * x
    g = np.exp(-0.5 * x * x)
    v = w[:, None, None] + w[None, :, None] + w[None, None, :]
    u = g[:, None, None] * g[None, :, None] * g[None, None, :]
    return v, u


def grayscott_spot(n, radius=0.2, amp=0.25, center=(0.5, 0.5)):
    """Start for the steady Gray-Scott system on the n x n nodes of [0, 1]^2
    (both ends included): (A, S) = (amp, 0.5) inside a disc of the given
    radius, the trivial state (0, 1) outside.  Shape (2, n, n)."""
    x = np.linspace(0.0, 1.0, n)
    X, Y = np.meshgrid(x, x)
    m = ((X - center[0]) ** 2 + (Y - center[1]) ** 2 < radius ** 2).astype(np.float64)
    return np.stack([amp * m, 1.0 - 0.5 * m])


def grayscott_source(n, rho=0.04):
    """The constant source F = (0, rho) of the steady Gray-Scott system."""
    f = np.zeros((2, n, n))
    f[1] = rho
    return f
