"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *generates inputs*: grid coordinates, manufactured exact
solutions and their continuous right-hand sides, seeded random tensors and
Gaussian random fields.  It holds none of the discrete method's arithmetic
(no stencil, no eigen-transform, no quasi-Newton step), so both the CPU oracle
and the GPU path can consume its arrays without sharing any solver code.

Array convention everywhere: C-order ``(nz, ny, nx)`` in 3D and ``(ny, nx)`` in
2D, x fastest, which is the paper's ``vec`` order (first index fastest,
Section 3.1, eq. vec-property).  ``n`` interior points per axis on (0, 1) with
spacing ``h = 1/(n+1)`` (Section 3.2, with the boundary nodes removed for
Dirichlet data); the Neumann workloads use all ``n`` nodes of ``[-1, 1]``,
``h = 2/(n-1)``.
"""

from .fields import (  # noqa: F401
    grid_coords,
    manufactured_c1,
    manufactured_c2,
    manufactured_c3,
    amplitude_c3,
    random_field,
    gaussian_random_field,
    batched_instance,
    learned_guess_rhs,
    node_coords,
    neumann_2d,
    neumann_3d,
    neumann_potential_3d,
    polynomial_coefficients,
    polynomial_perturbation,
    interior_coords,
    schrodinger_3d,
    grayscott_spot,
    grayscott_source,
    BATCH_SIZES,
)
