"""CPU FP64 oracle for the quasi-Newton / tensor-product solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy implementation of what the GPU library computes.  Only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import it; the product
path (``paper_2502_03611_amd``) never does, and the two share no code.  Inputs
come from ``synth`` (seeded generators with no solver arithmetic).

Contents, each following the cited passage of Hao, Lee & Zhang,
"An Efficient Quasi-Newton Method with Tensor Product Implementation ..."
(arXiv 2502.03611):

* ``spectral``  - 1D finite-difference stiffness matrix (Section 3.2, eq. Sy),
  its closed-form sine eigenpairs, the mass-weighted symmetric diagonalisation
  route of Section 4.2, and a textbook Jacobi eigensolver used only as a pin.
* ``operators`` - the discrete residual F^h(U) = A_h vec(U) + N_h(U)
  (Section 4, eq. F_u) for the semilinear cubic problem, the 2-component
  system (Section 4.3, eq. system) and the conservative quasi-linear flux
  form; the assembled Kronecker-sum A_h (eqs. A_definition_2D/3D).
* ``tensor``    - mode-n products, the tensor-product inverse of
  (c A_h + beta I) (Section 4.1, eq. fin_inverse) and direct solves.
* ``qn``        - the quasi-Newton iteration (Section 4, eq. identity-method)
  with the midpoint shift rule, the 2x2-block eigenvalue rule for systems
  (Section 4.3, eq. eigenvalues), and a dense Newton solver (eq. newton) used
  only to pin fixed points at tiny sizes.
* ``net``       - direct-loop FP64 convolution network pieces (forward,
  gradients, Adam) for the learned initial guess.
* ``splitbf16`` - the split-bf16 products of the reduced-precision transforms.
* ``neumann``   - the homogeneous-Neumann (ghost-point) variant of Section 3.2:
  stiffness matrix, cosine eigenpairs, mirrored stencil, solve and iteration.

Pins: every function here is checked in ``tests/test_oracle_*.py`` against
closed forms, invariants, brute force or library routines (see each test).
"""
