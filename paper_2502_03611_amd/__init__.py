"""MI355X (gfx950) implementation of the quasi-Newton method with a
tensor-product (fast-diagonalisation) solve of Hao, Lee & Zhang (arXiv
2502.03611).  The solver is the C-ABI library libqn.so (include/qn.h) built
from ``csrc/``; this package is its thin Python binding."""

from ._binding import (  # noqa: F401
    BETA_MODES,
    LIB_PATH,
    NONLINEARITIES,
    PRECISIONS,
    QN_ERR_DIVERGED,
    QN_ERR_HIP,
    QN_ERR_INVALID,
    QN_ERR_NOT_CONVERGED,
    QN_ERR_UNSUPPORTED,
    QN_ERR_WORKSPACE,
    QN_OK,
    QNError,
    Solver,
    last_error,
    lib,
)
