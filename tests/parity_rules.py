"""Shared parity rules of the GPU tests (no GPU code, no arithmetic of the
method).

Iteration counts under a stopping tolerance: both sides stop at the first
relres <= rtol.  The counts must be equal; a difference of one solve is
accepted only when the residual that decided it (the oracle's relres at the
smaller of the two counts) lies within a factor 1.001 of rtol, where
rounding differences in the residual may legitimately flip the decision.
"""

import numpy as np


def deciding_relres(gpu_iters, ref):
    """The oracle's relres at the iterate where the two stopping decisions
    part (ref: the dict returned by the oracle's qn_solve)."""
    return ref["relres"][min(gpu_iters, ref["iters"], len(ref["relres"]) - 1)]


def counts_agree(gpu_iters, ref, rtol=1e-10):
    """True when gpu_iters equals the oracle's count, or differs by one with
    the deciding relres within 0.1 % of rtol."""
    k = ref["iters"]
    if gpu_iters == k:
        return True
    if abs(gpu_iters - k) != 1:
        return False
    return abs(deciding_relres(gpu_iters, ref) / rtol - 1.0) < 1e-3


def rel_l2(a, b):
    """||a - b||_2 / ||b||_2."""
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))
