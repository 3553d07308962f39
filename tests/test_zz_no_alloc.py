"""The allocation-free residual (qn_residual_noalloc) against qn_residual:
the same kernels with the reduction scratch in the library's fixed device
array instead of the bound workspace, so the outputs must be bitwise equal.
Two calls in a row, the second on a smaller grid (the fixed array keeps the
first call's partials, which the second must not read), then the first
again.  (What the entry point refuses on the host, before any device work,
is tested on the CPU in test_abi.py.)"""

import ctypes

import numpy as np
import pytest
import torch

import synth
from oracle import qn as oqn
from paper_2502_03611_amd import Solver

pytestmark = pytest.mark.gpu

KIND = {"cubic": oqn.CUBIC, "system": oqn.SYSTEM, "quasilinear": oqn.QUASILINEAR}


def _case(kind, shape, seed):
    ncomp = 2 if kind == "system" else 1
    u = synth.random_field((ncomp,) + shape, seed)
    f = synth.random_field((ncomp,) + shape, seed + 1, scale=10.0)
    return u, f


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _both(kind, shape, seed, beta_mode="fixed"):
    """(R, red) from qn_residual on a workspace-bound context and from
    qn_residual_noalloc on a context without a workspace."""
    u, f = _case(kind, shape, seed)
    U, F = _dev(u), _dev(f)
    ref = Solver(shape, kind, beta=1.0 if kind != "quasilinear" else 0.0, beta_mode=beta_mode)
    red_ref = torch.full((4,), -7.0, dtype=torch.float64, device="cuda")
    r_ref = ref.residual(U, F, red=red_ref)
    s = Solver(shape, kind, beta=1.0 if kind != "quasilinear" else 0.0, beta_mode=beta_mode,
               workspace=False)
    R = torch.full_like(U, float("nan"))
    red = torch.full((4,), -7.0, dtype=torch.float64, device="cuda")
    s.residual_noalloc(U, F, R, red)
    torch.cuda.synchronize()
    return u, f, r_ref, red_ref, R, red


@pytest.mark.parametrize("first,second", [
    (("cubic", (255, 255, 255)), ("cubic", (63, 63))),
    (("system", (40, 70, 130)), ("quasilinear", (17, 9, 33))),
    (("quasilinear", (2048, 1500)), ("system", (31, 45))),
])
def test_noalloc_residual_equals_qn_residual_twice_shrinking(first, second):
    for kind, shape in (first, second, first):
        print(f"noalloc residual {kind} {shape}", flush=True)
        u, f, r_ref, red_ref, R, red = _both(kind, shape, 500 + len(shape))
        assert torch.equal(R, r_ref)
        assert torch.equal(red, red_ref)
        # and both are the oracle's residual (the bar of the residual parity tests)
        if np.prod(shape) <= 2 ** 21:
            ora = oqn.residual(KIND[kind], u, f)
            scale = float(np.linalg.norm(f)) + float(np.linalg.norm(ora - (-f)))
            assert np.linalg.norm(R.cpu().numpy() - ora) <= 1e-13 * scale
