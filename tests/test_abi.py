"""C-ABI checks that need no GPU: the library loads, exports every function
include/*.h declares, and host-side argument validation returns the documented
statuses without touching the device."""

import ctypes
import glob
import os
import re

import pytest

import paper_2502_03611_amd as qn
from paper_2502_03611_amd._binding import QNGrid, QNOptions, QNStats

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(q\w+)\s*\(", text):
            names.add(m.group(1))
    return sorted(n for n in names if n.startswith(("qn_", "qnn_", "qnb_")))


def test_every_declared_symbol_is_exported():
    lib = qn.lib()
    names = declared_functions()
    assert "qn_iterate" in names and "qn_fdm_solve" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def setup(dim=3, n=(9, 9, 9), ncomp=1, nl=0, beta=0.0, opt=None):
    g = QNGrid()
    g.dim = dim
    for a in range(3):
        g.n[a] = n[a]
    g.ncomp = ncomp
    ctx = ctypes.c_void_p()
    st = qn.lib().qn_setup(ctypes.byref(g), beta, nl, ctypes.byref(opt) if opt else None,
                           ctypes.byref(ctx))
    return st, ctx


@pytest.mark.parametrize("kw", [
    dict(dim=1), dict(dim=4), dict(n=(0, 9, 9)), dict(n=(9, 5000, 9)),
    dict(ncomp=2), dict(nl=2, ncomp=1), dict(nl=7), dict(beta=-1e9), dict(beta=float("nan")),
])
def test_setup_rejects_invalid(kw):
    st, ctx = setup(**kw)
    assert st == qn.QN_ERR_INVALID
    assert qn.last_error()


def test_setup_rejects_midpoint_for_quasilinear_and_bad_enums():
    o = QNOptions()
    o.beta_mode = 1
    assert setup(nl=1, opt=o)[0] == qn.QN_ERR_INVALID
    o = QNOptions()
    o.precision = 9
    assert setup(opt=o)[0] == qn.QN_ERR_INVALID


def test_workspace_size_and_unbound_errors():
    st, ctx = setup(n=(511, 511, 511), nl=1)
    assert st == qn.QN_OK
    L = qn.lib()
    nb = ctypes.c_size_t()
    assert L.qn_workspace_bytes(ctx, ctypes.byref(nb)) == qn.QN_OK
    p = 512 ** 3 * 8
    assert 2 * p <= nb.value <= 2 * p + 64 * 2 ** 20  # two padded FP64 tensors + eigen-data
    stats = QNStats()
    assert L.qn_iterate(ctx, None, None, 1e-10, 10, ctypes.byref(stats)) == qn.QN_ERR_WORKSPACE
    assert stats.status == qn.QN_ERR_WORKSPACE
    assert L.qn_residual(ctx, None, None, None, None) == qn.QN_ERR_WORKSPACE
    assert L.qn_bind_workspace(ctx, None, nb.value) == qn.QN_ERR_WORKSPACE
    assert L.qn_bind_workspace(ctx, ctypes.c_void_p(256 * 3 + 8), nb.value) == qn.QN_ERR_WORKSPACE
    assert L.qn_bind_workspace(ctx, ctypes.c_void_p(4096), nb.value - 1) == qn.QN_ERR_WORKSPACE
    L.qn_destroy(ctx)


def test_null_context_and_timing_table():
    L = qn.lib()
    assert L.qn_iterate(None, None, None, 0.0, 0, None) == qn.QN_ERR_INVALID
    assert L.qn_timing_count() >= 6
    L.qn_destroy(None)
