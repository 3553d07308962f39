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


def opts(**kw):
    o = QNOptions()
    for k, v in kw.items():
        setattr(o, k, v)
    return o


@pytest.mark.parametrize("kw,nl,ncomp,n,beta,want", [
    (dict(boundary=1), 0, 1, (9, 9, 9), 1.0, "ok"),
    (dict(boundary=1, lin=1.0), 0, 1, (9, 9, 1), 0.0, "ok"),  # 2D, beta 0 + lin: see below
    (dict(boundary=2), 0, 1, (9, 9, 9), 1.0, "invalid"),
    (dict(boundary=1), 0, 1, (1, 9, 9), 1.0, "invalid"),       # n < 2
    (dict(boundary=1), 0, 1, (9, 9, 9), 0.0, "invalid"),       # lam_min = 0: beta must be > 0
    (dict(boundary=1), 2, 2, (9, 9, 9), 1.0, "unsupported"),   # system
    (dict(boundary=1), 1, 1, (9, 9, 9), 1.0, "unsupported"),   # quasi-linear
    (dict(boundary=1, precision=2), 0, 1, (9, 9, 9), 1.0, "unsupported"),  # bf16x3
    (dict(length=-1.0), 0, 1, (9, 9, 9), 0.0, "invalid"),
    (dict(length=float("inf")), 0, 1, (9, 9, 9), 0.0, "invalid"),
    (dict(lin=float("nan")), 0, 1, (9, 9, 9), 0.0, "invalid"),
    (dict(lin=1.0), 2, 2, (9, 9, 9), 0.0, "invalid"),          # lin only for the cubic problem
    (dict(length=2.0, lin=0.5), 0, 1, (9, 9, 9), 0.0, "ok"),
    # cubic coefficient and potential (never dereferenced by setup)
    (dict(cub=float("nan")), 0, 1, (9, 9, 9), 0.0, "invalid"),
    (dict(cub=-0.5), 0, 1, (9, 9, 9), 0.0, "ok"),
    (dict(cub=2.0), 2, 2, (9, 9, 9), 0.0, "invalid"),          # cub != 1 only for cubic
    (dict(cub=1.0), 2, 2, (9, 9, 9), 0.0, "ok"),
    (dict(potential=4096), 1, 1, (9, 9, 9), 0.0, "invalid"),   # potential only for cubic
    (dict(potential=4096), 2, 2, (9, 9, 9), 0.0, "invalid"),
    (dict(boundary=1, lin=10.0, cub=10.0, potential=4096), 0, 1, (9, 9, 9), 1.0, "ok"),
    (dict(quad=-1.0, cub=1e-300), 0, 1, (9, 9, 9), 0.0, "ok"),       # eq. 2dex: no cubic term
    (dict(quad=float("inf")), 0, 1, (9, 9, 9), 0.0, "invalid"),
    (dict(quad=1.0), 2, 2, (9, 9, 9), 0.0, "invalid"),               # quad only for cubic
    # spectral elements (host-side setup: Gauss-Lobatto nodes, Jacobi eigen-data)
    (dict(discretization=1, sem_order=2), 0, 1, (11, 11, 11), 0.0, "ok"),
    (dict(discretization=1, sem_order=3, boundary=1), 0, 1, (10, 13, 7), 1.0, "ok"),
    (dict(discretization=1, sem_order=2), 0, 1, (10, 11, 11), 0.0, "invalid"),  # 10 + 1 odd
    (dict(discretization=1, sem_order=9), 0, 1, (17, 17, 17), 0.0, "invalid"),
    (dict(discretization=1, sem_order=2), 0, 1, (1027, 11, 11), 0.0, "invalid"),  # > 1025
    (dict(discretization=2), 0, 1, (9, 9, 9), 0.0, "invalid"),
    (dict(discretization=1, sem_order=2), 1, 1, (11, 11, 11), 0.0, "unsupported"),
    (dict(discretization=1, sem_order=2, precision=2), 0, 1, (11, 11, 11), 0.0, "unsupported"),
    # the Gray-Scott system (nl 3): 2D, two components, Neumann data, FP64/FP32
    (dict(boundary=1, step=0.1), 3, 2, (9, 9, 1), 0.0, "ok"),
    (dict(boundary=1, gs_da=1e-3, gs_ds=2e-3, gs_rho=0.05, gs_mu=0.01), 3, 2, (9, 9, 1), 0.0, "ok"),
    (dict(boundary=1, precision=1), 3, 2, (9, 9, 1), 0.0, "ok"),
    (dict(boundary=1), 3, 1, (9, 9, 1), 0.0, "invalid"),         # one component
    (dict(boundary=1), 3, 2, (9, 9, 9), 0.0, "unsupported"),     # 3D
    (dict(), 3, 2, (9, 9, 1), 0.0, "unsupported"),                # Dirichlet data
    (dict(boundary=1, precision=2), 3, 2, (9, 9, 1), 0.0, "unsupported"),
    (dict(boundary=1, gs_da=-1.0), 3, 2, (9, 9, 1), 0.0, "invalid"),
    (dict(boundary=1, gs_rho=float("nan")), 3, 2, (9, 9, 1), 0.0, "invalid"),
    (dict(gs_da=1.0), 0, 1, (9, 9, 9), 0.0, "invalid"),          # parameters for another problem
    (dict(step=-0.1), 0, 1, (9, 9, 9), 0.0, "invalid"),
    (dict(step=float("inf")), 0, 1, (9, 9, 9), 0.0, "invalid"),
    (dict(step=0.5), 0, 1, (9, 9, 9), 0.0, "ok"),
])
def test_setup_boundary_length_and_pointwise_terms(kw, nl, ncomp, n, beta, want):
    dim = 2 if n[2] == 1 else 3
    if dim == 2 and want == "ok" and kw.get("boundary") == 1:
        beta = 0.5  # a fixed shift must still be positive with Neumann data (lam_min = 0)
    st, ctx = setup(dim=dim, n=n, ncomp=ncomp, nl=nl, beta=beta, opt=opts(**kw))
    expect = {"ok": qn.QN_OK, "invalid": qn.QN_ERR_INVALID, "unsupported": qn.QN_ERR_UNSUPPORTED}
    assert st == expect[want], (st, qn.last_error())
    if st == qn.QN_OK:
        qn.lib().qn_destroy(ctx)


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


def test_noalloc_residual_host_checks():
    """qn_residual_noalloc needs no workspace and refuses on the host, before
    it reads a pointer: spectral elements (their operator bands live in the
    workspace) and, as a guard, a launch beyond the fixed array.  Every grid
    the library accepts fits that array: the 3D residual launches at most
    16384 workgroups of 1024 threads (here: 8 x 2048 tiles of 512 x 2
    columns, one slab) or 32768 of 512 threads (two components or Neumann
    data: 16 x 2048 tiles of 256 x 2), the 2D one 4096 at most, so null
    pointers meet the null check."""
    from paper_2502_03611_amd import Solver
    L = qn.lib()
    null = ctypes.c_void_p(None)
    for shape, kind in (((64, 4096, 3585), "cubic"), ((64, 4096, 3841), "system"),
                        ((4096, 4096), "cubic")):
        s = Solver(shape, kind, beta=1.0, workspace=False)
        assert L.qn_residual_noalloc(s._ctx, null, null, null, null) == qn.QN_ERR_INVALID
        assert "null" in qn.last_error()
        s.close()
    sem = Solver((15, 15), "cubic", beta=1.0, discretization="sem", sem_order=2, workspace=False)
    assert L.qn_residual_noalloc(sem._ctx, null, null, null, null) == qn.QN_ERR_UNSUPPORTED
    assert "spectral" in qn.last_error()
    sem.close()


def test_null_context_and_timing_table():
    L = qn.lib()
    assert L.qn_iterate(None, None, None, 0.0, 0, None) == qn.QN_ERR_INVALID
    assert L.qn_timing_count() >= 6
    L.qn_destroy(None)


def test_autotune_and_tile_info_need_a_workspace():
    L = qn.lib()
    L.qn_autotune.argtypes = [ctypes.c_void_p]
    L.qn_tile_info.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.qn_set_tile.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    info = (ctypes.c_int32 * 4)()
    assert L.qn_autotune(None) == qn.QN_ERR_INVALID
    st, ctx = setup(n=(33, 17, 9))
    assert st == qn.QN_OK
    assert L.qn_autotune(ctx) == qn.QN_ERR_WORKSPACE
    assert L.qn_tile_info(ctx, 0, info) == qn.QN_ERR_WORKSPACE
    assert L.qn_set_tile(ctx, 0, info) == qn.QN_ERR_WORKSPACE
    assert L.qn_set_tile(None, 0, info) == qn.QN_ERR_INVALID
    L.qn_destroy(ctx)


def _qnn():
    L = qn.lib()
    L.qnn_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                             ctypes.POINTER(ctypes.c_void_p)]
    L.qnn_workspace_bytes.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]
    L.qnn_bind_workspace.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
    L.qnn_forward.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int32, ctypes.c_void_p]
    L.qnn_adam_step.argtypes = [ctypes.c_void_p] + [ctypes.c_double] * 4
    L.qnn_guess_fallback.argtypes = [ctypes.c_void_p] * 4
    L.qnn_destroy.argtypes = [ctypes.c_void_p]
    L.qnn_destroy.restype = None
    return L


@pytest.mark.parametrize("H,W,B", [(0, 5, 1), (5, 4097, 1), (5, 5, 0), (5, 5, 1025)])
def test_qnn_create_rejects_invalid(H, W, B):
    L = _qnn()
    net = ctypes.c_void_p()
    assert L.qnn_create(H, W, B, ctypes.byref(net)) == qn.QN_ERR_INVALID
    assert qn.last_error()


def test_qnn_host_checks():
    L = _qnn()
    assert L.qnn_param_count() == 28641  # 2*32*9+32 + 3*(32*32*9+32) + 32*9+1
    net = ctypes.c_void_p()
    assert L.qnn_create(255, 255, 4, ctypes.byref(net)) == qn.QN_OK
    nb = ctypes.c_size_t()
    assert L.qnn_workspace_bytes(net, ctypes.byref(nb)) == qn.QN_OK
    assert nb.value > 4 * 255 * 255 * 32 * 4  # at least one FP32 activation tensor
    assert L.qnn_forward(net, None, None, 1, None) == qn.QN_ERR_WORKSPACE
    assert L.qnn_bind_workspace(net, ctypes.c_void_p(256 + 8), nb.value) == qn.QN_ERR_WORKSPACE
    assert L.qnn_bind_workspace(net, ctypes.c_void_p(4096), nb.value - 1) == qn.QN_ERR_WORKSPACE
    assert L.qnn_forward(None, None, None, 1, None) == qn.QN_ERR_INVALID
    assert L.qnn_guess_fallback(None, None, None, None) == qn.QN_ERR_INVALID
    assert L.qnn_guess_fallback(net, None, None, None) == qn.QN_ERR_INVALID
    L.qnn_destroy(net)
    L.qnn_destroy(None)


def _qnb():
    L = qn.lib()
    L.qnb_setup.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                            ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_void_p)]
    L.qnb_field_elems.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
    L.qnb_instance_layout.argtypes = [ctypes.c_void_p, ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    L.qnb_iterate.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_double, ctypes.c_int32,
                                                      ctypes.c_int32, ctypes.c_void_p]
    L.qnb_destroy.argtypes = [ctypes.c_void_p]
    L.qnb_destroy.restype = None
    return L


def _qnb_setup(n, nc, prec=1, bmode=1, beta=0.0):
    L = _qnb()
    a = (ctypes.c_int32 * len(n))(*n)
    b = (ctypes.c_int32 * len(nc))(*nc)
    ctx = ctypes.c_void_p()
    return L.qnb_setup(len(n), a, b, prec, bmode, beta, ctypes.byref(ctx)), ctx


@pytest.mark.parametrize("n,nc,prec,bmode,beta", [
    ([0], [1], 1, 1, 0.0), ([5000], [1], 1, 1, 0.0), ([9], [3], 1, 1, 0.0),
    ([9], [1], 7, 1, 0.0), ([9], [1], 1, 5, 0.0), ([9], [1], 1, 0, float("inf")),
])
def test_qnb_setup_rejects_invalid(n, nc, prec, bmode, beta):
    st, _ = _qnb_setup(n, nc, prec, bmode, beta)
    assert st == qn.QN_ERR_INVALID
    assert qn.last_error()


from paper_2502_03611_amd.batched import QNBOptions as _QNBOptions  # noqa: E402


def _qnb_setup_ex(n, nc, opt, prec=1, bmode=1, beta=0.0):
    L = qn.lib()
    L.qnb_setup_ex.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_double, ctypes.c_void_p,
                               ctypes.POINTER(ctypes.c_void_p)]
    L.qnb_destroy.argtypes = [ctypes.c_void_p]
    L.qnb_destroy.restype = None
    a = (ctypes.c_int32 * len(n))(*n)
    b = (ctypes.c_int32 * len(nc))(*nc)
    ctx = ctypes.c_void_p()
    o = ctypes.byref(_QNBOptions(*opt)) if opt is not None else None
    st = L.qnb_setup_ex(len(n), a, b, prec, bmode, beta, o, ctypes.byref(ctx))
    if st == qn.QN_OK:
        L.qnb_destroy(ctx)
    return st


@pytest.mark.parametrize("n,nc,opt,prec,bmode,beta", [
    ([9], [1], (2, 1.0, 0.0), 1, 1, 0.0),                      # unknown boundary
    ([9], [1], (0, -1.0, 0.0), 1, 1, 0.0),                     # negative length
    ([9], [1], (0, float("nan"), 0.0), 1, 1, 0.0),
    ([9], [1], (0, 1.0, float("inf")), 1, 1, 0.0),             # lin not finite
    ([9], [2], (0, 1.0, 1.0), 1, 1, 0.0),                      # lin on the system
    ([9], [2], (1, 1.0, 1.0), 1, 1, 0.0),                      # Neumann system
    ([1], [1], (1, 1.0, 1.0), 1, 1, 0.0),                      # Neumann n = 1
    ([9], [1], (1, 1.0, 1.0), 2, 1, 0.0),                      # Neumann with bf16x3
    ([9], [1], (1, 1.0, 1.0), 1, 0, 0.0),                      # Neumann fixed beta = 0
    ([9], [1], (1, 1.0, 0.0), 1, 1, 0.0),                      # Neumann midpoint, lin = 0
    ([9, 12], [1, 1], (0, 1.0, 0.0), 1, 0, -2.0 * 9.8),        # fixed beta below -lam_min
    ([9], [1], (1, 1.0, 0.0), 1, 2, 0.0),                      # Neumann max rule, lin = 0
    ([9], [2], (0, 10.0, 0.0), 1, 4, 0.0),                     # min rule, system, lam_min < 1
    ([9], [1], (0, 1.0, -25.0), 1, 1, 0.0),                    # lin below -lam_min = -19.6
    ([9], [1], (0, 1.0, -12.0), 1, 3, 0.0),                    # min + max: 2 lin below it
    ([9], [1], None, 1, 5, 0.0),                               # unknown rule
    ([9], [2], (1, 1.0, 0.0, 2), 1, 1, 0.0),                   # unknown system
    ([9], [2], (1, 1.0, 0.0, 1, -0.1), 1, 1, 0.0),             # negative step
    ([9], [2], (1, 1.0, 0.0, 1, 0.1, -1.0), 1, 1, 0.0),        # negative D_A
    ([9], [2], (1, 1.0, 0.0, 0, 0.0, 1e-3), 1, 1, 0.0),        # parameters for the cubic system
])
def test_qnb_setup_ex_rejects_invalid(n, nc, opt, prec, bmode, beta):
    assert _qnb_setup_ex(n, nc, opt, prec, bmode, beta) == qn.QN_ERR_INVALID
    assert qn.last_error()


@pytest.mark.parametrize("n,nc,opt,prec", [
    ([9], [2], (0, 1.0, 0.0, 1, 0.1), 1),                      # Gray-Scott with Dirichlet data
    ([9], [2], (1, 1.0, 0.0, 1, 0.1), 2),                      # with bf16x3
    ([9, 9], [2, 1], (1, 1.0, 0.0, 1, 0.1), 1),                # with a scalar instance
])
def test_qnb_setup_ex_grayscott_unsupported(n, nc, opt, prec):
    assert _qnb_setup_ex(n, nc, opt, prec, 1, 0.0) == qn.QN_ERR_UNSUPPORTED


@pytest.mark.parametrize("n,nc,opt,prec,bmode,beta", [
    ([9, 12, 9], [1, 1, 1], (1, 2.0, 1.0), 1, 1, 0.0),
    ([9, 12], [1, 1], (1, 2.0, 0.0), 0, 0, 3.0),
    ([9, 12], [1, 2], (0, 2.0, 0.0), 2, 1, 0.0),
    ([9], [1], None, 1, 1, 0.0),
    ([9, 12], [1, 2], None, 0, 2, 0.0),                        # max
    ([9, 12], [1, 2], None, 1, 3, 0.0),                        # min + max
    ([9, 12], [1, 2], None, 1, 4, 0.0),                        # min (lam_min > 1 here)
    ([9], [1], (0, 1.0, -12.0), 1, 1, 0.0),                    # midpoint: lin > -lam_min
    ([9, 12], [1, 1], (1, 2.0, 1.0), 1, 4, 0.0),               # Neumann min rule, lin > 0
    ([9, 12, 9], [2, 2, 2], (1, 1.0, 0.0, 1, 0.1), 1, 1, 0.0), # Gray-Scott, midpoint
    ([9], [2], (1, 1.0, 0.0, 1, 0.1, 1e-3, 2e-3, 0.05, 0.01), 0, 4, 0.0),  # own parameters, min
])
def test_qnb_setup_ex_accepts(n, nc, opt, prec, bmode, beta):
    assert _qnb_setup_ex(n, nc, opt, prec, bmode, beta) == qn.QN_OK


def test_qnb_layout_covers_pool_exactly():
    L = _qnb()
    n = [15, 31, 15, 8, 31, 15]
    nc = [1, 2, 1, 2, 2, 1]
    st, ctx = _qnb_setup(n, nc)
    assert st == qn.QN_OK
    total = ctypes.c_int64()
    assert L.qnb_field_elems(ctx, ctypes.byref(total)) == qn.QN_OK
    assert total.value == sum(c * k * k for k, c in zip(n, nc))
    covered = []
    for i, (k, c) in enumerate(zip(n, nc)):
        off, cs = ctypes.c_int64(), ctypes.c_int64()
        assert L.qnb_instance_layout(ctx, i, ctypes.byref(off), ctypes.byref(cs)) == qn.QN_OK
        for comp in range(c):
            covered.append((off.value + comp * cs.value, k * k))
    covered.sort()
    pos = 0
    for start, size in covered:  # disjoint, gap-free tiling of the pool
        assert start == pos
        pos += size
    assert pos == total.value
    assert L.qnb_instance_layout(ctx, len(n), ctypes.byref(off), ctypes.byref(cs)) == qn.QN_ERR_INVALID
    assert L.qnb_iterate(ctx, None, None, 1e-10, 10, 4, None) == qn.QN_ERR_WORKSPACE
    L.qnb_destroy(ctx)


@pytest.mark.parametrize("kw,n,bc", [(dict(), (9, 12, 7), "dirichlet"),
                                     (dict(boundary=1, length=2.0), (9, 12, 7), "neumann"),
                                     (dict(discretization=1, sem_order=3), (11, 8, 5), "dirichlet"),
                                     (dict(discretization=1, sem_order=2, boundary=1,
                                           length=3.0), (9, 13, 5), "neumann")])
def test_node_coordinates(kw, n, bc):
    """qn_nodes (host only) against the definitions: finite-difference nodes
    (i + 1) h or i h, and the spectral element Gauss-Lobatto nodes of the
    oracle."""
    import numpy as np
    from oracle import sem
    st, ctx = setup(dim=3, n=n, nl=0, beta=1.0, opt=opts(**kw))
    assert st == qn.QN_OK, qn.last_error()
    L = kw.get("length", 1.0)
    for a in range(3):
        x = (ctypes.c_double * n[a])()
        assert qn.lib().qn_nodes(ctx, a, x) == qn.QN_OK
        x = np.array(x)
        if kw.get("discretization") == 1:
            k = kw["sem_order"]
            e = (n[a] - 1) // k if bc == "neumann" else (n[a] + 1) // k
            ref = sem.nodes_and_matrices(e, k, L, bc)[0]
        elif bc == "neumann":
            ref = np.arange(n[a]) * L / (n[a] - 1)
        else:
            ref = np.arange(1, n[a] + 1) * L / (n[a] + 1)
        np.testing.assert_allclose(x, ref, rtol=0, atol=1e-14)
    x = (ctypes.c_double * 4)()
    assert qn.lib().qn_nodes(ctx, 3, x) == qn.QN_ERR_INVALID
    qn.lib().qn_destroy(ctx)


@pytest.mark.parametrize("mode,nl,want", [(2, 0, "ok"), (3, 0, "ok"), (4, 2, "ok"),
                                          (5, 0, "invalid"), (2, 1, "invalid"),
                                          (3, 1, "invalid")])
def test_shift_rule_modes(mode, nl, want):
    """QN_BETA_MAX / SUM / MIN: accepted for the cubic problem and the system,
    refused for the quasi-linear problem (coefficient rule); 5 is unknown."""
    st, ctx = setup(nl=nl, ncomp=2 if nl == 2 else 1, beta=0.0, opt=opts(beta_mode=mode))
    assert st == (qn.QN_OK if want == "ok" else qn.QN_ERR_INVALID), qn.last_error()
    if st == qn.QN_OK:
        qn.lib().qn_destroy(ctx)
