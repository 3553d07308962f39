"""ctypes binding of the batched solver (include/qn_batched.h).  Argument
marshalling only; the iteration runs in libqn's kernels from a replayed
hipGraph."""

import ctypes

import numpy as np
import torch

from ._binding import BETA_MODES, BOUNDARIES, PRECISIONS, c_vp, check, lib, last_error

_B = None


class QNBOptions(ctypes.Structure):
    _fields_ = [("boundary", ctypes.c_int32), ("length", ctypes.c_double), ("lin", ctypes.c_double),
                ("system", ctypes.c_int32), ("step", ctypes.c_double), ("gs_da", ctypes.c_double),
                ("gs_ds", ctypes.c_double), ("gs_rho", ctypes.c_double), ("gs_mu", ctypes.c_double)]


class QNBResult(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("relres", ctypes.c_double),
                ("relres0", ctypes.c_double)]


def _qnb():
    global _B
    if _B is not None:
        return _B
    L = lib()
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    L.qnb_setup.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32, ctypes.c_int32,
                            ctypes.c_double, ctypes.POINTER(c_vp)]
    L.qnb_setup_ex.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_double, ctypes.POINTER(QNBOptions), ctypes.POINTER(c_vp)]
    L.qnb_field_elems.argtypes = [c_vp, i64p]
    L.qnb_instance_layout.argtypes = [c_vp, ctypes.c_int32, i64p, i64p]
    L.qnb_workspace_bytes.argtypes = [c_vp, ctypes.POINTER(ctypes.c_size_t)]
    L.qnb_bind_workspace.argtypes = [c_vp, c_vp, ctypes.c_size_t]
    L.qnb_set_stream.argtypes = [c_vp, c_vp]
    L.qnb_autotune.argtypes = [c_vp]
    L.qnb_class_count.argtypes = [c_vp, i32p]
    L.qnb_class_info.argtypes = [c_vp, ctypes.c_int32, i32p]
    L.qnb_iterate.argtypes = [c_vp, c_vp, c_vp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                              ctypes.POINTER(QNBResult)]
    L.qnb_fdm_solve.argtypes = [c_vp, c_vp, ctypes.c_double, ctypes.c_double, c_vp]
    L.qnb_destroy.argtypes = [c_vp]
    L.qnb_destroy.restype = None
    for n in ("qnb_setup", "qnb_setup_ex", "qnb_field_elems", "qnb_instance_layout", "qnb_workspace_bytes",
              "qnb_bind_workspace", "qnb_set_stream", "qnb_autotune", "qnb_class_count",
              "qnb_class_info", "qnb_iterate", "qnb_fdm_solve"):
        getattr(L, n).restype = ctypes.c_int32
    _B = L
    return L


class BatchedSolver:
    """Independent 2D instances: sizes[i] points per side (interior points
    with Dirichlet data, all nodes with Neumann data), ncomp[i] in {1 (cubic),
    2 (system)}; one U pool and one F pool of FP64 on the GPU.  boundary,
    length (the side of the square; default 1 for Dirichlet, 2 for Neumann
    data, as for the single-problem solver) and lin apply to every instance
    (qnb_options).  system: the 2-component problem, "cubic" (Section 4.3)
    or "grayscott" (Section 6.2; gs = (D_A, D_S, rho, mu), None = the
    paper's); step: the step size of every update."""

    def __init__(self, sizes, ncomp, precision="fp32", beta_mode="midpoint", beta=0.0,
                 device="cuda", boundary="dirichlet", length=None, lin=0.0, system="cubic",
                 step=1.0, gs=None):
        L = _qnb()
        self.count = len(sizes)
        self.sizes = [int(s) for s in sizes]
        self.ncomp = [int(c) for c in ncomp]
        self.device = torch.device(device)
        n_arr = (ctypes.c_int32 * self.count)(*self.sizes)
        c_arr = (ctypes.c_int32 * self.count)(*self.ncomp)
        ctx = c_vp()
        if length is None:
            length = 2.0 if boundary == "neumann" else 1.0
        opt = QNBOptions(BOUNDARIES[boundary], float(length), float(lin),
                         {"cubic": 0, "grayscott": 1}[system], float(step),
                         *(float(v) for v in (gs if gs is not None else (0.0, 0.0, 0.0, 0.0))))
        check(L.qnb_setup_ex(self.count, n_arr, c_arr, PRECISIONS[precision],
                             BETA_MODES[beta_mode], float(beta), ctypes.byref(opt),
                             ctypes.byref(ctx)))
        self._ctx = ctx
        fe = ctypes.c_int64()
        check(L.qnb_field_elems(ctx, ctypes.byref(fe)))
        self.field_elems = fe.value
        self.layout = []
        for i in range(self.count):
            off, cs = ctypes.c_int64(), ctypes.c_int64()
            check(L.qnb_instance_layout(ctx, i, ctypes.byref(off), ctypes.byref(cs)))
            self.layout.append((off.value, cs.value))
        nb = ctypes.c_size_t()
        check(L.qnb_workspace_bytes(ctx, ctypes.byref(nb)))
        self._ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        self._stream()
        check(L.qnb_bind_workspace(ctx, ctypes.c_void_p(self._ws.data_ptr()), nb.value))

    def _stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        check(_qnb().qnb_set_stream(self._ctx, ctypes.c_void_p(s)))

    def pool(self):
        return torch.zeros(self.field_elems, dtype=torch.float64, device=self.device)

    def view(self, pool, i):
        """Component views (ncomp, n, n) of instance i inside a pool."""
        off, cs = self.layout[i]
        n, c = self.sizes[i], self.ncomp[i]
        return torch.as_strided(pool, (c, n, n), (cs, n, 1), off)

    def fill(self, pool, i, arr):
        self.view(pool, i).copy_(torch.from_numpy(np.asarray(arr, dtype=np.float64)))

    def autotune(self):
        self._stream()
        check(_qnb().qnb_autotune(self._ctx))

    def classes(self):
        L = _qnb()
        k = ctypes.c_int32()
        check(L.qnb_class_count(self._ctx, ctypes.byref(k)))
        out = []
        for i in range(k.value):
            info = (ctypes.c_int32 * 8)()
            check(L.qnb_class_info(self._ctx, i, info))
            n, c, K, tmL, tnL, tmR, tnR, p = list(info)
            out.append({"n": n, "ncomp": c, "count": K, "tile_y": (tmL, tnL), "tile_x": (tmR, tnR),
                        "padded": p})
        return out

    def iterate(self, U, F, rtol=1e-10, max_iter=200, graph_iters=4):
        for t, nm in ((U, "U"), (F, "F")):
            if t.dtype != torch.float64 or not t.is_cuda or t.numel() != self.field_elems:
                raise ValueError(f"{nm} must be a float64 CUDA pool of {self.field_elems} elements")
        res = (QNBResult * self.count)()
        self._stream()
        status = _qnb().qnb_iterate(self._ctx, ctypes.c_void_p(U.data_ptr()),
                                    ctypes.c_void_p(F.data_ptr()), float(rtol), int(max_iter),
                                    int(graph_iters), res)
        if status not in (0, 3, 4):
            check(status)
        return status, [{"iters": r.iters, "status": r.status, "relres": r.relres,
                         "relres0": r.relres0} for r in res]

    def fdm_solve(self, R, scale=1.0, shift=0.0, X=None):
        """X_i = (scale A_h + shift I)^-1 R_i for every instance (pool layout)."""
        if R.dtype != torch.float64 or not R.is_cuda or R.numel() != self.field_elems:
            raise ValueError(f"R must be a float64 CUDA pool of {self.field_elems} elements")
        X = self.pool() if X is None else X
        self._stream()
        check(_qnb().qnb_fdm_solve(self._ctx, ctypes.c_void_p(R.data_ptr()), float(scale),
                                   float(shift), ctypes.c_void_p(X.data_ptr())))
        return X

    def close(self):
        if getattr(self, "_ctx", None):
            _qnb().qnb_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["BatchedSolver", "last_error"]
