"""ctypes binding of libqn (include/qn.h).  Argument marshalling only: every
step of the solver runs in the library's HIP kernels.  PyTorch provides the
device memory (caller tensors and the workspace) and the current stream."""

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqn.so")

QN_OK = 0
QN_ERR_INVALID = 1
QN_ERR_HIP = 2
QN_ERR_NOT_CONVERGED = 3
QN_ERR_DIVERGED = 4
QN_ERR_WORKSPACE = 5
QN_ERR_UNSUPPORTED = 6

NONLINEARITIES = {"cubic": 0, "quasilinear": 1, "system": 2, "grayscott": 3}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}
BETA_MODES = {"fixed": 0, "midpoint": 1, "max": 2, "sum": 3, "min": 4}

c_i32 = ctypes.c_int32
c_dbl = ctypes.c_double
c_vp = ctypes.c_void_p


class QNGrid(ctypes.Structure):
    _fields_ = [("dim", c_i32), ("n", c_i32 * 3), ("ncomp", c_i32)]


class QNOptions(ctypes.Structure):
    _fields_ = [("precision", c_i32), ("beta_mode", c_i32), ("timing", c_i32),
                ("boundary", c_i32), ("stream", c_vp), ("length", c_dbl), ("lin", c_dbl),
                ("cub", c_dbl), ("potential", c_vp), ("discretization", c_i32),
                ("sem_order", c_i32), ("quad", c_dbl), ("step", c_dbl), ("gs_da", c_dbl),
                ("gs_ds", c_dbl), ("gs_rho", c_dbl), ("gs_mu", c_dbl)]


BOUNDARIES = {"dirichlet": 0, "neumann": 1}
DISCRETIZATIONS = {"fd": 0, "sem": 1}


class QNStats(ctypes.Structure):
    _fields_ = [("iters", c_i32), ("status", c_i32), ("relres", c_dbl), ("relres0", c_dbl),
                ("beta_last", c_dbl), ("scale_last", c_dbl), ("seconds", c_dbl)]


class QNError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libqn status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libqn.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2502_03611_amd.build` "
                           "(there is no fallback implementation)")
    L = ctypes.CDLL(LIB_PATH)
    L.qn_setup.argtypes = [ctypes.POINTER(QNGrid), c_dbl, c_i32, ctypes.POINTER(QNOptions),
                           ctypes.POINTER(c_vp)]
    L.qn_workspace_bytes.argtypes = [c_vp, ctypes.POINTER(ctypes.c_size_t)]
    L.qn_bind_workspace.argtypes = [c_vp, c_vp, ctypes.c_size_t]
    L.qn_set_stream.argtypes = [c_vp, c_vp]
    L.qn_residual.argtypes = [c_vp, c_vp, c_vp, c_vp, c_vp]
    L.qn_residual_noalloc.argtypes = [c_vp, c_vp, c_vp, c_vp, c_vp]
    L.qn_fdm_solve.argtypes = [c_vp, c_vp, c_dbl, c_dbl, c_vp]
    L.qn_iterate.argtypes = [c_vp, c_vp, c_vp, c_dbl, c_i32, ctypes.POINTER(QNStats)]
    L.qn_timing_count.argtypes = []
    L.qn_timing_read.argtypes = [c_vp, c_i32, ctypes.POINTER(ctypes.c_char_p),
                                 ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(c_dbl)]
    L.qn_timing_reset.argtypes = [c_vp]
    L.qn_eigen_residual.argtypes = [c_vp, c_vp, c_vp, c_vp]
    L.qn_eigen_iterate.argtypes = [c_vp, c_vp, c_dbl, c_i32, ctypes.POINTER(QNStats),
                                   ctypes.POINTER(c_dbl)]
    L.qn_nodes.argtypes = [c_vp, c_i32, c_vp]
    L.qn_probe_sink_bytes.argtypes = []
    L.qn_probe_sink_bytes.restype = ctypes.c_size_t
    L.qn_probe_mfma.argtypes = [c_i32, c_vp, ctypes.c_size_t, c_vp, ctypes.POINTER(c_dbl)]
    L.qn_probe_mfma.restype = c_i32
    L.qn_autotune.argtypes = [c_vp]
    L.qn_tile_info.argtypes = [c_vp, c_i32, ctypes.POINTER(c_i32)]
    L.qn_set_tile.argtypes = [c_vp, c_i32, ctypes.POINTER(c_i32)]
    L.qn_destroy.argtypes = [c_vp]
    L.qn_destroy.restype = None
    L.qn_last_error.argtypes = []
    L.qn_last_error.restype = ctypes.c_char_p
    for name in ("qn_setup", "qn_workspace_bytes", "qn_bind_workspace", "qn_set_stream",
                 "qn_residual", "qn_residual_noalloc", "qn_fdm_solve", "qn_iterate", "qn_timing_count",
                 "qn_timing_read", "qn_timing_reset", "qn_autotune", "qn_tile_info",
                 "qn_set_tile", "qn_eigen_residual", "qn_eigen_iterate", "qn_nodes"):
        getattr(L, name).restype = c_i32
    _lib = L
    return L


def last_error():
    return lib().qn_last_error().decode()


def check(status):
    if status != QN_OK:
        raise QNError(status, last_error())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Solver:
    """One problem instance: grid, nonlinearity, shift rule and precision.

    shape: array shape of one component, (ny, nx) or (nz, ny, nx), interior
    nodes.  Field tensors passed to the methods are float64, contiguous, on
    the GPU, with shape (ncomp,) + shape.
    """

    def __init__(self, shape, nonlinearity="cubic", beta=0.0, beta_mode="fixed",
                 precision="fp64", timing=False, device="cuda", boundary="dirichlet",
                 length=None, lin=0.0, cub=1.0, potential=None, discretization="fd",
                 sem_order=0, quad=0.0, workspace=True, step=1.0, gs=None):
        """boundary: "dirichlet" (n interior nodes per axis, h = L/(n+1)) or
        "neumann" (n nodes including both ends, zero normal derivative,
        h = L/(n-1)); length: the domain side L (default 1 for Dirichlet, 2 for
        Neumann, i.e. [-1, 1]).  Cubic problem only: lin, quad, cub, potential
        give -Lap u + lin u + quad u^2 + cub u^3 + V u = f (cub = 0 means 1; pass
        1e-300 or smaller for no cubic term); potential: None or a float64
        device tensor V of the grid's shape, kept referenced by the solver
        (the library reads it on every residual).  discretization: "fd" or "sem"
        (Q^k spectral elements of order sem_order; n = E k - 1 interior nodes for
        Dirichlet data, E k + 1 for Neumann data).  workspace=False skips the
        device workspace (only residual_noalloc may then be called).  step: the
        step size of iterate (U -= step dU).  gs: "grayscott" only, (D_A, D_S,
        rho, mu), None = the values of the paper's example."""
        L = lib()
        self.shape = tuple(int(s) for s in shape)
        self.dim = len(self.shape)
        self.nl = nonlinearity
        self.ncomp = 2 if nonlinearity in ("system", "grayscott") else 1
        self.device = torch.device(device)
        g = QNGrid()
        g.dim = self.dim
        rev = list(reversed(self.shape)) + [1] * (3 - self.dim)
        for a in range(3):
            g.n[a] = rev[a]
        g.ncomp = self.ncomp
        o = QNOptions()
        o.precision = PRECISIONS[precision]
        o.beta_mode = BETA_MODES[beta_mode]
        o.timing = 1 if timing else 0
        o.boundary = BOUNDARIES[boundary]
        o.length = float(length if length is not None else (2.0 if boundary == "neumann" else 1.0))
        o.lin = float(lin)
        o.cub = float(cub)
        o.quad = float(quad)
        o.discretization = DISCRETIZATIONS[discretization]
        o.sem_order = int(sem_order)
        o.step = float(step)
        if gs is not None:
            o.gs_da, o.gs_ds, o.gs_rho, o.gs_mu = (float(v) for v in gs)
        self._potential = None
        if potential is not None:
            if (potential.dtype != torch.float64 or tuple(potential.shape) != self.shape
                    or not potential.is_contiguous() or potential.device.type != "cuda"):
                raise ValueError("potential must be a contiguous float64 CUDA tensor of shape "
                                 f"{self.shape}")
            self._potential = potential
            o.potential = potential.data_ptr()
        o.stream = None
        self.boundary = boundary
        ctx = c_vp()
        check(L.qn_setup(ctypes.byref(g), float(beta), NONLINEARITIES[nonlinearity],
                         ctypes.byref(o), ctypes.byref(ctx)))
        self._ctx = ctx
        nbytes = ctypes.c_size_t()
        check(L.qn_workspace_bytes(ctx, ctypes.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        self._ws = None
        if workspace:
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
            self._sync_stream()
            check(L.qn_bind_workspace(ctx, _ptr(self._ws), self.workspace_bytes))

    # -- helpers
    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        check(lib().qn_set_stream(self._ctx, ctypes.c_void_p(s)))

    def _field(self, t, name):
        want = (self.ncomp,) + self.shape
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
            raise ValueError(f"{name} must be a float64 CUDA tensor")
        if tuple(t.shape) != want or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {want}, got {tuple(t.shape)}")
        return t

    def empty(self):
        return torch.empty((self.ncomp,) + self.shape, dtype=torch.float64, device=self.device)

    # -- entry points
    def residual(self, U, F, R=None, red=None):
        """R = F^h(U); red (optional, float64[4] CUDA) gets {sum R^2, min mu, max mu, sum F^2}."""
        self._field(U, "U")
        self._field(F, "F")
        R = self.empty() if R is None else self._field(R, "R")
        self._sync_stream()
        check(lib().qn_residual(self._ctx, _ptr(U), _ptr(F), _ptr(R), _ptr(red)))
        return R

    def residual_noalloc(self, U, F, R, red=None):
        """qn_residual_noalloc: as residual(), with the reduction scratch in the
        library's fixed device array (no workspace needed, nothing allocated;
        R and red are caller-provided)."""
        self._field(U, "U")
        self._field(F, "F")
        self._field(R, "R")
        self._sync_stream()
        check(lib().qn_residual_noalloc(self._ctx, _ptr(U), _ptr(F), _ptr(R), _ptr(red)))
        return R

    def fdm_solve(self, R, scale=1.0, shift=0.0, X=None):
        """X = (scale A_h + shift I)^-1 R per component."""
        self._field(R, "R")
        X = self.empty() if X is None else self._field(X, "X")
        self._sync_stream()
        check(lib().qn_fdm_solve(self._ctx, _ptr(R), float(scale), float(shift), _ptr(X)))
        return X

    def iterate(self, U, F, rtol=1e-10, max_iter=200, raise_on_error=False):
        """Run the quasi-Newton iteration in place on U; returns a stats dict."""
        self._field(U, "U")
        self._field(F, "F")
        self._sync_stream()
        st = QNStats()
        status = lib().qn_iterate(self._ctx, _ptr(U), _ptr(F), float(rtol), int(max_iter),
                                  ctypes.byref(st))
        if status in (QN_ERR_INVALID, QN_ERR_HIP, QN_ERR_WORKSPACE, QN_ERR_UNSUPPORTED) or (
                raise_on_error and status != QN_OK):
            check(status)
        return {"status": status, "iters": st.iters, "relres": st.relres, "relres0": st.relres0,
                "beta_last": st.beta_last, "scale_last": st.scale_last, "seconds": st.seconds,
                "message": last_error() if status != QN_OK else ""}

    def nodes(self, axis):
        """Coordinates of the unknowns along array axis `axis` (C order: the last
        axis is x), measured from one end of the side."""
        n = self.shape[axis]
        x = (c_dbl * n)()
        check(lib().qn_nodes(self._ctx, self.dim - 1 - axis, x))
        return np.frombuffer(x, dtype=np.float64).copy()

    def eigen_residual(self, U, R=None, out=None):
        """Eigenproblem residual at U / ||U||_M (U unchanged): R = A_h U + f(U) - lam U;
        out (optional, float64[6] CUDA) gets {lam, 1/||U||_M, ||R||_M^2, min mu,
        max mu, ||R||_M / |lam|}."""
        self._field(U, "U")
        R = self.empty() if R is None else self._field(R, "R")
        self._sync_stream()
        check(lib().qn_eigen_residual(self._ctx, _ptr(U), _ptr(R), _ptr(out)))
        return R

    def eigen_iterate(self, U, rtol=1e-10, max_iter=2000, raise_on_error=False):
        """Nonlinear eigenproblem iteration in place on U (normalised on return);
        returns a stats dict with the eigenvalue under "lam"."""
        self._field(U, "U")
        self._sync_stream()
        st = QNStats()
        lam = c_dbl()
        status = lib().qn_eigen_iterate(self._ctx, _ptr(U), float(rtol), int(max_iter),
                                        ctypes.byref(st), ctypes.byref(lam))
        if status in (QN_ERR_INVALID, QN_ERR_HIP, QN_ERR_WORKSPACE, QN_ERR_UNSUPPORTED) or (
                raise_on_error and status != QN_OK):
            check(status)
        return {"status": status, "iters": st.iters, "relres": st.relres, "relres0": st.relres0,
                "beta_last": st.beta_last, "lam": lam.value, "seconds": st.seconds,
                "message": last_error() if status != QN_OK else ""}

    def timing(self, reset=False):
        """{kernel name: (launches, total ms)} for timing-enabled solvers."""
        L = lib()
        out = {}
        for i in range(L.qn_timing_count()):
            name = ctypes.c_char_p()
            n = ctypes.c_int64()
            ms = c_dbl()
            check(L.qn_timing_read(self._ctx, i, ctypes.byref(name), ctypes.byref(n),
                                   ctypes.byref(ms)))
            out[name.value.decode()] = (n.value, ms.value)
        if reset:
            check(L.qn_timing_reset(self._ctx))
        return out

    def autotune(self):
        """Time every admissible tile of each mode-product launch and keep the
        fastest (overwrites the transform workspace; synchronous)."""
        self._sync_stream()
        check(lib().qn_autotune(self._ctx))

    def set_tile(self, i, info):
        """Pin launch i to the tile info = (kind, axis, tile_m, tile_n) as
        returned by tiles(); raises QNError when the shape is not admissible."""
        check(lib().qn_set_tile(self._ctx, int(i), (c_i32 * 4)(*[int(v) for v in info])))

    def tiles(self):
        """[(kind, axis, tile_m, tile_n)] of the solve's mode-product launches
        (kind: 0 x fwd, 1 y/z fwd, 2 y/z inv, 3 x inv; +4 paired; + the LDS
        stage depth when it is not the kernel's default: 32 or 64)."""
        out = []
        info = (c_i32 * 4)()
        for i in range(6 if self.dim == 3 else 4):
            check(lib().qn_tile_info(self._ctx, i, info))
            out.append(tuple(int(v) for v in info))
        return out

    def close(self):
        if getattr(self, "_ctx", None):
            lib().qn_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def probe_mfma(precision="fp64", device="cuda"):
    """Dense MFMA rate (TFLOP/s) of a register-only instruction chain (see
    qn_probe_mfma): the measured matrix-core ceiling of this device."""
    L = lib()
    sink = torch.empty(L.qn_probe_sink_bytes(), dtype=torch.uint8, device=device)
    out = c_dbl()
    stream = torch.cuda.current_stream(device).cuda_stream
    st = L.qn_probe_mfma(PRECISIONS[precision], c_vp(sink.data_ptr()), sink.numel(),
                         c_vp(stream), ctypes.byref(out))
    if st != QN_OK:  # the probe records no message of its own
        raise QNError(st, "qn_probe_mfma failed: precision must be fp64, fp32 or bf16x3")
    return out.value
