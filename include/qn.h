/*
 * qn.h - C ABI of the MI355X (gfx950) quasi-Newton / tensor-product solver.
 *
 * Method: Hao, Lee & Zhang, "An Efficient Quasi-Newton Method with Tensor
 * Product Implementation for Solving Quasi-Linear Elliptic Equations and
 * Systems" (arXiv 2502.03611).  The library runs the quasi-Newton iteration
 *     vec(U_{k+1}) = vec(U_k) - tau [c_k A_h + beta_k I]^-1 F^h(U_k)
 * (Section 4, eq. identity-method; tau = 1 unless a step size is set, as for
 * the Gray-Scott system of Section 6.2) on 2D and 3D grids: finite differences
 * with homogeneous Dirichlet or Neumann data (Section 3.2) or Q^k spectral
 * elements (Section 3.1), applying the inverse by the tensor-product (fast
 * diagonalisation) formula of Section 4.1 (eq. fin_inverse): mode-n products
 * with the 1D eigenvector matrix along every axis, a pointwise divide by
 * c (lam_i + lam_j (+ lam_k)) + beta, and the inverse mode-n products.  It
 * also solves the nonlinear eigenproblem of Section 4.4 (qn_eigen_*).  Which
 * combinations of problem, data, discretisation and precision are built is
 * stated at qn_setup and in the option comments below.
 *
 * Data layout (all device arrays): FP64, contiguous, C-order
 * (ncomp, nz, ny, nx) in 3D and (ncomp, ny, nx) in 2D, x fastest; this is the
 * paper's vec order (first index fastest).  n[a] counts the unknowns along
 * axis a: with Dirichlet data the INTERIOR nodes of the side L,
 * h_a = L/(n[a]+1), boundary values zero and not stored; with Neumann data
 * all nodes, h_a = L/(n[a]-1) (see qn_boundary); spectral elements see
 * qn_discretization.  The source F is the PDE right-hand side sampled at the
 * unknowns.
 *
 * Problems (the paper's model -Lap u + lambda u + f(x,u) = 0, Section 2, with
 * lambda = 0):
 *   QN_NL_CUBIC       -Lap u + u^3 = f                      (ncomp = 1)
 *   QN_NL_SYS2_CUBIC  -Lap u + u^3 - v = f1,
 *                     -Lap v + v^3 - u = f2 (Section 4.3)     (ncomp = 2)
 *   QN_NL_QUASILIN    -div((1+u^2) grad u) = f, conservative flux form with
 *                     arithmetic-mean face coefficients       (ncomp = 1)
 *   QN_NL_GRAYSCOTT   the steady Gray-Scott system of Section 6.2 (ncomp = 2,
 *                     2D, Neumann data; see qn_options)
 *
 * Shift rules (beta_mode):
 *   QN_BETA_FIXED     beta_k = beta (the value given to qn_setup), c_k = 1.
 *   QN_BETA_MIDPOINT  beta_k = (min mu + max mu)/2 over the grid, c_k = 1,
 *                     where mu = f_u = 3U^2 (Section 4, midpoint rule) or,
 *                     for the system, mu ranges over the 2x2-block
 *                     eigenvalues of Section 4.3 eq. eigenvalues.
 *   QN_BETA_MAX, QN_BETA_SUM, QN_BETA_MIN  beta_k = max mu, min mu + max mu,
 *                     min mu: the alternatives the paper's tables compare
 *                     the midpoint with (Sections 6.2-6.3), c_k = 1.
 *   QN_NL_QUASILIN always uses c_k = (min a + max a)/2, a = 1 + U^2, and the
 *   fixed beta; every other beta_mode is rejected for it.
 *
 * Precision (transforms only; residual, norms, shift rule and the update are
 * always FP64): QN_PREC_FP64 (FP64 MFMA), QN_PREC_FP32 (FP32 MFMA),
 * QN_PREC_BF16X3 (each operand split into bf16 hi + lo parts, three bf16 MFMA
 * products hi*hi + hi*lo + lo*hi accumulated in FP32), QN_PREC_BF16X6 (three
 * bf16 parts, the six part products of combined order below 3; FP32-level
 * accuracy on the bf16 matrix cores).
 *
 * Ownership: the library never allocates or frees device memory.  The caller
 * queries qn_workspace_bytes, allocates that many bytes of device memory
 * (256-byte aligned) and binds it with qn_bind_workspace; the eigenvector
 * matrices, eigenvalues and transform scratch live there.  All device
 * pointers passed in stay owned by the caller.
 *
 * Ordering: every call is enqueued on the context's stream (options.stream,
 * NULL = the default stream).  qn_residual and qn_fdm_solve are asynchronous.
 * qn_iterate reads a few scalars back per iteration (the residual norm and
 * the shift) while the next iteration (up to max_iter) is already enqueued
 * (the solve and residual of an iteration that has stopped skip themselves on
 * the device), and returns after the stream has drained.  qn_bind_workspace
 * also creates the iteration's read-back buffer (two small slots of pinned,
 * coherent host memory that the device writes directly) and events.
 *
 * Errors: every entry point returns a qn_status; nothing aborts or throws
 * across the ABI.  qn_last_error() gives a thread-local message for the last
 * non-OK status.  A HIP runtime error is sticky: the context must then be
 * destroyed.  Out-parameters are written only on QN_OK, except qn_iterate,
 * which always fills *stats and leaves U at the last iterate.
 *
 * Threading: a context is not thread-safe; distinct contexts on distinct
 * streams are independent.
 */
#ifndef QN_H
#define QN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QN_OK = 0,
  QN_ERR_INVALID = 1,       /* bad argument, null/misaligned pointer, singular shift */
  QN_ERR_HIP = 2,           /* HIP runtime error (sticky) */
  QN_ERR_NOT_CONVERGED = 3, /* max_iter solves done without reaching rtol */
  QN_ERR_DIVERGED = 4,      /* residual became non-finite or exceeded 1e30 * ||F|| */
  QN_ERR_WORKSPACE = 5,     /* workspace missing, too small or misaligned */
  QN_ERR_UNSUPPORTED = 6    /* valid request this build does not implement */
} qn_status;

typedef enum {
  QN_NL_CUBIC = 0,
  QN_NL_QUASILIN = 1,
  QN_NL_SYS2_CUBIC = 2,
  QN_NL_GRAYSCOTT = 3 /* the steady Gray-Scott system, see qn_options */
} qn_nonlinearity;
typedef enum {
  QN_PREC_FP64 = 0,
  QN_PREC_FP32 = 1,
  QN_PREC_BF16X3 = 2,
  QN_PREC_BF16X6 = 3
} qn_precision;
typedef enum {
  QN_BETA_FIXED = 0,
  QN_BETA_MIDPOINT = 1,
  QN_BETA_MAX = 2,  /* beta_k = max mu: an alternative the paper's tables compare */
  QN_BETA_SUM = 3,  /* beta_k = min mu + max mu: likewise                        */
  QN_BETA_MIN = 4   /* beta_k = min mu: likewise                                 */
} qn_beta_mode;

/* dim: 2 or 3.  n[0] = nx, n[1] = ny, n[2] = nz (ignored when dim = 2);
 * 1 <= n[a] <= 4096.  ncomp: 1, or 2 for QN_NL_SYS2_CUBIC. */
typedef struct {
  int32_t dim;
  int32_t n[3];
  int32_t ncomp;
} qn_grid;

/* Boundary data (Section 3.2), homogeneous in both cases:
 * QN_BC_DIRICHLET: u = 0 on the boundary; the unknowns are the n interior
 *   nodes per axis of an interval of length L, h = L / (n + 1).
 * QN_BC_NEUMANN: zero normal derivative by ghost nodes (the ghost value is the
 *   mirror image of the first interior neighbour); the unknowns are all n
 *   nodes including both ends, h = L / (n - 1), n >= 2.  The 1D stiffness
 *   matrix has the rows h^-2 (2, -2) and h^-2 (-2, 2) at the ends and the
 *   cosine eigenvectors cos(j k pi / (n - 1)); its lowest eigenvalue is 0, so
 *   solves need a positive shift.  Supported for QN_NL_CUBIC with the FP64
 *   and FP32 precisions. */
typedef enum { QN_BC_DIRICHLET = 0, QN_BC_NEUMANN = 1 } qn_boundary;

/* Discretisation of -Lap:
 * QN_DISC_FD: second-order finite differences (Section 3.2), as above.
 * QN_DISC_SEM: Q^k spectral elements with Gauss-Lobatto nodes (Section 3.1 and
 *   its remark on Gauss-Lobatto integration): per axis E equal elements of
 *   order k = sem_order (1..8) on the side L; the unknowns are the E k - 1
 *   interior nodes (Dirichlet) or all E k + 1 nodes (Neumann), so n must be of
 *   that form (n <= 1025).  The mass matrix is diagonal and the nonlinearity
 *   acts node by node, so F^h(U) = A_h U + f(U) - F with A_h the Kronecker sum
 *   of H = M^-1 S; H = T Lam T^-1 through the symmetric M^-1/2 S M^-1/2
 *   (Section 4.2), computed on the host at setup by Jacobi rotations on its
 *   even and odd halves.  QN_NL_CUBIC with FP64 or FP32 transforms only; not
 *   for the eigenproblem. */
typedef enum { QN_DISC_FD = 0, QN_DISC_SEM = 1 } qn_discretization;

/* precision: qn_precision; beta_mode: qn_beta_mode; timing: nonzero records
 * HIP events around every kernel launch (see qn_timing_*); boundary:
 * qn_boundary; stream: a hipStream_t, NULL = default stream; length: the
 * side L of the domain (every axis), 0 = 1.0.
 * The pointwise term of QN_NL_CUBIC is the paper's model
 * -Lap u + lambda u + f(x, u) = 0 (Section 2) with f(x, u) = b u^3 + q u^2 +
 * V(x) u - f_src(x) (Section 6.3, eq. ex3d1, has lambda = b = 10 and a
 * potential V; Section 6.2, eq. 2dex, has b = 0 and q = -1):
 * F^h(U) = A_h U + lambda U + q U^2 + b U^3 + V U - F, Jacobian diagonal
 * 3 b U^2 + 2 q U + lambda + V.
 * lin: lambda (finite), default 0.
 * cub: b (finite); 0 = 1.0 (the default problem), a magnitude below 1e-200
 *   selects b = 0.
 * quad: q (finite), default 0; not for the eigenproblem.
 * potential: NULL (V = 0) or a device array V of one component in the grid's
 *   layout ([nz,] ny, nx); read by every qn_residual and qn_iterate call;
 *   owned by the caller, who keeps it valid and unchanged while the context
 *   is in use.
 * The other nonlinearities need lin = 0, cub in {0, 1}, quad = 0 and
 * potential = NULL.
 * discretization: qn_discretization (0: finite differences); sem_order: the
 *   element order k of QN_DISC_SEM.
 * step: the step size tau of qn_iterate, U_{k+1} = U_k - tau dU_k (Section
 *   6.2 uses 0.1 for the Gray-Scott system); 0 = 1 (the undamped step).
 * gs_da, gs_ds, gs_rho, gs_mu: QN_NL_GRAYSCOTT only (0 = the values of
 *   Section 6.2: 2.5e-4, 5e-4, 0.04, 0.065).  The steady Gray-Scott system of
 *   Section 6.2 (eq. 2dgrayeq), 2D with Neumann data, components (A, S):
 *     F^h = (D_A A_h A - S A^2 + (mu + rho) A, D_S A_h S + S A^2 + rho S) - F,
 *   F = (0, rho) supplied by the caller as the source; A_h acts with the
 *   diffusion coefficient of each component, every reaction term is in N_h,
 *   and the shift rules use the real parts of the eigenvalues of the 2 x 2
 *   reaction block [[-2SA + mu + rho, -A^2], [2SA, A^2 + rho]] (Section 4.3,
 *   eq. eigenvalues).  Solves apply (D_c scale A_h + shift I)^-1 to component
 *   c.  FP64 and FP32 transforms, finite differences. */
typedef struct {
  int32_t precision;
  int32_t beta_mode;
  int32_t timing;
  int32_t boundary;
  void* stream;
  double length;
  double lin;
  double cub;
  const double* potential;
  int32_t discretization;
  int32_t sem_order;
  double quad;
  double step;
  double gs_da, gs_ds, gs_rho, gs_mu;
} qn_options;

/* iters: solves performed; status: the qn_status qn_iterate returned;
 * relres: ||F^h(U)||_2 / ||F||_2 at the returned U; relres0: same at U_0;
 * beta_last / scale_last: shift and scale of the last solve; seconds: wall
 * time of the call. */
typedef struct {
  int32_t iters;
  int32_t status;
  double relres;
  double relres0;
  double beta_last;
  double scale_last;
  double seconds;
} qn_stats;

typedef struct qn_ctx_s* qn_ctx;

/* Create a context: validates the grid, computes the closed-form eigenpairs
 * of the 1D stiffness matrix per axis on the host: sine modes of
 * h^-2 tridiag(-1,2,-1) (Section 3.2 eq. Sy; Section 4.2 with M = I) for
 * Dirichlet data, cosine modes of the ghost-point matrix for Neumann data.  beta: the fixed
 * shift (must satisfy beta + sum_a lam_min,a > 0).  opt may be NULL (FP64,
 * fixed beta, no timing, default stream).  No device memory is touched.
 * Errors: QN_ERR_INVALID for dim not in {2,3}, n out of range, ncomp
 * inconsistent with nonlinearity, unknown enum values, a singular shift,
 * QN_BETA_MIDPOINT with QN_NL_QUASILIN, a non-positive or non-finite length,
 * a non-finite lin or cub, a nonzero lin, a cub other than 0 or 1 or a
 * potential with a nonlinearity other than QN_NL_CUBIC, n < 2 with
 * QN_BC_NEUMANN, an unknown discretization, a sem_order outside 1..8 or an n
 * that is not a spectral element grid; QN_ERR_UNSUPPORTED for QN_BC_NEUMANN
 * or QN_DISC_SEM with another nonlinearity than QN_NL_CUBIC or a split-bf16
 * precision. */
qn_status qn_setup(const qn_grid* grid, double beta, int32_t nonlinearity,
                   const qn_options* opt, qn_ctx* out);

/* Coordinates of the unknowns along one axis (0 x, 1 y, 2 z), measured from
 * one end of the side L: Dirichlet finite differences (i + 1) h, Neumann
 * finite differences i h, spectral elements the Gauss-Lobatto nodes of the
 * elements (Section 3.1).  x: host array of n[axis] doubles.  Host only. */
qn_status qn_nodes(qn_ctx ctx, int32_t axis, double* x);

/* Bytes of device workspace the context needs (written to *bytes). */
qn_status qn_workspace_bytes(qn_ctx ctx, size_t* bytes);

/* Bind caller-owned device memory of at least qn_workspace_bytes bytes,
 * 256-byte aligned, and upload the eigen-data into it (stream-ordered).
 * The memory must stay valid until the context is destroyed or rebound.
 * Errors: QN_ERR_WORKSPACE if too small or misaligned. */
qn_status qn_bind_workspace(qn_ctx ctx, void* d_ws, size_t bytes);

/* Change the stream subsequent calls are enqueued on (NULL = default). */
qn_status qn_set_stream(qn_ctx ctx, void* stream);

/* Residual F^h(U) = A_h vec(U) + N_h(U) (Section 4, eq. F_u; system:
 * Section 4.3) with its reductions.  d_U, d_F: inputs; d_R: output (may not
 * alias d_U); all (ncomp, [nz,] ny, nx).  d_red: NULL or device double[4]
 * receiving { sum R^2, min mu, max mu, sum F^2 }, where mu is f_u =
 * 3 b U^2 + lambda + V (cubic), the block eigenvalues lam_- (min) / lam_+ (max) (system), or
 * a = 1 + U^2 (quasi-linear).  Asynchronous. */
qn_status qn_residual(qn_ctx ctx, const double* d_U, const double* d_F, double* d_R,
                      double* d_red);

/* Allocation-free residual, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same F^h(U) and reductions as qn_residual, the same
 * arguments and error behaviour, but the context needs no bound workspace
 * (qn_setup alone suffices) and the call allocates nothing: the workgroup
 * partials and the finalize scalars live in a fixed array of the library,
 * QN_NOALLOC_MAX_BLOCKS * 32 bytes plus 256, which each device holds from the
 * first call on it until the process ends.  Every call on a device shares
 * that array, so calls that overlap on one device (other streams, other
 * threads) race; calls on one stream are ordered.  Call with the context's
 * device current.  Finite differences only.
 * Every grid qn_setup accepts fits: the 3D residual launches at most 16384
 * workgroups of 1024 threads (tiles of whole 512- to 64-column row segments,
 * z-slabs sized to about one resident round of workgroups) or 32768 of 512
 * threads (two components or Neumann data), the 2D one at most 4096
 * (256-column strips).
 * Errors: as qn_residual, plus QN_ERR_UNSUPPORTED for spectral elements and,
 * as a guard, QN_ERR_WORKSPACE for a launch that would need more than
 * QN_NOALLOC_MAX_BLOCKS workgroup partials.  These two are checked before the
 * pointers.
 */
#define QN_NOALLOC_MAX_BLOCKS 65536
qn_status qn_residual_noalloc(qn_ctx ctx, const double* d_U, const double* d_F, double* d_R,
                              double* d_red);

/* Tensor-product solve X = (scale A_h + shift I)^-1 R per component
 * (Section 4.1, eq. fin_inverse), in the context's precision.  d_X may alias
 * d_R.  Errors: QN_ERR_INVALID if scale <= 0 or scale*sum lam_min + shift <= 0.
 * Asynchronous. */
qn_status qn_fdm_solve(qn_ctx ctx, const double* d_R, double scale, double shift,
                       double* d_X);

/* Quasi-Newton iteration from d_U (in: U_0, out: last iterate) for source
 * d_F, until ||F^h(U_k)|| / ||F|| <= rtol or max_iter solves.  rtol = 0 runs
 * exactly max_iter solves (status QN_ERR_NOT_CONVERGED).  Returns QN_OK,
 * QN_ERR_NOT_CONVERGED or QN_ERR_DIVERGED; *stats (may be NULL) is always
 * filled.  ||F|| = 0 gives QN_ERR_INVALID. */
qn_status qn_iterate(qn_ctx ctx, double* d_U, const double* d_F, double rtol,
                     int32_t max_iter, qn_stats* stats);

/* Nonlinear eigenproblem (Section 4.4, eqs. Eigenvalue_p, system_qusi and
 * system_normal; Section 6.3 Example 2, eq. ex3d2 with b = 1600, lambda = 0 and
 * a potential V on (-8, 8)^3) for a QN_NL_CUBIC context with FP64 or FP32
 * transforms: find U and lam with A_h U + f(U) = lam U and ||U||_M = 1, where
 * f(U) = b U^3 + (lambda + V) U takes the context's cub, lin and potential, and
 * <X, Y>_M = h^d sum W X Y is the lumped mass inner product (W = 1 for
 * Dirichlet data; trapezoid weights, 1/2 at each end of an axis, for Neumann
 * data).  The context's source-free parts only are used (no F).
 * Errors: QN_ERR_UNSUPPORTED for another nonlinearity or a split-bf16
 * precision; QN_ERR_WORKSPACE when unbound; QN_ERR_INVALID for null or
 * misaligned pointers. */

/* For the stored d_U (not modified): U = d_U / ||d_U||_M, the Rayleigh
 * quotient lam = <A_h U + f(U), U>_M and d_R = A_h U + f(U) - lam U (output,
 * interior layout, may not alias d_U).  d_out: NULL or device double[6]
 * receiving {lam, 1 / ||d_U||_M, ||R||_M^2, min mu, max mu, ||R||_M / |lam|}
 * with mu = 3 b U^2 + lambda + V - lam.  Asynchronous. */
qn_status qn_eigen_residual(qn_ctx ctx, const double* d_U, double* d_R, double* d_out);

/* The iteration from d_U (in: U_0, any nonzero multiple; out: the last
 * iterate U_n, normalised): lam_n and R_n = A_h U_n + f(U_n) - lam_n U_n; stop
 * when ||R_n||_M / |lam_n| <= rtol (rtol = 0: exactly max_iter solves) or
 * after max_iter solves; beta_n = the context's fixed beta, or with
 * QN_BETA_MIDPOINT (min mu + max mu) / 2 at U_n; U~ = U_n - (A_h + beta_n I)^-1
 * R_n; U_{n+1} = U~ / ||U~||_M.  Returns QN_OK, QN_ERR_NOT_CONVERGED or
 * QN_ERR_DIVERGED (a non-finite residual, or a shift with
 * lam_min(A_h) + beta_n <= 0).  *stats (may be NULL) as for qn_iterate
 * (relres = ||R||_M / |lam|); *lam_out (host, may be NULL) receives the last
 * lam.  Synchronous on return. */
qn_status qn_eigen_iterate(qn_ctx ctx, double* d_U, double rtol, int32_t max_iter,
                           qn_stats* stats, double* lam_out);

/* Matrix-core throughput probe (measurement only, not a step of the solver):
 * a register-only chain of 16x16x4 FP64 (QN_PREC_FP64), 16x16x4 FP32
 * (QN_PREC_FP32) or 16x16x32 bf16 (QN_PREC_BF16X3) MFMA instructions on
 * 8192 waves, timed with HIP events on `stream` (NULL = default); *tflops
 * receives the dense rate reached, the ceiling the mode-product kernels are
 * compared with beside the published peak.  d_sink: caller-owned device
 * memory of at least qn_probe_sink_bytes() bytes (overwritten).  Synchronous.
 * Errors: QN_ERR_INVALID (null or short sink, other precision), QN_ERR_HIP. */
size_t qn_probe_sink_bytes(void);
qn_status qn_probe_mfma(int32_t precision, void* d_sink, size_t bytes, void* stream,
                        double* tflops);

/* Tile selection for the mode products (Section 4.1, eq. fin_inverse, as
 * reflection-folded matrix-core products).  The solve is a fixed list of
 * launches (3D: 6, 2D: 4; the x forward product first, the x inverse product
 * with the update last).  By default each folded launch takes the first
 * instantiated tile shape that divides its extents and gives at least 512
 * workgroups (else the shape with the most workgroups); the dense
 * split-bf16 launches take the largest side that divides each extent.  qn_autotune times every admissible shape
 * of every launch on the bound workspace (its transform tensors are
 * overwritten; the x inverse is timed with a plain store) and keeps the
 * fastest for all later calls.  Results do not depend on the tile shapes
 * (bitwise).  Synchronous.  The split-bf16 precisions use dense
 * (unfolded) products; their tiles are tuned the same way. */
qn_status qn_autotune(qn_ctx ctx);
/* Launch i of the solve: info4 = {kind, axis (0 x, 1 y, 2 z), tile_m,
 * tile_n}; kind is 0 x forward, 1 y/z forward, 2 y/z inverse, 3 x inverse,
 * plus 4 when one tile computes both the even and the odd spectral half
 * (paired forward tiles; tile_m or tile_n then counts fold indices), plus
 * the tile's LDS stage depth tk when it is not the kernel's default (32 or 64
 * contraction rows per stage: deep stages for short contractions).
 * Requires a bound workspace. */
qn_status qn_tile_info(qn_ctx ctx, int32_t i, int32_t* info4);
/* Pin launch i to the tile info4 (same encoding as qn_tile_info), e.g. one
 * that qn_autotune chose for another context of the same grid.  The shape must
 * be instantiated and admissible for the launch (QN_ERR_INVALID otherwise);
 * the other launches keep their current tiles.  Host only. */
qn_status qn_set_tile(qn_ctx ctx, int32_t i, const int32_t* info4);

/* Kernel timing (contexts created with options.timing != 0).  qn_timing_read
 * synchronises the stream, folds all recorded launches into the table, and
 * writes entry i: its kernel name (static string), launch count and total
 * milliseconds.  i ranges over 0 .. qn_timing_count()-1.  qn_timing_reset
 * clears the table. */
int32_t qn_timing_count(void);
qn_status qn_timing_read(qn_ctx ctx, int32_t i, const char** name, int64_t* launches,
                         double* total_ms);
qn_status qn_timing_reset(qn_ctx ctx);

/* Destroy a context (NULL is a no-op).  Does not free the bound workspace. */
void qn_destroy(qn_ctx ctx);

/* Message for the last non-OK status returned on this thread. */
const char* qn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QN_H */
