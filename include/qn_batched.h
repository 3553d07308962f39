/*
 * qn_batched.h - C ABI of the batched quasi-Newton solver: many independent
 * 2D instances of uneven size, scalar -Lap u + lin u + u^3 = f and 2-component
 * systems -Lap u + u^3 - v = f1, -Lap v + v^3 - u = f2 (Section 4.3,
 * eq. system), each iterated with the quasi-Newton step of Section 4
 * (eq. identity-method) and the tensor-product solve of Section 4.1
 * (eq. fin_inverse), with one shift beta per instance from the range of the
 * Jacobian-diagonal / 2x2-block eigenvalues (Section 4.3 eq. eigenvalues):
 * its midpoint, max, min + max or min (the rules the tables of Sections
 * 6.2-6.3 compare), or a fixed value.
 *
 * Execution: instances of equal (n, ncomp) form a class.  One iteration is,
 * per class, a residual launch, a finalize launch (stopping and shift rules on
 * the device) and four mode-product launches; the classes run on concurrent
 * streams.  A number of iterations is captured once in a hipGraph and the
 * graph is replayed until every instance has stopped; finished instances are
 * skipped on the device by per-instance flags.  Mode-product tile shapes are
 * chosen per class by qnb_autotune (measured with HIP events) or by a default
 * rule.  Transforms run in the chosen precision; residuals, norms, shift rule
 * and update are FP64.
 *
 * Fields: the caller allocates two FP64 device pools (U and F) of
 * qnb_field_elems() doubles.  Instance i's component c occupies n*n
 * contiguous doubles (x fastest) at element offset
 *     offset[i] + c * comp_stride[i]   (qnb_instance_layout).
 * Workspace, ownership, ordering and errors follow qn.h.
 */
#ifndef QN_BATCHED_H
#define QN_BATCHED_H

#include <stddef.h>
#include <stdint.h>

#include "qn.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qnb_ctx_s* qnb_ctx;

/* Per-instance result of qnb_iterate. */
typedef struct {
  int32_t iters;   /* solves performed */
  int32_t status;  /* QN_OK, QN_ERR_NOT_CONVERGED or QN_ERR_DIVERGED */
  double relres;   /* ||F^h(U)|| / ||F|| at the returned U */
  double relres0;  /* same at U_0 */
} qnb_result;

/* count instances (1..65536); n[i] interior points per side (1..4096);
 * ncomp[i] in {1, 2}; precision: qn_precision of the transforms (FP64, FP32
 * or BF16X3; QN_PREC_BF16X6 is rejected with QN_ERR_INVALID); beta_mode
 * (any qn_beta_mode) and beta as in qn_setup (applied to every instance);
 * QN_ERR_INVALID also for a fixed beta <= -lam_min(A_h) of some instance and
 * for QN_BETA_MIN with a 2-component instance whose lam_min(A_h) <= 1 (that
 * rule can give beta = -1 there).  Every instance lives on the unit square
 * with Dirichlet data.  Host only. */
qn_status qnb_setup(int32_t count, const int32_t* n, const int32_t* ncomp, int32_t precision,
                    int32_t beta_mode, double beta, qnb_ctx* out);

/* Problem options shared by every instance of a batch (qnb_setup_ex):
 *   boundary  qn_boundary.  QN_BC_DIRICHLET: n[i] interior points per side,
 *             h = length / (n[i] + 1).  QN_BC_NEUMANN: zero normal derivative
 *             by ghost nodes (Section 3.2), all n[i] nodes of the closed
 *             square are unknowns, h = length / (n[i] - 1); the 1D factors are
 *             the cosine eigenpairs, whose lowest eigenvalue is 0.
 *   length    side of the square (0 means 1).
 *   lin       coefficient of the linear term of the scalar problem
 *             -Lap u + lin u + u^3 = f (Section 6.2, Example 1, eq. ex2d1 has
 *             lin = 1 with Neumann data); its Jacobian diagonal is 3 u^2 + lin.
 */
typedef struct {
  int32_t boundary;
  double length;
  double lin;
  /* system: the problem of the 2-component instances: 0 the cubic system of
   * Section 4.3 (eq. system), 1 the steady Gray-Scott system of Section 6.2
   * (eq. 2dgrayeq; see QN_NL_GRAYSCOTT in qn.h: Neumann data, FP64 or FP32
   * transforms, every instance 2-component, the caller's F = (0, rho)).
   * step: the step size of every update, U -= step dU (0 = 1).
   * gs_da, gs_ds, gs_rho, gs_mu: the Gray-Scott parameters (0 = the values of
   * Section 6.2). */
  int32_t system;
  double step;
  double gs_da, gs_ds, gs_rho, gs_mu;
} qnb_options;

/* qnb_setup with options (NULL: the defaults of qnb_setup).  Besides the
 * checks of qnb_setup, QN_ERR_INVALID for: an unknown boundary; a length
 * that is negative or not finite; a lin that is not finite; lin != 0 with a
 * 2-component instance; Neumann data with n[i] < 2, a 2-component instance
 * or BF16X3 transforms; and a shift rule whose beta can reach -lam_min(A_h)
 * of a scalar instance: every rule on the range of 3 u^2 + lin gives at least
 * lin (min + max: 2 lin when lin < 0), so lam_min(A_h) + that bound must be
 * positive.  With Neumann data lam_min(A_h) = 0: a fixed beta must be > 0
 * and a shift rule needs lin > 0.  The Gray-Scott system (system = 1): its
 * shift rules can give beta <= 0, which would make the solve singular; an
 * instance whose beta_k leaves D_min lam_min(A_h) + beta_k <= 0 stops with
 * QN_ERR_DIVERGED instead.  QN_ERR_UNSUPPORTED for Gray-Scott with Dirichlet
 * data, BF16X3 transforms or a scalar instance; QN_ERR_INVALID for a step or
 * Gray-Scott parameter that is not positive and finite.
 * Host only. */
qn_status qnb_setup_ex(int32_t count, const int32_t* n, const int32_t* ncomp, int32_t precision,
                       int32_t beta_mode, double beta, const qnb_options* opt, qnb_ctx* out);
qn_status qnb_field_elems(qnb_ctx ctx, int64_t* elems);
qn_status qnb_instance_layout(qnb_ctx ctx, int32_t i, int64_t* offset, int64_t* comp_stride);
qn_status qnb_workspace_bytes(qnb_ctx ctx, size_t* bytes);
qn_status qnb_bind_workspace(qnb_ctx ctx, void* d_ws, size_t bytes);
qn_status qnb_set_stream(qnb_ctx ctx, void* stream);

/* Tensor-product solve of every instance (Section 4.1, eq. fin_inverse):
 * X_i = (scale A_h + shift I)^-1 R_i per component (Gray-Scott: with D_c scale
 * A_h), on the pools' layout; d_X may alias d_R.  Uses the transform
 * workspace (any graph of qnb_iterate stays valid).  Asynchronous on the
 * context's stream.  Errors: QN_ERR_INVALID if scale <= 0 or
 * scale lam_min(A_h) + shift <= 0 for some instance. */
qn_status qnb_fdm_solve(qnb_ctx ctx, const double* d_R, double scale, double shift, double* d_X);

/* Time every admissible tile shape of every class's mode products on the
 * bound workspace (contents are overwritten) and keep the fastest.
 * Synchronous. */
qn_status qnb_autotune(qnb_ctx ctx);
/* Number of classes, and class k's (n, ncomp, instance count, tile_m, tile_n
 * of the y products, tile_m, tile_n of the x products). */
qn_status qnb_class_count(qnb_ctx ctx, int32_t* classes);
qn_status qnb_class_info(qnb_ctx ctx, int32_t k, int32_t* info8);

/* Iterate every instance from the U pool (in: U_0, out: last iterates) until
 * relres <= rtol or max_iter solves.  graph_iters iterations are captured per
 * graph replay (>= 1; the graph is rebuilt when pointers or parameters
 * change).  results: host array of count entries (may be NULL).  Returns
 * QN_OK if every instance converged, QN_ERR_NOT_CONVERGED or QN_ERR_DIVERGED
 * if any did not. */
qn_status qnb_iterate(qnb_ctx ctx, double* d_U, const double* d_F, double rtol, int32_t max_iter,
                      int32_t graph_iters, qnb_result* results);

void qnb_destroy(qnb_ctx ctx);

#ifdef __cplusplus
}
#endif

#endif /* QN_BATCHED_H */
