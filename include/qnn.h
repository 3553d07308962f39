/*
 * qnn.h - C ABI of the learned initial-guess network for the quasi-Newton
 * solver (include/qn.h).  Not part of the paper's method: a small
 * convolutional network supplies the starting iterate U_0 of the quasi-Newton
 * iteration (Section 4, eq. identity-method) for 2D -Lap u + u^3 = f.
 *
 * Formulation: the network sees two channels, f / 50 and v0 = A_h^-1 f (one
 * tensor-product solve of the source, Section 4.1), and predicts g, the
 * pointwise nonlinear term U*^3 at the solution.  qnn_forward returns the
 * corrected source f - g; its tensor-product solve A_h^-1 (f - g) is the
 * initial guess.  (A U = f - U^3 holds exactly at the solution, so a
 * prediction of U^3 turns into a smooth, globally consistent U_0, which a
 * 3x3 network with an 11 x 11 receptive field cannot produce directly.)
 * Callers fall back to U_0 = 0 when the guess has a larger residual
 * (qnn_guess_fallback takes that decision on the device).
 *
 * Network: five 3x3 cross-correlation layers with zero "same" padding,
 * channels 2 -> 32 -> 32 -> 32 -> 32 -> 1, exact GELU x*Phi(x) after layers
 * 1-4.  Loss: mean squared error of g over all pixels of the batch.
 * Optimiser: Adam.  All network arithmetic is FP32 (the 32 -> 32 layers on
 * FP32 matrix cores); fields at the ABI are FP64.
 *
 * Parameters: a flat FP32 vector of qnn_param_count() = 28641 entries in the
 * order W1 (32,2,3,3), b1 (32), W2, b2, W3, b3, W4, b4 (each (32,32,3,3),
 * (32)), W5 (1,32,3,3), b5 (1); weights indexed (out, in, dy, dx).
 *
 * Fields: FP64 device arrays (batch, H, W), C-order, x fastest.
 *
 * Ownership and ordering follow qn.h: the caller allocates the workspace
 * (qnn_workspace_bytes, 256-byte aligned) and keeps it alive; calls are
 * enqueued on the net's stream; functions that return host values
 * synchronise that stream.  Errors are qn_status codes with qn_last_error().
 * Reductions are fixed-order, so results are bitwise reproducible.
 */
#ifndef QNN_H
#define QNN_H

#include <stddef.h>
#include <stdint.h>

#include "qn.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qnn_net_s* qnn_net;

/* Create a network for H x W images and batches of at most max_batch
 * (1 <= H, W <= 4096, 1 <= max_batch <= 1024).  Host only. */
qn_status qnn_create(int32_t H, int32_t W, int32_t max_batch, qnn_net* out);
qn_status qnn_workspace_bytes(qnn_net net, size_t* bytes);
/* Bind caller device memory; parameters are initialised He-normal (std
 * sqrt(2/fan_in), splitmix64 + Box-Muller from seed 0), biases zero, Adam
 * moments zero, step 0. */
qn_status qnn_bind_workspace(qnn_net net, void* d_ws, size_t bytes);
qn_status qnn_set_stream(qnn_net net, void* stream);
int32_t qnn_param_count(void);

/* Host <-> device parameter transfer (synchronous).  set_params also resets
 * the Adam moments and step counter. */
qn_status qnn_set_params(qnn_net net, const float* h_params);
qn_status qnn_get_params(qnn_net net, float* h_params);
/* Gradient of the last qnn_loss_grad call (synchronous). */
qn_status qnn_get_grads(qnn_net net, float* h_grads);

/* d_out = d_f - g, g = net(d_f / 50, d_v), for `batch` images, where d_v is
 * the caller's A_h^-1 f (asynchronous).  d_out may not alias d_f or d_v. */
qn_status qnn_forward(qnn_net net, const double* d_f, const double* d_v, int32_t batch,
                      double* d_out);

/* The whole initial guess for one H x W image with a solver context of the
 * same 2D grid (qn.h, QN_NL_CUBIC, workspace bound): v0 = A_h^-1 f,
 * d_u0 = A_h^-1 (f - g(f / 50, v0)), its residual sums into d_red
 * (device double[4], as qn_residual), and the fallback to U_0 = 0 of
 * qnn_guess_fallback (d_used as there).  d_tmp: caller device scratch of one
 * image (overwritten).  Every step is enqueued on the network's stream (the
 * solver context's stream is set to it); asynchronous.  Errors: those of the
 * steps, QN_ERR_INVALID for null or aliased arrays. */
qn_status qnn_guess(qnn_net net, qn_ctx solver, const double* d_f, double* d_u0, double* d_tmp,
                    double* d_red, int32_t* d_used);

/* Inference path of qnn_forward (training always uses FP32): f16 = 0, the FP32
 * layer kernels (default); f16 = 1, one fused kernel for all five layers with
 * FP16 activations and weights on the FP16 matrix cores (FP32 accumulation):
 * each workgroup computes a 16 x 16 output tile and recomputes the halo its
 * receptive field needs, so no activation leaves the chip.  Its g differs from
 * the FP32 network's by FP16 rounding (about 1e-3 relative); the guess only
 * starts the iteration, which reaches the same tolerance.  Host only.
 * Errors: QN_ERR_INVALID for another value. */
qn_status qnn_set_inference(qnn_net net, int32_t f16);

/* Fallback to U_0 = 0, stream-ordered and without a host round trip.
 * d_red is the device[4] reduction that qn_residual wrote for the guess
 * d_u0 (H x W, FP64): {sum R^2, min mu, max mu, sum F^2}.  When
 * !(sum R^2 < sum F^2), i.e. the guess's residual is not smaller than that of
 * U_0 = 0 (whose residual is -F) or is not finite, every entry of d_u0 is set
 * to zero.  d_used (device int32, may be NULL) receives 1 when the guess is
 * kept and 0 otherwise.  One image (batch 1); asynchronous. */
qn_status qnn_guess_fallback(qnn_net net, const double* d_red, double* d_u0, int32_t* d_used);

/* Forward, MSE loss of g against d_target (the nonlinear term at the
 * solution) and backward; gradients are kept in the workspace.  *h_loss (may
 * be NULL) receives the loss (synchronises). */
qn_status qnn_loss_grad(qnn_net net, const double* d_f, const double* d_v, const double* d_target,
                        int32_t batch, double* h_loss);

/* One Adam step with the stored gradients (t advances by one). */
qn_status qnn_adam_step(qnn_net net, double lr, double beta1, double beta2, double eps);

void qnn_destroy(qnn_net net);

#ifdef __cplusplus
}
#endif

#endif /* QNN_H */
