// Host side of the learned initial-guess network: the C ABI of include/qnn.h.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>

#include "../../include/qn.h"
#include "../../include/qnn.h"
#include "qn_internal.h"
#include "qnn_internal.h"

namespace qn {
qn_status set_error(qn_status s, const char* fmt, ...);
}

using qnn::Buffers;
using qnn::NPARAM;

struct qnn_net_s {
  int H = 0, W = 0, max_batch = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t need = 0;
  Buffers B{};
  long long step = 0;
  hipError_t sticky = hipSuccess;
};

namespace {

size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

qn_status bad(qn_status s, const char* msg) { return qn::set_error(s, "%s", msg); }

qn_status hip_bad(qnn_net n, hipError_t e, const char* what) {
  n->sticky = e;
  return qn::set_error(QN_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

qn_status check(qnn_net n, bool need_ws) {
  if (!n) return bad(QN_ERR_INVALID, "null network");
  if (n->sticky != hipSuccess) return qn::set_error(QN_ERR_HIP, "sticky HIP error: %s", hipGetErrorString(n->sticky));
  if (need_ws && !n->ws) return bad(QN_ERR_WORKSPACE, "workspace not bound");
  return QN_OK;
}

// He-normal initial weights (std sqrt(2 / fan_in)) from a splitmix64 stream
// and the Box-Muller transform; biases zero.
void he_init(std::vector<float>& p, uint64_t seed) {
  uint64_t s = seed;
  auto next = [&]() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  auto uniform = [&]() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); };
  auto normal = [&]() {
    const double u1 = uniform(), u2 = uniform();
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  };
  p.assign(NPARAM, 0.f);
  const int cin[5] = {qnn::CIN0, 32, 32, 32, 32}, cout[5] = {32, 32, 32, 32, 1};
  for (int l = 0; l < 5; ++l) {
    const int off = qnn::layer_offset(l);
    const double sd = std::sqrt(2.0 / (9.0 * cin[l]));
    for (int i = 0; i < cout[l] * cin[l] * 9; ++i) p[off + i] = (float)(sd * normal());
  }
}

}  // namespace

extern "C" {

int32_t qnn_param_count(void) { return NPARAM; }

qn_status qnn_create(int32_t H, int32_t W, int32_t max_batch, qnn_net* out) {
  if (!out) return bad(QN_ERR_INVALID, "null output pointer");
  if (H < 1 || W < 1 || H > 4096 || W > 4096) return bad(QN_ERR_INVALID, "H and W must be in [1, 4096]");
  if (max_batch < 1 || max_batch > 1024) return bad(QN_ERR_INVALID, "max_batch must be in [1, 1024]");
  qnn_net n = new qnn_net_s();
  n->H = H;
  n->W = W;
  n->max_batch = max_batch;
  const size_t pix = (size_t)max_batch * H * W;
  const size_t tiles = (size_t)max_batch * ((H + 7) / 8) * ((W + 31) / 32);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += a256(bytes);
    return o;
  };
  // record offsets in the (unbound) Buffers as byte offsets; rebased at bind
  struct { size_t params, grads, m, v, wf[3], wb[3], x0, z[4], a[4], d[2], out, gout, part, lpart, loss, wh; } o{};
  o.params = take(NPARAM * 4);
  o.grads = take(NPARAM * 4);
  o.m = take(NPARAM * 4);
  o.v = take(NPARAM * 4);
  for (int i = 0; i < 3; ++i) o.wf[i] = take(9216 * 4);
  for (int i = 0; i < 3; ++i) o.wb[i] = take(9216 * 4);
  o.x0 = take(pix * qnn::CIN0 * 4);
  for (int i = 0; i < 4; ++i) o.z[i] = take(pix * 32 * 4);
  for (int i = 0; i < 4; ++i) o.a[i] = take(pix * 32 * 4);
  for (int i = 0; i < 2; ++i) o.d[i] = take(pix * 32 * 4);
  o.out = take(pix * 4);
  o.gout = take(pix * 4);
  o.part = take(tiles * qnn::QNN_WGRAD_STRIDE * 4);
  o.lpart = take(((pix + 255) / 256) * 8);
  o.loss = take(8);
  o.wh = take(qnn::WH_SIZE * 2);
  n->need = off;
  // stash offsets as fake pointers (rebased by qnn_bind_workspace)
  Buffers& B = n->B;
  B.H = H;
  B.W = W;
  B.params = (float*)o.params;
  B.grads = (float*)o.grads;
  B.m = (float*)o.m;
  B.v = (float*)o.v;
  for (int i = 0; i < 3; ++i) {
    B.wf[i] = (float*)o.wf[i];
    B.wb[i] = (float*)o.wb[i];
  }
  B.x0 = (float*)o.x0;
  for (int i = 0; i < 4; ++i) {
    B.z[i] = (float*)o.z[i];
    B.a[i] = (float*)o.a[i];
  }
  B.d[0] = (float*)o.d[0];
  B.d[1] = (float*)o.d[1];
  B.out = (float*)o.out;
  B.gout = (float*)o.gout;
  B.part = (float*)o.part;
  B.lpart = (double*)o.lpart;
  B.loss = (double*)o.loss;
  B.wh = (uint16_t*)o.wh;
  B.infer_f16 = 0;
  *out = n;
  return QN_OK;
}

qn_status qnn_workspace_bytes(qnn_net n, size_t* bytes) {
  if (!n || !bytes) return bad(QN_ERR_INVALID, "null argument");
  *bytes = n->need;
  return QN_OK;
}

qn_status qnn_set_stream(qnn_net n, void* stream) {
  if (!n) return bad(QN_ERR_INVALID, "null network");
  n->stream = (hipStream_t)stream;
  return QN_OK;
}

qn_status qnn_set_params(qnn_net n, const float* h) {
  qn_status s = check(n, true);
  if (s != QN_OK) return s;
  if (!h) return bad(QN_ERR_INVALID, "null parameter vector");
  hipError_t e = hipMemcpyAsync(n->B.params, h, NPARAM * 4, hipMemcpyHostToDevice, n->stream);
  if (e == hipSuccess) e = qn::launch_zero(n->B.m, a256(NPARAM * 4), n->stream);
  if (e == hipSuccess) e = qn::launch_zero(n->B.v, a256(NPARAM * 4), n->stream);
  if (e == hipSuccess) e = qnn::prep_weights(n->B, n->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  if (e != hipSuccess) return hip_bad(n, e, "set params");
  n->step = 0;
  return QN_OK;
}

qn_status qnn_bind_workspace(qnn_net n, void* d_ws, size_t bytes) {
  if (!n) return bad(QN_ERR_INVALID, "null network");
  if (!d_ws || ((uintptr_t)d_ws & 255u)) return bad(QN_ERR_WORKSPACE, "workspace null or not 256-byte aligned");
  if (bytes < n->need) return qn::set_error(QN_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", bytes, n->need);
  char* base = (char*)d_ws;
  // If rebinding, offsets are recovered from the previous base.
  const uintptr_t old = (uintptr_t)n->ws;
  auto rebase = [&](auto*& p) { p = reinterpret_cast<std::remove_reference_t<decltype(p)>>(base + ((uintptr_t)p - old)); };
  Buffers& B = n->B;
  rebase(B.params);
  rebase(B.grads);
  rebase(B.m);
  rebase(B.v);
  for (int i = 0; i < 3; ++i) {
    rebase(B.wf[i]);
    rebase(B.wb[i]);
  }
  rebase(B.x0);
  for (int i = 0; i < 4; ++i) {
    rebase(B.z[i]);
    rebase(B.a[i]);
  }
  rebase(B.d[0]);
  rebase(B.d[1]);
  rebase(B.out);
  rebase(B.gout);
  rebase(B.part);
  rebase(B.lpart);
  rebase(B.loss);
  rebase(B.wh);
  n->ws = base;
  std::vector<float> p;
  he_init(p, 0);
  return qnn_set_params(n, p.data());
}

qn_status qnn_get_params(qnn_net n, float* h) {
  qn_status s = check(n, true);
  if (s != QN_OK) return s;
  if (!h) return bad(QN_ERR_INVALID, "null output");
  hipError_t e = hipMemcpyAsync(h, n->B.params, NPARAM * 4, hipMemcpyDeviceToHost, n->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  if (e != hipSuccess) return hip_bad(n, e, "get params");
  return QN_OK;
}

qn_status qnn_get_grads(qnn_net n, float* h) {
  qn_status s = check(n, true);
  if (s != QN_OK) return s;
  if (!h) return bad(QN_ERR_INVALID, "null output");
  hipError_t e = hipMemcpyAsync(h, n->B.grads, NPARAM * 4, hipMemcpyDeviceToHost, n->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  if (e != hipSuccess) return hip_bad(n, e, "get grads");
  return QN_OK;
}

qn_status qnn_forward(qnn_net n, const double* d_f, const double* d_v, int32_t batch,
                      double* d_out) {
  qn_status s = check(n, true);
  if (s != QN_OK) return s;
  if (!d_f || !d_v || !d_out) return bad(QN_ERR_INVALID, "null f, v or out");
  if (batch < 1 || batch > n->max_batch) return bad(QN_ERR_INVALID, "batch out of range");
  hipError_t e = qnn::forward(n->B, d_f, d_v, batch, d_out, n->stream);
  if (e != hipSuccess) return hip_bad(n, e, "forward");
  return QN_OK;
}

qn_status qnn_guess_fallback(qnn_net n, const double* d_red, double* d_u0, int32_t* d_used) {
  qn_status s = check(n, false);
  if (s != QN_OK) return s;
  if (!d_red || !d_u0) return bad(QN_ERR_INVALID, "null reduction or guess");
  hipError_t e = qnn::guess_fallback(d_red, d_u0, d_used, n->H * n->W, n->stream);
  if (e != hipSuccess) return hip_bad(n, e, "guess fallback");
  return QN_OK;
}

qn_status qnn_loss_grad(qnn_net n, const double* d_f, const double* d_v, const double* d_target,
                        int32_t batch, double* h_loss) {
  qn_status s = check(n, true);
  if (s != QN_OK) return s;
  if (!d_f || !d_v || !d_target) return bad(QN_ERR_INVALID, "null f, v or target");
  if (batch < 1 || batch > n->max_batch) return bad(QN_ERR_INVALID, "batch out of range");
  hipError_t e = qnn::loss_grad(n->B, d_f, d_v, d_target, batch, n->stream);
  if (e == hipSuccess && h_loss) {
    e = hipMemcpyAsync(h_loss, n->B.loss, 8, hipMemcpyDeviceToHost, n->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  }
  if (e != hipSuccess) return hip_bad(n, e, "loss/grad");
  return QN_OK;
}

qn_status qnn_adam_step(qnn_net n, double lr, double beta1, double beta2, double eps) {
  qn_status s = check(n, true);
  if (s != QN_OK) return s;
  if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return bad(QN_ERR_INVALID, "invalid Adam hyper-parameters");
  n->step += 1;
  const double bc1 = 1.0 - std::pow(beta1, (double)n->step);
  const double bc2 = 1.0 - std::pow(beta2, (double)n->step);
  hipError_t e = qnn::adam(n->B, (float)lr, (float)beta1, (float)beta2, (float)eps, (float)bc1,
                           (float)bc2, n->stream);
  if (e != hipSuccess) return hip_bad(n, e, "adam");
  return QN_OK;
}

qn_status qnn_guess(qnn_net n, qn_ctx solver, const double* d_f, double* d_u0, double* d_tmp,
                    double* d_red, int32_t* d_used) {
  qn_status s = check(n, true);
  if (s != QN_OK) return s;
  if (!solver || !d_f || !d_u0 || !d_tmp || !d_red)
    return bad(QN_ERR_INVALID, "null solver, f, u0, tmp or red");
  if (d_u0 == d_f || d_tmp == d_f || d_tmp == d_u0)
    return bad(QN_ERR_INVALID, "f, u0 and tmp must be distinct arrays");
  // every step on the network's stream, in order
  s = qn_set_stream(solver, n->stream);
  if (s == QN_OK) s = qn_fdm_solve(solver, d_f, 1.0, 0.0, d_tmp);       // v0 = A^-1 f
  if (s == QN_OK) s = qnn_forward(n, d_f, d_tmp, 1, d_u0);              // f - g
  if (s == QN_OK) s = qn_fdm_solve(solver, d_u0, 1.0, 0.0, d_u0);       // U_0 = A^-1 (f - g)
  if (s == QN_OK) s = qn_residual(solver, d_u0, d_f, d_tmp, d_red);     // F^h(U_0)
  if (s == QN_OK) s = qnn_guess_fallback(n, d_red, d_u0, d_used);       // U_0 = 0 if worse
  return s;
}

qn_status qnn_set_inference(qnn_net n, int32_t f16) {
  if (!n) return bad(QN_ERR_INVALID, "null network");
  if (f16 != 0 && f16 != 1) return bad(QN_ERR_INVALID, "f16 must be 0 or 1");
  n->B.infer_f16 = f16;
  return QN_OK;
}

void qnn_destroy(qnn_net n) { delete n; }

}  // extern "C"
