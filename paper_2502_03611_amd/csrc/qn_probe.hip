// Matrix-core throughput probe (measurement only; not a step of the solver):
// every wave runs a register-only chain of MFMA instructions with eight
// independent accumulators (consecutive instructions do not wait on each
// other), and enough waves are launched to fill every SIMD.  The rate it
// reaches is the ceiling the mode-product kernels can be compared with beside
// the published peak.  Each lane stores the sum of its accumulators (a vector
// store) so no instruction is dead.

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "qn.h"
#include "qn_mfma.h"

namespace qn {

namespace {

typedef __bf16 pb8_t __attribute__((ext_vector_type(8)));
typedef float pf4_t __attribute__((ext_vector_type(4)));

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_BLOCKS = 2048;  // 8192 waves: 8 per SIMD on 256 CUs
constexpr int PROBE_ITERS = 2048;
constexpr int NCHAIN = 8;  // independent accumulators per wave

template <typename T>
__global__ __launch_bounds__(PROBE_THREADS) void k_probe(int iters, double* __restrict__ sink) {
  using M = Mfma<T>;
  const int t = blockIdx.x * PROBE_THREADS + threadIdx.x;
  const T a = (T)(1.0 + 1e-3 * (threadIdx.x & 15)), b = (T)(1.0 - 1e-3 * (threadIdx.x >> 4));
  typename M::v4 c[NCHAIN] = {};
  for (int i = 0; i < iters; i += 4) {  // four rounds per trip
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int j = 0; j < NCHAIN; ++j) c[j] = M::op((j & 1) ? a : b, (j & 2) ? a : b, c[j]);
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < NCHAIN; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) s += (double)c[j][q];
  sink[t] = s;
}

__global__ __launch_bounds__(PROBE_THREADS) void k_probe_bf16(int iters, double* __restrict__ sink) {
  const int t = blockIdx.x * PROBE_THREADS + threadIdx.x;
  pb8_t a, b;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    a[j] = (__bf16)(1.0f + 1e-2f * (float)((threadIdx.x + j) & 7));
    b[j] = (__bf16)(1.0f - 1e-2f * (float)((threadIdx.x + 2 * j) & 7));
  }
  pf4_t c[NCHAIN] = {};
  for (int i = 0; i < iters; i += 4) {  // four rounds per trip
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int j = 0; j < NCHAIN; ++j)
        c[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16((j & 1) ? a : b, (j & 2) ? a : b, c[j], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < NCHAIN; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) s += (double)c[j][q];
  sink[t] = s;
}

}  // namespace

}  // namespace qn

extern "C" {

size_t qn_probe_sink_bytes(void) {
  return (size_t)qn::PROBE_BLOCKS * qn::PROBE_THREADS * sizeof(double);
}

qn_status qn_probe_mfma(int32_t precision, void* d_sink, size_t bytes, void* stream,
                        double* tflops) {
  using namespace qn;
  if (!d_sink || !tflops || bytes < qn_probe_sink_bytes()) return QN_ERR_INVALID;
  if (precision < QN_PREC_FP64 || precision > QN_PREC_BF16X3) return QN_ERR_INVALID;
  hipStream_t st = (hipStream_t)stream;
  double* sink = (double*)d_sink;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  auto launch = [&](int iters) {
    if (precision == QN_PREC_FP64)
      hipLaunchKernelGGL(k_probe<double>, dim3(PROBE_BLOCKS), dim3(PROBE_THREADS), 0, st, iters, sink);
    else if (precision == QN_PREC_FP32)
      hipLaunchKernelGGL(k_probe<float>, dim3(PROBE_BLOCKS), dim3(PROBE_THREADS), 0, st, iters, sink);
    else
      hipLaunchKernelGGL(k_probe_bf16, dim3(PROBE_BLOCKS), dim3(PROBE_THREADS), 0, st, iters, sink);
    return hipGetLastError();
  };
  if (e == hipSuccess) e = launch(64);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  if (e == hipSuccess) e = launch(PROBE_ITERS);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (e != hipSuccess) return QN_ERR_HIP;
  // flops per wave instruction: 2 * 16 * 16 * K (K = 4 FP64 / FP32, 32 bf16)
  const double per = precision == QN_PREC_BF16X3 ? 2.0 * 16 * 16 * 32 : 2.0 * 16 * 16 * 4;
  const double waves = (double)PROBE_BLOCKS * PROBE_THREADS / 64.0;
  *tflops = waves * PROBE_ITERS * (double)NCHAIN * per / (ms * 1e-3) / 1e12;
  return QN_OK;
}

}  // extern "C"
