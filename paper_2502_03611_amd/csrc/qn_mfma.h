// Matrix-core traits shared by the mode-product kernels: the 16x16x4 MFMA of
// each element type and the row of the 16x16 output block that accumulator
// element q of a lane holds (the column is lane % 16).  The FP64 and FP32
// instructions differ in that output layout (both checked on the device).
#pragma once

#include <hip/hip_runtime.h>

namespace qn {

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static constexpr int TK = 16;
  __device__ static inline v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int q) { return (lane >> 4) + 4 * q; }
};

template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static constexpr int TK = 32;
  __device__ static inline v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int q) { return 4 * (lane >> 4) + q; }
};

// x / d for the spectral divide (d > 0: the shifted eigenvalue sum, padded
// spectral entries included), from the hardware reciprocal refined by two
// Newton steps and one residual correction of the quotient: within about an
// FP64 ulp of the IEEE quotient in a third of its instructions.
__device__ __forceinline__ double quot(double x, double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
  r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
  const double q = x * r;
  return __builtin_fma(__builtin_fma(-d, q, x), r, q);
}

// x / d in FP32 for d > 0: the hardware reciprocal refined by one Newton
// step, then one residual correction of the quotient (about an FP32 ulp).
// For divides whose result is stored in FP32 (or split from it).
__device__ __forceinline__ float quotf(float x, float d) {
  float r = __builtin_amdgcn_rcpf(d);
  r = __builtin_fmaf(__builtin_fmaf(-d, r, 1.0f), r, r);
  const float q = x * r;
  return __builtin_fmaf(__builtin_fmaf(-d, q, x), r, q);
}

// Tile index for workgroup w of `total`: workgroups are dealt to the 8 XCDs
// round-robin (XCD w % 8), so XCD j is given the contiguous range of
// total / 8 (+1 for j < total % 8) tiles starting at j * (total / 8) +
// min(j, total % 8).  A bijection on [0, total).
__device__ inline int xcd_tile(int w, int total) {
  const int q = total >> 3, r = total & 7, j = w & 7;
  return j * q + (j < r ? j : r) + (w >> 3);
}

}  // namespace qn
