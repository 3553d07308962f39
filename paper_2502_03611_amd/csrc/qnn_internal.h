// Internal declarations of the learned initial-guess network (include/qnn.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qnn {

constexpr int CIN0 = 2;  // input channels: f / 50 and v0 = A_h^-1 f
constexpr int L1_SIZE = 32 * CIN0 * 9 + 32;
constexpr int NPARAM = L1_SIZE + 3 * 9248 + 289;
// Flat parameter offsets: layer 1 (W 32x2x3x3, b 32), layers 2-4 (W 32x32x3x3,
// b 32), layer 5 (W 1x32x3x3, b 1).
constexpr int OFF_L1 = 0;
constexpr int OFF_L5 = L1_SIZE + 3 * 9248;
__host__ __device__ constexpr int layer_offset(int l) { return l == 0 ? 0 : L1_SIZE + (l - 1) * 9248; }

// Per-workgroup partial strides of the weight-gradient kernels (floats).
constexpr int QNN_WGRAD_STRIDE = 9248;  // 32 x 288 weights + 32 biases
constexpr int QNN_SMALL_STRIDE = L1_SIZE;

struct Buffers {
  int H, W;
  float* params;  // NPARAM
  float* grads;   // NPARAM
  float* m;       // Adam first moment
  float* v;       // Adam second moment
  float* wf[3];   // k-major forward weights of layers 2-4 (288 x 32)
  float* wb[3];   // flipped backward-data weights of layers 2-4
  float* x0;      // (B, H, W, 2) input features (f / 50, v0)
  float* z[4];    // (B, H, W, 32) pre-activations of layers 1-4
  float* a[4];    // gelu(z)
  float* d[2];    // (B, H, W, 32) gradient ping-pong buffers
  float* out;     // (B, H, W) network output
  float* gout;    // (B, H, W) dL/dout
  float* part;    // weight-gradient partials
  double* lpart;  // loss partials
  double* loss;   // 1 double
  uint16_t* wh;   // FP16 matrix-core fragments of all five layers (fused inference)
  int infer_f16;  // inference path: 0 the FP32 layer kernels, 1 the fused FP16 kernel
};

// FP16 fragment layout of the fused inference kernel (halves):
// layer 1 [half 2][lane 64][8], layers 2-4 [layer 3][half 2][tap 9][lane 64][8],
// layer 5 [tap 9][lane 64][8].
constexpr int WH_L1 = 0;
constexpr int WH_CONV = 2 * 64 * 8;
constexpr int WH_L5 = WH_CONV + 3 * 2 * 9 * 64 * 8;
constexpr int WH_SIZE = WH_L5 + 9 * 64 * 8;

// Network forward.  out64 == nullptr: training (keeps x0, z and the FP32 output
// for the backward pass); else inference, writing only out64 = f - g (FP64).
hipError_t forward(const Buffers& B, const double* f, const double* v, int batch, double* out64,
                   hipStream_t st);
hipError_t loss_grad(const Buffers& B, const double* f, const double* v, const double* target,
                     int batch, hipStream_t st);
hipError_t prep_weights(const Buffers& B, hipStream_t st);
// u0[0..n) = 0 unless red[0] < red[3]; *used (nullable) = kept.
hipError_t guess_fallback(const double* red, double* u0, int* used, int n, hipStream_t st);
hipError_t adam(const Buffers& B, float lr, float b1, float b2, float eps, float bc1, float bc2,
                hipStream_t st);

}  // namespace qnn
