// Kernels of the learned initial-guess network (include/qnn.h): five 3x3
// convolutions 2 -> 32 -> 32 -> 32 -> 32 -> 1 with exact GELU, MSE loss,
// backward pass and Adam, all FP32.
//
// Activations are NHWC with 32 channels contiguous, so the reduction index
// k = (tap, channel) of a 32 -> 32 layer is contiguous per pixel.  Those
// layers (forward, backward-data and weight-gradient) run as implicit GEMMs
// on v_mfma_f32_16x16x4f32 with the input tile and its one-pixel halo staged
// in LDS; channel strides in LDS are padded (36 / 48 floats) so the 16 pixels
// or 16 channels of a fragment fall on distinct banks.  The 2 -> 32 and
// 32 -> 1 layers are small VALU kernels with coalesced 128-byte channel runs.  Weight gradients are reduced by
// writing one partial per workgroup and summing the partials in a fixed order,
// so every result is bitwise reproducible.

#include <algorithm>
#include <cmath>

#include "qnn_internal.h"

namespace qnn {

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
// GELU for the FP16 inference kernel, whose activations are stored in FP16
// (2^-11 relative): erf by the rational-exponential approximation of
// Abramowitz & Stegun (Handbook of Mathematical Functions, eq. 7.1.26;
// |error| <= 1.5e-7), erf(z) = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5))))
// exp(-z^2), t = 1 / (1 + p |z|), with the sign of z; a third of the
// instructions of the library erff, which bounded the fused kernel.
__device__ inline float gelu_fast(float x) {
  const float z = fabsf(x) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(0.3275911f, z, 1.0f));
  float poly = __builtin_fmaf(t, 1.061405429f, -1.453152027f);
  poly = __builtin_fmaf(t, poly, 1.421413741f);
  poly = __builtin_fmaf(t, poly, -0.284496736f);
  poly = __builtin_fmaf(t, poly, 0.254829592f);
  const float e = 1.0f - t * poly * __expf(-z * z);  // erf(|x| / sqrt 2)
  return 0.5f * x * (1.0f + copysignf(e, x));
}
__device__ inline float gelu_grad(float x) {
  const float cdf = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
  const float pdf = expf(-0.5f * x * x) * 0.39894228040143268f;
  return cdf + x * pdf;
}

// ---------------------------------------------------------------- layer 1

// Layer 1: x0 = (f / 50, v0); z1 = b1 + W1 * x0; a1 = gelu(z1).  One thread
// per pixel computes all 32 channels; the weights (32, 2, 3, 3) are staged in
// LDS and read at wave-uniform addresses (broadcast).  The 128 x 32 outputs
// of a workgroup go through LDS (row stride 33: conflict-free columns) so that
// the stores are one contiguous 16 KB run.  TRAIN also keeps x0 and z1 for the
// backward pass.
constexpr int L1_PX = 128;
template <bool TRAIN>
__global__ __launch_bounds__(L1_PX) void k_in_fwd(const double* __restrict__ f,
                                                  const double* __restrict__ v,
                                                  const float* __restrict__ p1,
                                                  float* __restrict__ x0, float* __restrict__ z1,
                                                  float* __restrict__ a1, int H, int W,
                                                  long long npix) {
  __shared__ float sw[L1_SIZE];
  __shared__ float sz[TRAIN ? L1_PX * 33 : 1];
  __shared__ float sa[L1_PX * 33];
  const int l = threadIdx.x;
  for (int i = l; i < L1_SIZE; i += L1_PX) sw[i] = p1[i];
  __syncthreads();
  const long long p0 = (long long)blockIdx.x * L1_PX, p = p0 + l;
  if (p < npix) {
    const int x = (int)(p % W), y = (int)((p / W) % H);
    const long long b = p / ((long long)W * H);
    float nb[CIN0][9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
      const bool in = yy >= 0 && yy < H && xx >= 0 && xx < W;
      const long long q = (b * H + yy) * W + xx;
      nb[0][t] = in ? (float)(f[q] * (1.0 / 50.0)) : 0.0f;
      nb[1][t] = in ? (float)v[q] : 0.0f;
    }
    if (TRAIN) {
      x0[2 * p] = nb[0][4];
      x0[2 * p + 1] = nb[1][4];
    }
#pragma unroll 4
    for (int c = 0; c < 32; ++c) {
      float s = sw[32 * CIN0 * 9 + c];
#pragma unroll
      for (int ci = 0; ci < CIN0; ++ci)
#pragma unroll
        for (int t = 0; t < 9; ++t) s += sw[(c * CIN0 + ci) * 9 + t] * nb[ci][t];
      if (TRAIN) sz[l * 33 + c] = s;
      sa[l * 33 + c] = gelu(s);
    }
  }
  __syncthreads();
  const int np = (int)min((long long)L1_PX, npix - p0);
#pragma unroll 4
  for (int j = 0; j < 32; ++j) {
    const int idx = j * L1_PX + l, px = idx >> 5, c = idx & 31;
    if (px < np) {
      if (TRAIN) z1[(p0 + px) * 32 + c] = sz[px * 33 + c];
      a1[(p0 + px) * 32 + c] = sa[px * 33 + c];
    }
  }
}

// ---------------------------------------------------------------- 32 -> 32 layers

constexpr int CT_Y = 16, CT_X = 32;         // output pixel tile
constexpr int HY = CT_Y + 2, HX = CT_X + 2;  // with halo
constexpr int CP = 36;                       // LDS channel stride (floats)
constexpr int CH = 16;                       // output channels per workgroup

// MODE 0 (forward):  z = bias + sum_k in[p + tap][ci] * Wk[k][co]; writes gelu(z),
// and z too when out0 is not null (training keeps it for the backward pass).
// MODE 1 (backward-data): g = (sum_k dz[p - tap][co] * Wk[k][ci]) * gelu'(zprev[p][ci]).
// Wk is the k-major weight matrix (288 x 32) prepared by k_prep_weights
// (flipped taps for MODE 1).  One workgroup = 8 waves = a 16 x 32 pixel tile
// and one half (16) of the 32 output channels, so a single 255 x 255 image
// still spreads over 256 workgroups; wave w owns rows 2w, 2w+1 (4 MFMA row
// blocks of 16 pixels).  The weight half sits in LDS with row stride 16: the
// four k rows of a fragment then fall on distinct banks.
template <int MODE>
__global__ __launch_bounds__(512) void k_conv32(const float* __restrict__ in,
                                                const float* __restrict__ wk,
                                                const float* __restrict__ bias,
                                                const float* __restrict__ zprev,
                                                float* __restrict__ out0, float* __restrict__ out1,
                                                int H, int W, int tiles_x, int tiles_y) {
  __shared__ __attribute__((aligned(16))) float s_in[HY * HX * CP];
  __shared__ __attribute__((aligned(16))) float s_w[288 * CH];
  const int tid = threadIdx.x;
  int t = blockIdx.x;
  const int half = t & 1;
  t >>= 1;
  const int tx = t % tiles_x;
  t /= tiles_x;
  const int ty = t % tiles_y;
  const int b = t / tiles_y;
  const int y0 = ty * CT_Y, x0 = tx * CT_X;

  for (int i = tid; i < 288 * 4; i += 512) {
    const int k = i >> 2, c4 = i & 3;
    *reinterpret_cast<float4*>(&s_w[k * CH + c4 * 4]) =
        reinterpret_cast<const float4*>(wk)[k * 8 + half * 4 + c4];
  }
  for (int i = tid; i < HY * HX * 8; i += 512) {
    const int c4 = i & 7, pix = i >> 3;
    const int hy = pix / HX, hx = pix % HX;
    const int yy = y0 + hy - 1, xx = x0 + hx - 1;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (yy >= 0 && yy < H && xx >= 0 && xx < W)
      v = reinterpret_cast<const float4*>(in + (((long long)b * H + yy) * W + xx) * 32)[c4];
    *reinterpret_cast<float4*>(&s_in[pix * CP + c4 * 4]) = v;
  }
  __syncthreads();

  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  f4v acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = f4v{0, 0, 0, 0};
  for (int tap = 0; tap < 9; ++tap) {
    const int dy = tap / 3, dx = tap % 3;
#pragma unroll
    for (int c0 = 0; c0 < 32; c0 += 4) {
      const float bw = s_w[(tap * 32 + c0 + lk) * CH + lr];
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        const int r = 2 * wave + (mb >> 1), xh = (mb & 1) * 16;
        const float a = s_in[((r + dy) * HX + xh + lr + dx) * CP + c0 + lk];
        acc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bw, acc[mb], 0, 0, 0);
      }
    }
  }
  const int c = half * CH + lr;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    const int y = y0 + 2 * wave + (mb >> 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int x = x0 + (mb & 1) * 16 + 4 * lk + q;
      if (y >= H || x >= W) continue;
      const long long base = (((long long)b * H + y) * W + x) * 32;
      const float v = acc[mb][q];
      if (MODE == 0) {
        const float z = v + bias[c];
        if (out0) out0[base + c] = z;
        out1[base + c] = gelu(z);
      } else {
        out0[base + c] = v * gelu_grad(zprev[base + c]);
      }
    }
  }
}

constexpr int GT_Y = 8, GT_X = 32;            // weight-gradient pixel tile
constexpr int GHY = GT_Y + 2, GHX = GT_X + 2;  // with halo
constexpr int DS = 48;                         // LDS stride of the dz tile

// Partial weight gradient of a 32 -> 32 layer over one 8 x 32 pixel tile:
// part[co*288 + ci*9 + tap] = sum_p dz[p][co] * act[p + tap][ci] and
// part[9216 + co] = sum_p dz[p][co].  GEMM M = 32 (co) x N = 288 (tap, ci) x
// K = 256 pixels; wave w owns row block w&1 and column blocks (w>>1) + 2i.
__global__ __launch_bounds__(256) void k_conv32_wgrad(const float* __restrict__ act,
                                                      const float* __restrict__ dz,
                                                      float* __restrict__ part, int H, int W,
                                                      int tiles_x, int tiles_y) {
  __shared__ __attribute__((aligned(16))) float s_a[GHY * GHX * CP];
  __shared__ __attribute__((aligned(16))) float s_d[GT_Y * GT_X * DS];
  const int tid = threadIdx.x;
  int t = blockIdx.x;
  const int tx = t % tiles_x;
  t /= tiles_x;
  const int ty = t % tiles_y;
  const int b = t / tiles_y;
  const int y0 = ty * GT_Y, x0 = tx * GT_X;
  for (int i = tid; i < GHY * GHX * 8; i += 256) {
    const int c4 = i & 7, pix = i >> 3;
    const int hy = pix / GHX, hx = pix % GHX;
    const int yy = y0 + hy - 1, xx = x0 + hx - 1;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (yy >= 0 && yy < H && xx >= 0 && xx < W)
      v = reinterpret_cast<const float4*>(act + (((long long)b * H + yy) * W + xx) * 32)[c4];
    *reinterpret_cast<float4*>(&s_a[pix * CP + c4 * 4]) = v;
  }
  for (int i = tid; i < GT_Y * GT_X * 8; i += 256) {
    const int c4 = i & 7, pix = i >> 3;
    const int yy = y0 + pix / GT_X, xx = x0 + pix % GT_X;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (yy < H && xx < W)
      v = reinterpret_cast<const float4*>(dz + (((long long)b * H + yy) * W + xx) * 32)[c4];
    *reinterpret_cast<float4*>(&s_d[pix * DS + c4 * 4]) = v;
  }
  __syncthreads();

  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int mb = wave & 1;
  f4v acc[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) acc[i] = f4v{0, 0, 0, 0};
  for (int kp = 0; kp < GT_Y * GT_X; kp += 4) {
    const int p = kp + lk;
    const int py = p / GT_X, px = p % GT_X;
    const float a = s_d[p * DS + mb * 16 + lr];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int nb = (wave >> 1) + 2 * i;
      const int tap = nb >> 1, ci = (nb & 1) * 16 + lr;
      const float bv = s_a[((py + tap / 3) * GHX + px + tap % 3) * CP + ci];
      acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc[i], 0, 0, 0);
    }
  }
  float* pw = part + (long long)blockIdx.x * QNN_WGRAD_STRIDE;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int nb = (wave >> 1) + 2 * i;
    const int tap = nb >> 1, ci = (nb & 1) * 16 + lr;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int co = mb * 16 + 4 * lk + q;
      pw[co * 288 + ci * 9 + tap] = acc[i][q];
    }
  }
  if (tid < 32) {
    float s = 0.f;
    for (int p = 0; p < GT_Y * GT_X; ++p) s += s_d[p * DS + tid];
    pw[9216 + tid] = s;
  }
}

// ---------------------------------------------------------------- layer 5

// g = b5 + sum_{tap, ci} W5[ci][tap] * a4[p + tap][ci].  Eight lanes per pixel,
// lane c4 over channels 4 c4 .. 4 c4 + 3 of all nine taps (one 16-byte load per
// tap; the eight lanes of a pixel cover its 128-byte channel run), then a
// fixed-order butterfly sum over the eight lanes.  Each lane keeps its 36
// weights in registers (staged through LDS once per workgroup) and walks the
// pixels with a grid stride.  SRC = false stores g (FP32, training); SRC = true
// stores the corrected source f - g in FP64.
template <bool SRC>
__global__ __launch_bounds__(256) void k_out_fwd(const float* __restrict__ a4,
                                                 const float* __restrict__ p5,  // W5 (32x9), b5
                                                 const double* __restrict__ f,
                                                 float* __restrict__ out,
                                                 double* __restrict__ out64, int H, int W,
                                                 int npix) {
  __shared__ float sw[289];
  for (int i = threadIdx.x; i < 289; i += 256) sw[i] = p5[i];
  __syncthreads();
  const int c4 = threadIdx.x & 7;
  float w[4][9];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int t = 0; t < 9; ++t) w[j][t] = sw[(4 * c4 + j) * 9 + t];
  const float bias = sw[288];
  const long long stride = (long long)gridDim.x * 32;
  // The trip count is uniform across each group of eight lanes, so the
  // shuffles below always find their partners.
  for (long long p = ((long long)blockIdx.x * 256 + threadIdx.x) >> 3; p < npix; p += stride) {
    const int x = (int)(p % W), y = (int)((p / W) % H);
    const long long b = p / ((long long)W * H);
    float s = 0.f;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (yy >= 0 && yy < H && xx >= 0 && xx < W)
        v = reinterpret_cast<const float4*>(a4 + ((b * H + yy) * W + xx) * 32)[c4];
      s += w[0][t] * v.x + w[1][t] * v.y + w[2][t] * v.z + w[3][t] * v.w;
    }
    s += __shfl_xor(s, 1, 8);
    s += __shfl_xor(s, 2, 8);
    s += __shfl_xor(s, 4, 8);
    if (c4 == 0) {
      const float g = bias + s;
      if (SRC)
        out64[p] = f[p] - (double)g;
      else
        out[p] = g;
    }
  }
}

// gout = 2 (out - target) / npix; per-block partial of sum (out - target)^2.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ out,
                                             const double* __restrict__ target,
                                             float* __restrict__ gout, double* __restrict__ lpart,
                                             int npix) {
  __shared__ double red[4];
  const int p = blockIdx.x * 256 + threadIdx.x;
  double e2 = 0.0;
  if (p < npix) {
    const double d = (double)out[p] - target[p];
    gout[p] = (float)(2.0 * d / (double)npix);
    e2 = d * d;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) e2 += __shfl_xor(e2, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e2;
  __syncthreads();
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(1024) void k_sum_partials(const double* __restrict__ lpart, int n,
                                                       double scale, double* __restrict__ out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) s += lpart[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < 16; ++i) t += red[i];
    out[0] = t * scale;
  }
}

// dz4[q][ci] = gelu'(z4[q][ci]) * sum_tap gout[q - tap + 1] * W5[ci][tap]
__global__ __launch_bounds__(256) void k_out_bwd(const float* __restrict__ gout,
                                                 const float* __restrict__ p5,
                                                 const float* __restrict__ z4,
                                                 float* __restrict__ dz4, int H, int W, int npix) {
  __shared__ float sw[288];
  for (int i = threadIdx.x; i < 288; i += 256) sw[i] = p5[i];
  __syncthreads();
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= npix) return;
  const int x = p % W, y = (p / W) % H, b = p / (W * H);
  float g[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int yy = y - (t / 3 - 1), xx = x - (t % 3 - 1);
    g[t] = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? gout[((long long)b * H + yy) * W + xx] : 0.f;
  }
  const long long base = (long long)p * 32;
#pragma unroll 4
  for (int c = 0; c < 32; ++c) {
    float s = 0.f;
#pragma unroll
    for (int t = 0; t < 9; ++t) s += g[t] * sw[c * 9 + t];
    dz4[base + c] = s * gelu_grad(z4[base + c]);
  }
}

// Partial weight gradient of the first or last layer over an 8 x 32 pixel
// tile.  IN1 = 1: layer 1, G = dz1 (32 ch), X = x0 (2 ch):
//   part[(co*2 + ci)*9 + tap] = sum_p G[p][co] X[p + tap][ci], part[576 + co] = sum_p G[p][co].
// IN1 = 0: layer 5, G = gout (1 ch), X = a4 (32 ch):
//   part[ci*9 + tap] = sum_p G[p] X[p + tap][ci], part[288] = sum_p G[p].
// One thread per output entry.
template <int IN1>
__global__ __launch_bounds__(640) void k_small_wgrad(const float* __restrict__ G,
                                                     const float* __restrict__ X,
                                                     float* __restrict__ part, int H, int W,
                                                     int tiles_x, int tiles_y) {
  constexpr int GC = IN1 ? 32 : 1, XC = IN1 ? CIN0 : 32;
  constexpr int NW = IN1 ? 32 * CIN0 * 9 : 288;  // weight entries
  constexpr int NB = IN1 ? 32 : 1;               // bias entries
  __shared__ float s_g[GT_Y * GT_X * GC];
  __shared__ float s_x[GHY * GHX * XC];
  int t = blockIdx.x;
  const int tx = t % tiles_x;
  t /= tiles_x;
  const int ty = t % tiles_y;
  const int b = t / tiles_y;
  const int y0 = ty * GT_Y, x0 = tx * GT_X;
  for (int i = threadIdx.x; i < GT_Y * GT_X * GC; i += 640) {
    const int c = i % GC, pix = i / GC;
    const int yy = y0 + pix / GT_X, xx = x0 + pix % GT_X;
    s_g[i] = (yy < H && xx < W) ? G[(((long long)b * H + yy) * W + xx) * GC + c] : 0.f;
  }
  for (int i = threadIdx.x; i < GHY * GHX * XC; i += 640) {
    const int c = i % XC, pix = i / XC;
    const int yy = y0 + pix / GHX - 1, xx = x0 + pix % GHX - 1;
    s_x[i] = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? X[(((long long)b * H + yy) * W + xx) * XC + c] : 0.f;
  }
  __syncthreads();
  const int j = threadIdx.x;
  float* pw = part + (long long)blockIdx.x * QNN_SMALL_STRIDE;
  if (j < NW) {
    const int tap = j % 9, dy = tap / 3, dx = tap % 3;
    const int gc = IN1 ? j / (9 * CIN0) : 0;       // channel of G
    const int xc = IN1 ? (j / 9) % CIN0 : j / 9;   // channel of X
    float s = 0.f;
    for (int p = 0; p < GT_Y * GT_X; ++p) {
      const int py = p / GT_X, px = p % GT_X;
      s += s_g[p * GC + gc] * s_x[((py + dy) * GHX + px + dx) * XC + xc];
    }
    pw[j] = s;
  } else if (j < NW + NB) {
    const int c = j - NW;
    float s = 0.f;
    for (int p = 0; p < GT_Y * GT_X; ++p) s += s_g[p * GC + c];
    pw[j] = s;
  }
}

// grads[dst + j] = sum_{w < nparts} part[w * stride + j], j < len (fixed order,
// accumulated in FP64).
__global__ __launch_bounds__(256) void k_reduce_parts(const float* __restrict__ part, int nparts,
                                                      int stride, int len,
                                                      float* __restrict__ dst) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= len) return;
  double s = 0.0;
  for (int w = 0; w < nparts; ++w) s += part[(long long)w * stride + j];
  dst[j] = (float)s;
}

// Layer l (2..4) parameters -> k-major forward weights Wf[tap*32 + ci][co] and
// flipped backward-data weights Wb[tap*32 + co][ci] = W[co][ci][8 - tap].
__global__ __launch_bounds__(256) void k_prep_weights(const float* __restrict__ wl,
                                                      float* __restrict__ wf,
                                                      float* __restrict__ wb) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= 9216) return;
  const int co = i / 288, ci = (i / 9) % 32, tap = i % 9;
  const float v = wl[i];
  wf[(tap * 32 + ci) * 32 + co] = v;
  wb[((8 - tap) * 32 + co) * 32 + ci] = v;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int n,
                                              float lr, float b1, float b2, float eps, float bc1,
                                              float bc2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// u0 = 0 unless red[0] < red[3] (the guess's sum R^2 below sum F^2, the
// residual of U_0 = 0); used = whether the guess is kept.
__global__ __launch_bounds__(256) void k_guess_fallback(const double* __restrict__ red,
                                                        double* __restrict__ u0,
                                                        int* __restrict__ used, int n) {
  const bool keep = red[0] < red[3];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i == 0 && used) used[0] = keep ? 1 : 0;
  if (!keep && i < n) u0[i] = 0.0;
}

// ---------------------------------------------------------------- launchers

static unsigned blocks(long long n, int per) { return (unsigned)((n + per - 1) / per); }

template <int MODE>
static void launch_conv32(const float* in, const float* wk, const float* bias, const float* zprev,
                          float* out0, float* out1, int H, int W, int batch, hipStream_t st) {
  const int tx = (W + CT_X - 1) / CT_X, ty = (H + CT_Y - 1) / CT_Y;
  hipLaunchKernelGGL((k_conv32<MODE>), dim3((unsigned)(2 * tx * ty * batch)), dim3(512), 0, st, in,
                     wk, bias, zprev, out0, out1, H, W, tx, ty);
}

// ------------------------------------------------- fused inference (FP16)
//
// All five layers of one 16 x 16 output tile in one workgroup, activations in
// LDS as FP16, every layer on v_mfma_f32_16x16x32_f16 with FP32 accumulation.
// Layer l's output region extends 5 - l pixels beyond the tile on each side
// (the receptive field of the layers after it), so a workgroup needs no data
// from its neighbours: the halo is recomputed (layers 2-4 compute 1.57 times
// the tile's pixels).  One MFMA covers 16 pixels (rows) x 16 output channels
// (columns) x 32 input channels (the contraction): a 32 -> 32 layer takes one
// MFMA per 3 x 3 tap and channel half; layer 1 packs its 2 channels x 9 taps
// into one 32-deep contraction (18 used), layer 5 uses output column 0 only.
// Positions outside the image are stored as zero (the zero "same" padding of
// every layer).  Weights come as per-lane FP16 fragments (k_prep_half) and
// stay in registers for the whole layer.
constexpr int FT = 16;               // output tile side
constexpr int FSI = FT + 10;         // input region side
constexpr int FS1 = FT + 8;          // layer-1 output side
constexpr int FPS = 40;              // LDS pixel stride in halves (16-byte aligned, conflict-free)
constexpr int FUSED_THREADS = 1024;

typedef _Float16 h8v __attribute__((ext_vector_type(8)));

// One layer with 32 input channels: out region side S (origin o pixels
// before the tile), input region side S + 2 in `src`.  A wave takes pairs of
// 16-pixel blocks and computes both output-channel halves of each from one
// load of its A fragment per tap: four independent accumulation chains.
// LAST (32 -> 1): only output column 0 of the first half is real; writes
// f - (acc + b5) to out64 instead of GELU into `dst`.
template <int NT, int S, int O, bool LAST>
__device__ inline void fused_conv32(const _Float16* __restrict__ src, _Float16* __restrict__ dst,
                                    const uint16_t* __restrict__ wfrag, const float* __restrict__ bias,
                                    int oy, int ox, int H, int W, int b,
                                    const double* __restrict__ f, double* __restrict__ out64) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  constexpr int NH = LAST ? 1 : 2;  // output-channel halves
  constexpr int nblk = (S * S + 15) / 16, SI = S + 2, o = O;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  h8v w[NH][9];
#pragma unroll
  for (int h = 0; h < NH; ++h)
#pragma unroll
    for (int t = 0; t < 9; ++t) w[h][t] = reinterpret_cast<const h8v*>(wfrag)[(h * 9 + t) * 64 + lane];
  for (int blk0 = 2 * wave; blk0 < nblk; blk0 += 2 * (NT / 64)) {
    const _Float16* a0[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int p = min((blk0 + q) * 16 + (lane & 15), S * S - 1);
      a0[q] = src + ((p / S) * SI + p % S) * FPS + 8 * (lane >> 4);
    }
    f4 ac[2][NH];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int h = 0; h < NH; ++h) ac[q][h] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int off = ((t / 3) * SI + (t % 3)) * FPS;
      const h8v a_0 = *reinterpret_cast<const h8v*>(a0[0] + off);
      const h8v a_1 = *reinterpret_cast<const h8v*>(a0[1] + off);
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        ac[0][h] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_0, w[h][t], ac[0][h], 0, 0, 0);
        ac[1][h] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_1, w[h][t], ac[1][h], 0, 0, 0);
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int blk = blk0 + q;
      if (blk >= nblk) break;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int px = blk * 16 + 4 * (lane >> 4) + j;
        if (px >= S * S) continue;
        const int yy = oy - o + px / S, xx = ox - o + px % S;
        const bool in = yy >= 0 && yy < H && xx >= 0 && xx < W;
        if (LAST) {
          if ((lane & 15) == 0 && in) {
            const long long g = ((long long)b * H + yy) * W + xx;
            out64[g] = f[g] - (double)(ac[q][0][j] + bias[0]);
          }
        } else {
#pragma unroll
          for (int h = 0; h < NH; ++h) {
            const int co = 16 * h + (lane & 15);
            dst[px * FPS + co] = (_Float16)(in ? gelu_fast(ac[q][h][j] + bias[co]) : 0.0f);
          }
        }
      }
    }
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_net_fused(const double* __restrict__ f,
                                                             const double* __restrict__ v,
                                                             const float* __restrict__ params,
                                                             const uint16_t* __restrict__ wh,
                                                             double* __restrict__ out64, int H,
                                                             int W, int tiles_x, int tiles_y) {
  __shared__ float s_in[FSI * FSI * 2];
  __shared__ __attribute__((aligned(16))) _Float16 s_x[FS1 * FS1 * FPS];
  __shared__ __attribute__((aligned(16))) _Float16 s_y[(FT + 6) * (FT + 6) * FPS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int t = blockIdx.x;
  const int tx = t % tiles_x;
  t /= tiles_x;
  const int ty = t % tiles_y;
  const int b = t / tiles_y;
  const int ox = tx * FT, oy = ty * FT;
  for (int i = tid; i < FSI * FSI; i += NT) {
    const int yy = oy - 5 + i / FSI, xx = ox - 5 + i % FSI;
    float a = 0.f, c = 0.f;
    if (yy >= 0 && yy < H && xx >= 0 && xx < W) {
      const long long q = ((long long)b * H + yy) * W + xx;
      a = (float)(f[q] * (1.0 / 50.0));
      c = (float)v[q];
    }
    s_in[2 * i] = a;
    s_in[2 * i + 1] = c;
  }
  __syncthreads();
  // layer 1 (2 -> 32): contraction index k = 2 tap + channel (k < 18)
  {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const float* b1 = params + OFF_L1 + 32 * CIN0 * 9;
    const h8v w0 = reinterpret_cast<const h8v*>(wh + WH_L1)[lane];
    const h8v w1 = reinterpret_cast<const h8v*>(wh + WH_L1)[64 + lane];
    constexpr int S = FS1, nblk = (S * S + 15) / 16;
    for (int blk = wave; blk < nblk; blk += NT / 64) {
      const int p = min(blk * 16 + (lane & 15), S * S - 1);
      const int r = p / S, c = p % S;
      h8v a;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = 8 * (lane >> 4) + j;
        const int tap = k >> 1, ch = k & 1;
        a[j] = (_Float16)(k < 18 ? s_in[((r + tap / 3) * (S + 2) + c + tap % 3) * 2 + ch] : 0.0f);
      }
      const f4 z = {0.f, 0.f, 0.f, 0.f};
      const f4 ac0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, w0, z, 0, 0, 0);
      const f4 ac1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, w1, z, 0, 0, 0);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int q = blk * 16 + 4 * (lane >> 4) + j;
        if (q >= S * S) continue;
        const int yy = oy - 4 + q / S, xx = ox - 4 + q % S;
        const bool in = yy >= 0 && yy < H && xx >= 0 && xx < W;
        const int co = lane & 15;
        s_x[q * FPS + co] = (_Float16)(in ? gelu_fast(ac0[j] + b1[co]) : 0.0f);
        s_x[q * FPS + 16 + co] = (_Float16)(in ? gelu_fast(ac1[j] + b1[16 + co]) : 0.0f);
      }
    }
  }
  __syncthreads();
  const uint16_t* wc = wh + WH_CONV;
  fused_conv32<NT, FT + 6, 3, false>(s_x, s_y, wc, params + layer_offset(1) + 9216, oy, ox, H, W,
                                     b, nullptr, nullptr);
  __syncthreads();
  fused_conv32<NT, FT + 4, 2, false>(s_y, s_x, wc + 2 * 9 * 64 * 8, params + layer_offset(2) + 9216,
                                     oy, ox, H, W, b, nullptr, nullptr);
  __syncthreads();
  fused_conv32<NT, FT + 2, 1, false>(s_x, s_y, wc + 2 * 2 * 9 * 64 * 8,
                                     params + layer_offset(3) + 9216, oy, ox, H, W, b, nullptr,
                                     nullptr);
  __syncthreads();
  fused_conv32<NT, FT, 0, true>(s_y, nullptr, wh + WH_L5, params + OFF_L5 + 288, oy, ox, H, W, b, f,
                                out64);
}

// FP16 fragments of the fused inference kernel from the FP32 parameters:
// lane l holds output channel (16 half + l % 16) and contraction rows
// 8 (l / 16) .. 8 (l / 16) + 7 of each layer's B operand.
__global__ __launch_bounds__(256) void k_prep_half(const float* __restrict__ params,
                                                   uint16_t* __restrict__ wh) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= WH_SIZE) return;
  float v = 0.f;
  if (i < WH_CONV) {  // layer 1: [half][lane][j], k = 2 tap + ch
    const int j = i & 7, lane = (i >> 3) & 63, h = i >> 9;
    const int co = 16 * h + (lane & 15), k = 8 * (lane >> 4) + j;
    if (k < 18) v = params[OFF_L1 + (co * CIN0 + (k & 1)) * 9 + (k >> 1)];
  } else if (i < WH_L5) {  // layers 2-4: [layer][half][tap][lane][j], k = input channel
    const int r = i - WH_CONV;
    const int j = r & 7, lane = (r >> 3) & 63, t = (r >> 9) % 9, h = (r / (9 * 512)) & 1,
              l = r / (2 * 9 * 512);
    const int co = 16 * h + (lane & 15), ci = 8 * (lane >> 4) + j;
    v = params[layer_offset(l + 1) + (co * 32 + ci) * 9 + t];
  } else {  // layer 5: [tap][lane][j], output channel 0 in column 0
    const int r = i - WH_L5;
    const int j = r & 7, lane = (r >> 3) & 63, t = r >> 9;
    if ((lane & 15) == 0) v = params[OFF_L5 + (8 * (lane >> 4) + j) * 9 + t];
  }
  const _Float16 hv = (_Float16)v;
  wh[i] = *reinterpret_cast<const uint16_t*>(&hv);
}

hipError_t forward(const Buffers& B, const double* f, const double* v, int batch, double* out64,
                   hipStream_t st) {
  const int H = B.H, W = B.W;
  const int npix = batch * H * W;
  const bool train = out64 == nullptr;
  if (!train && B.infer_f16) {
    const int tx = (W + FT - 1) / FT, ty = (H + FT - 1) / FT;
    hipLaunchKernelGGL(k_net_fused<FUSED_THREADS>, dim3(tx * ty * batch), dim3(FUSED_THREADS), 0, st,
                       f, v, B.params, B.wh, out64, H, W, tx, ty);
    return hipGetLastError();
  }
  // Grid-stride kernels: at most eight workgroups per compute unit.
  const unsigned g1 = blocks(npix, L1_PX);
  if (train)
    hipLaunchKernelGGL((k_in_fwd<true>), dim3(g1), dim3(L1_PX), 0, st, f, v, B.params + OFF_L1,
                       B.x0, B.z[0], B.a[0], H, W, (long long)npix);
  else
    hipLaunchKernelGGL((k_in_fwd<false>), dim3(g1), dim3(L1_PX), 0, st, f, v, B.params + OFF_L1,
                       (float*)nullptr, (float*)nullptr, B.a[0], H, W, (long long)npix);
  for (int l = 1; l < 4; ++l)
    launch_conv32<0>(B.a[l - 1], B.wf[l - 1], B.params + layer_offset(l) + 9216,
                     (const float*)nullptr, train ? B.z[l] : (float*)nullptr, B.a[l], H, W, batch,
                     st);
  const unsigned g8 = std::min(blocks(8LL * npix, 256), 2048u);
  if (train)
    hipLaunchKernelGGL((k_out_fwd<false>), dim3(g8), dim3(256), 0, st, B.a[3], B.params + OFF_L5,
                       f, B.out, (double*)nullptr, H, W, npix);
  else
    hipLaunchKernelGGL((k_out_fwd<true>), dim3(g8), dim3(256), 0, st, B.a[3], B.params + OFF_L5,
                       f, (float*)nullptr, out64, H, W, npix);
  return hipGetLastError();
}

hipError_t loss_grad(const Buffers& B, const double* f, const double* v, const double* target,
                     int batch, hipStream_t st) {
  hipError_t e = forward(B, f, v, batch, nullptr, st);
  if (e != hipSuccess) return e;
  const int H = B.H, W = B.W;
  const int npix = batch * H * W;
  const unsigned nb = blocks(npix, 256);
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, st, B.out, target, B.gout, B.lpart, npix);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, st, B.lpart, (int)nb,
                     1.0 / (double)npix, B.loss);
  // layer 5
  hipLaunchKernelGGL(k_out_bwd, dim3(nb), dim3(256), 0, st, B.gout, B.params + OFF_L5, B.z[3], B.d[0],
                     H, W, npix);
  const int gtx = (W + GT_X - 1) / GT_X, gty = (H + GT_Y - 1) / GT_Y;
  const int nparts = gtx * gty * batch;
  hipLaunchKernelGGL((k_small_wgrad<0>), dim3((unsigned)nparts), dim3(640), 0, st, B.gout, B.a[3],
                     B.part, H, W, gtx, gty);
  hipLaunchKernelGGL(k_reduce_parts, dim3(blocks(289, 256)), dim3(256), 0, st, B.part, nparts,
                     QNN_SMALL_STRIDE, 289, B.grads + OFF_L5);
  // layers 4, 3, 2: weight gradient from (a[l-1], dz_l), then dz_{l-1}
  int cur = 0;
  for (int l = 3; l >= 1; --l) {
    hipLaunchKernelGGL(k_conv32_wgrad, dim3((unsigned)nparts), dim3(256), 0, st, B.a[l - 1],
                       B.d[cur], B.part, H, W, gtx, gty);
    hipLaunchKernelGGL(k_reduce_parts, dim3(blocks(9248, 256)), dim3(256), 0, st, B.part, nparts,
                       QNN_WGRAD_STRIDE, 9248, B.grads + layer_offset(l));
    launch_conv32<1>(B.d[cur], B.wb[l - 1], (const float*)nullptr, B.z[l - 1], B.d[cur ^ 1],
                     (float*)nullptr, H, W, batch, st);
    cur ^= 1;
  }
  // layer 1
  hipLaunchKernelGGL((k_small_wgrad<1>), dim3((unsigned)nparts), dim3(640), 0, st, B.d[cur], B.x0,
                     B.part, H, W, gtx, gty);
  hipLaunchKernelGGL(k_reduce_parts, dim3(blocks(L1_SIZE, 256)), dim3(256), 0, st, B.part, nparts,
                     QNN_SMALL_STRIDE, L1_SIZE, B.grads + OFF_L1);
  return hipGetLastError();
}

hipError_t guess_fallback(const double* red, double* u0, int* used, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_guess_fallback, dim3(blocks(n, 256)), dim3(256), 0, st, red, u0, used, n);
  return hipGetLastError();
}

hipError_t prep_weights(const Buffers& B, hipStream_t st) {
  for (int l = 1; l < 4; ++l)
    hipLaunchKernelGGL(k_prep_weights, dim3(blocks(9216, 256)), dim3(256), 0, st,
                       B.params + layer_offset(l), B.wf[l - 1], B.wb[l - 1]);
  hipLaunchKernelGGL(k_prep_half, dim3(blocks(WH_SIZE, 256)), dim3(256), 0, st, B.params, B.wh);
  return hipGetLastError();
}

hipError_t adam(const Buffers& B, float lr, float b1, float b2, float eps, float bc1, float bc2,
                hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3(blocks(NPARAM, 256)), dim3(256), 0, st, B.params, B.grads, B.m,
                     B.v, NPARAM, lr, b1, b2, eps, bc1, bc2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return prep_weights(B, st);
}

}  // namespace qnn
