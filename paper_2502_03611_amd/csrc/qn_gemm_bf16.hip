// Split-bf16 mode products ("bf16x3"): each FP32 operand x is split into
// bf16 parts x = hi + lo (hi = RNE(x), lo = RNE(x - hi)) and the product is
// formed from three bf16 matrix-core products hi*hi + hi*lo + lo*hi
// accumulated in FP32 (the lo*lo term, of relative size 2^-16 * 2^-16, is
// dropped).  The 1D eigenvector matrix is split once at setup; the tensor
// operand is split while it is staged into LDS.  Same two forms, tiling,
// XCD-aware tile order and epilogues as the FP64/FP32 kernels.
//
// v_mfma_f32_16x16x32_bf16 takes, per lane, 8 consecutive k values of one row
// of A (row = lane % 16, k = 8 * (lane / 16) ..) and of one column of B, so
// both operands are staged in LDS with k contiguous: [m][k] and [n][k], rows
// padded to 40 elements (80 bytes) so that 16 lanes reading 16 rows hit
// distinct 16-byte bank groups.

#include "qn_internal.h"

namespace qn {

typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ inline void split2(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

__device__ inline f4_t mfma3(const bf8_t& ah, const bf8_t& al, const bf8_t& bh, const bf8_t& bl,
                             f4_t c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
  return c;
}

__device__ inline int bf_tile(int w, int total) {
  return (total % 8 == 0) ? (w % 8) * (total / 8) + (w / 8) : w;
}

constexpr int BTK = 32;  // k per chunk = one MFMA k-step
constexpr int BKP = 40;  // padded LDS row length (bf16 elements)

template <int TM, int TN, int EPI>
__global__ __launch_bounds__(256, 2) void k_gemm_left_bf3(const __bf16* __restrict__ Shi,
                                                          const __bf16* __restrict__ Slo,
                                                          const float* __restrict__ B,
                                                          float* __restrict__ C, int M, int ncols,
                                                          int batch, long long bstride,
                                                          EpiArgs ep) {
  constexpr int WM = TM / 2, WN = TN / 2, BM = WM / 16, BN = WN / 16;
  constexpr int NAV = TM * (BTK / 8);        // 16-byte vectors per A part
  constexpr int NBV = (BTK / 4) * (TN / 4);  // (4 rows x 4 cols) B blocks
  constexpr int PA = (NAV + 255) / 256, PB = (NBV + 255) / 256;
  __shared__ __attribute__((aligned(16))) __bf16 Ah[2][TM][BKP];
  __shared__ __attribute__((aligned(16))) __bf16 Al[2][TM][BKP];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[2][TN][BKP];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[2][TN][BKP];

  const int MT = M / TM, NT = ncols / TN;
  const int t = bf_tile(blockIdx.x, batch * MT * NT);
  const int mt = t % MT, rest = t / MT, nt = rest % NT, b = rest / NT;
  const int inst = b % ep.inst_mod;
  if (ep.skip && ep.skip[inst]) return;  // whole workgroup: finished instance
  const int m0 = mt * TM, n0 = nt * TN;
  const float* Bb = B + (long long)b * bstride;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;

  f4_t acc[BM][BN];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) acc[i][j] = f4_t{0, 0, 0, 0};

  bf8_t rah[PA], ral[PA];
  f4_t rb[PB][4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int p = 0; p < PA; ++p) {
      const int v = tid + 256 * p;
      if (v < NAV) {
        const int m = v / (BTK / 8), kv = (v % (BTK / 8)) * 8;
        // S[m][k] with S symmetric: row m, 8 consecutive k.
        const long long off = (long long)(m0 + m) * M + k0 + kv;
        rah[p] = *reinterpret_cast<const bf8_t*>(Shi + off);
        ral[p] = *reinterpret_cast<const bf8_t*>(Slo + off);
      }
    }
#pragma unroll
    for (int p = 0; p < PB; ++p) {
      const int v = tid + 256 * p;
      if (v < NBV) {
        const int g = v / (TN / 4), nq = (v % (TN / 4)) * 4;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          rb[p][r] = *reinterpret_cast<const f4_t*>(Bb + (long long)(k0 + 4 * g + r) * ncols + n0 + nq);
      }
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int p = 0; p < PA; ++p) {
      const int v = tid + 256 * p;
      if (v < NAV) {
        const int m = v / (BTK / 8), kv = (v % (BTK / 8)) * 8;
        *reinterpret_cast<bf8_t*>(&Ah[buf][m][kv]) = rah[p];
        *reinterpret_cast<bf8_t*>(&Al[buf][m][kv]) = ral[p];
      }
    }
#pragma unroll
    for (int p = 0; p < PB; ++p) {
      const int v = tid + 256 * p;
      if (v < NBV) {
        const int g = v / (TN / 4), nq = (v % (TN / 4)) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          bf4_t h, l;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            __bf16 hh, ll;
            split2(rb[p][r][e], hh, ll);
            h[r] = hh;
            l[r] = ll;
          }
          *reinterpret_cast<bf4_t*>(&Bh[buf][nq + e][4 * g]) = h;
          *reinterpret_cast<bf4_t*>(&Bl[buf][nq + e][4 * g]) = l;
        }
      }
    }
  };

  const int nk = M / BTK;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) gload((kc + 1) * BTK);
    const int ko = 8 * (lane >> 4);
    bf8_t ah[BM], al[BM];
#pragma unroll
    for (int i = 0; i < BM; ++i) {
      ah[i] = *reinterpret_cast<const bf8_t*>(&Ah[buf][wm + 16 * i + (lane & 15)][ko]);
      al[i] = *reinterpret_cast<const bf8_t*>(&Al[buf][wm + 16 * i + (lane & 15)][ko]);
    }
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      const bf8_t bh = *reinterpret_cast<const bf8_t*>(&Bh[buf][wn + 16 * j + (lane & 15)][ko]);
      const bf8_t bl = *reinterpret_cast<const bf8_t*>(&Bl[buf][wn + 16 * j + (lane & 15)][ko]);
#pragma unroll
      for (int i = 0; i < BM; ++i) acc[i][j] = mfma3(ah[i], al[i], bh, bl, acc[i][j]);
    }
    if (kc + 1 < nk) lstore(buf ^ 1);
    __syncthreads();
  }

  float* Cb = C + (long long)b * bstride;
  double scale = 0.0, beta = 0.0;
  if (EPI == EPI_DIVIDE) {
    const double* cf = ep.coef + (long long)inst * ep.coef_stride;
    scale = cf[0];
    beta = cf[1];
  }
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + q;
        const int n = n0 + wn + 16 * j + (lane & 15);
        float v = acc[i][j][q];
        if (EPI == EPI_DIVIDE) {
          const double ly = ep.lamY ? ep.lamY[n / ep.px] : 0.0;
          const double d = scale * (ep.lamM[m] + ep.lamX[n % ep.px] + ly) + beta;
          v = (float)((double)v / d);
        }
        Cb[(long long)m * ncols + n] = v;
      }
}

template <int TM, int TN, int EPI>
__global__ __launch_bounds__(256, 2) void k_gemm_right_bf3(const float* __restrict__ A,
                                                           const __bf16* __restrict__ Shi,
                                                           const __bf16* __restrict__ Slo,
                                                           float* __restrict__ C, int rows, int K,
                                                           EpiArgs ep) {
  constexpr int WM = TM / 2, WN = TN / 2, BM = WM / 16, BN = WN / 16;
  constexpr int NAV = TM * (BTK / 8);  // (row, 8 consecutive k) groups of the tensor chunk
  constexpr int NBV = TN * (BTK / 8);  // 16-byte vectors per S part
  constexpr int PA = (NAV + 255) / 256, PB = (NBV + 255) / 256;
  __shared__ __attribute__((aligned(16))) __bf16 Ah[2][TM][BKP];
  __shared__ __attribute__((aligned(16))) __bf16 Al[2][TM][BKP];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[2][TN][BKP];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[2][TN][BKP];

  const int MT = rows / TM, NT = K / TN;
  const int t = bf_tile(blockIdx.x, MT * NT);
  const int nt = t % NT, mt = t / NT;
  const int r0 = mt * TM, n0 = nt * TN;
  if (ep.skip && ep.skip[(r0 / ep.py / ep.pz) % ep.inst_mod]) return;  // finished instance
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;

  f4_t acc[BM][BN];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) acc[i][j] = f4_t{0, 0, 0, 0};

  f4_t ra[PA][2];
  bf8_t rbh[PB], rbl[PB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int p = 0; p < PA; ++p) {
      const int v = tid + 256 * p;
      if (v < NAV) {
        const int r = v / (BTK / 8), kv = (v % (BTK / 8)) * 8;
        const float* src = A + (long long)(r0 + r) * K + k0 + kv;
        ra[p][0] = *reinterpret_cast<const f4_t*>(src);
        ra[p][1] = *reinterpret_cast<const f4_t*>(src + 4);
      }
    }
#pragma unroll
    for (int p = 0; p < PB; ++p) {
      const int v = tid + 256 * p;
      if (v < NBV) {
        const int n = v / (BTK / 8), kv = (v % (BTK / 8)) * 8;
        // S[k][n] = S[n][k]: row n, 8 consecutive k.
        const long long off = (long long)(n0 + n) * K + k0 + kv;
        rbh[p] = *reinterpret_cast<const bf8_t*>(Shi + off);
        rbl[p] = *reinterpret_cast<const bf8_t*>(Slo + off);
      }
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int p = 0; p < PA; ++p) {
      const int v = tid + 256 * p;
      if (v < NAV) {
        const int r = v / (BTK / 8), kv = (v % (BTK / 8)) * 8;
        bf8_t h, l;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          __bf16 hh, ll;
          split2(ra[p][e >> 2][e & 3], hh, ll);
          h[e] = hh;
          l[e] = ll;
        }
        *reinterpret_cast<bf8_t*>(&Ah[buf][r][kv]) = h;
        *reinterpret_cast<bf8_t*>(&Al[buf][r][kv]) = l;
      }
    }
#pragma unroll
    for (int p = 0; p < PB; ++p) {
      const int v = tid + 256 * p;
      if (v < NBV) {
        const int n = v / (BTK / 8), kv = (v % (BTK / 8)) * 8;
        *reinterpret_cast<bf8_t*>(&Bh[buf][n][kv]) = rbh[p];
        *reinterpret_cast<bf8_t*>(&Bl[buf][n][kv]) = rbl[p];
      }
    }
  };

  const int nk = K / BTK;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) gload((kc + 1) * BTK);
    const int ko = 8 * (lane >> 4);
    bf8_t ah[BM], al[BM];
#pragma unroll
    for (int i = 0; i < BM; ++i) {
      ah[i] = *reinterpret_cast<const bf8_t*>(&Ah[buf][wm + 16 * i + (lane & 15)][ko]);
      al[i] = *reinterpret_cast<const bf8_t*>(&Al[buf][wm + 16 * i + (lane & 15)][ko]);
    }
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      const bf8_t bh = *reinterpret_cast<const bf8_t*>(&Bh[buf][wn + 16 * j + (lane & 15)][ko]);
      const bf8_t bl = *reinterpret_cast<const bf8_t*>(&Bl[buf][wn + 16 * j + (lane & 15)][ko]);
#pragma unroll
      for (int i = 0; i < BM; ++i) acc[i][j] = mfma3(ah[i], al[i], bh, bl, acc[i][j]);
    }
    if (kc + 1 < nk) lstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + wm + 16 * i + 4 * (lane >> 4) + q;
        const int n = n0 + wn + 16 * j + (lane & 15);
        const float v = acc[i][j][q];
        if (EPI == EPI_STORE) {
          C[(long long)r * K + n] = v;
        } else {
          const int y = r % ep.py, zc = r / ep.py, z = zc % ep.pz, c = zc / ep.pz;
          if (n < ep.nx && y < ep.ny && z < ep.nz) {
            const long long idx = (((long long)c * ep.nz + z) * ep.ny + y) * ep.nx + n;
            if (EPI == EPI_SUB_DENSE)
              ep.dense[idx] -= (double)v;
            else
              ep.dense[idx] = (double)v;
          }
        }
      }
}

template <int TM, int TN>
static hipError_t bl_tn(const GemmOperands& s, const float* B, float* C, int M, int ncols,
                        int batch, long long bstride, int epi, const EpiArgs& ep, hipStream_t st) {
  const long long tiles = (long long)batch * (M / TM) * (ncols / TN);
  const __bf16* hi = (const __bf16*)s.Shi;
  const __bf16* lo = (const __bf16*)s.Slo;
  if (epi == EPI_DIVIDE)
    hipLaunchKernelGGL((k_gemm_left_bf3<TM, TN, EPI_DIVIDE>), dim3((unsigned)tiles), dim3(256), 0,
                       st, hi, lo, B, C, M, ncols, batch, bstride, ep);
  else
    hipLaunchKernelGGL((k_gemm_left_bf3<TM, TN, EPI_STORE>), dim3((unsigned)tiles), dim3(256), 0,
                       st, hi, lo, B, C, M, ncols, batch, bstride, ep);
  return hipGetLastError();
}

template <int TM, int TN>
static hipError_t br_tn(const GemmOperands& s, const float* A, float* C, int rows, int K, int epi,
                        const EpiArgs& ep, hipStream_t st) {
  const long long tiles = (long long)(rows / TM) * (K / TN);
  const __bf16* hi = (const __bf16*)s.Shi;
  const __bf16* lo = (const __bf16*)s.Slo;
  switch (epi) {
    case EPI_SUB_DENSE:
      hipLaunchKernelGGL((k_gemm_right_bf3<TM, TN, EPI_SUB_DENSE>), dim3((unsigned)tiles),
                         dim3(256), 0, st, A, hi, lo, C, rows, K, ep);
      break;
    case EPI_STORE_DENSE:
      hipLaunchKernelGGL((k_gemm_right_bf3<TM, TN, EPI_STORE_DENSE>), dim3((unsigned)tiles),
                         dim3(256), 0, st, A, hi, lo, C, rows, K, ep);
      break;
    default:
      hipLaunchKernelGGL((k_gemm_right_bf3<TM, TN, EPI_STORE>), dim3((unsigned)tiles), dim3(256),
                         0, st, A, hi, lo, C, rows, K, ep);
  }
  return hipGetLastError();
}

template <int TM>
static hipError_t bl_tm(int tn, const GemmOperands& s, const float* B, float* C, int M,
                        int ncols, int batch, long long bstride, int epi, const EpiArgs& ep,
                        hipStream_t st) {
  switch (tn) {
    case 128: return bl_tn<TM, 128>(s, B, C, M, ncols, batch, bstride, epi, ep, st);
    case 64: return bl_tn<TM, 64>(s, B, C, M, ncols, batch, bstride, epi, ep, st);
    default: return bl_tn<TM, 32>(s, B, C, M, ncols, batch, bstride, epi, ep, st);
  }
}

template <int TM>
static hipError_t br_tm(int tn, const GemmOperands& s, const float* A, float* C, int rows, int K,
                        int epi, const EpiArgs& ep, hipStream_t st) {
  switch (tn) {
    case 128: return br_tn<TM, 128>(s, A, C, rows, K, epi, ep, st);
    case 64: return br_tn<TM, 64>(s, A, C, rows, K, epi, ep, st);
    default: return br_tn<TM, 32>(s, A, C, rows, K, epi, ep, st);
  }
}

hipError_t launch_gemm_bf16x3_left(const GemmOperands& s, const float* B, float* C, int M,
                                   int ncols, int batch, long long bstride, int epi,
                                   const EpiArgs& ep, int tm, int tn, hipStream_t st) {
  switch (tm) {
    case 128: return bl_tm<128>(tn, s, B, C, M, ncols, batch, bstride, epi, ep, st);
    case 64: return bl_tm<64>(tn, s, B, C, M, ncols, batch, bstride, epi, ep, st);
    default: return bl_tm<32>(tn, s, B, C, M, ncols, batch, bstride, epi, ep, st);
  }
}

hipError_t launch_gemm_bf16x3_right(const GemmOperands& s, const float* A, float* C, int rows,
                                    int K, int epi, const EpiArgs& ep, int tm, int tn,
                                    hipStream_t st) {
  switch (tm) {
    case 128: return br_tm<128>(tn, s, A, C, rows, K, epi, ep, st);
    case 64: return br_tm<64>(tn, s, A, C, rows, K, epi, ep, st);
    default: return br_tm<32>(tn, s, A, C, rows, K, epi, ep, st);
  }
}

}  // namespace qn
