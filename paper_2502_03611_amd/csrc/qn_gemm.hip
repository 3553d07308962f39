// Mode-n products of the tensor-product solve (Section 4.1, eq. fin_inverse):
// dense GEMMs of the grid with the symmetric 1D eigenvector matrix S, on the
// gfx950 matrix cores, with the spectral divide and the quasi-Newton update
// fused into the epilogues.
//
// Two forms cover the three axes of a C-order (.., z, y, x) tensor:
//   form L  C[b][m][n] = sum_k S[m][k] B[b][k][n]   (y and z products; B rows
//           are contiguous in n, b runs over the batch of slabs)
//   form R  C[r][n]    = sum_k A[r][k] S[k][n]      (x product; A rows are the
//           x-lines of the tensor, contiguous in k)
// S is P x P (P = padded axis length, a multiple of 32) and zero outside the
// N x N block, so padded rows and columns of every tensor stay exactly zero.
//
// Work decomposition: a 256-thread workgroup (four wave64s in a 2 x 2 grid)
// owns a TM x TN output tile and walks K in chunks of TK, staging both
// operand chunks in LDS (double buffered, one barrier per chunk).  Each wave
// computes a (TM/2) x (TN/2) sub-tile as 16 x 16 MFMA blocks.  FP64 uses
// v_mfma_f64_16x16x4f64, FP32 v_mfma_f32_16x16x4f32.  Chunks read from S
// and the form-L tensor chunk are stored in LDS k-major ([k][m], [k][n]), so
// a fragment read is 16 contiguous elements per 16-lane group; the form-R
// tensor chunk keeps its [r][k] layout with padded rows.  Tiles are numbered so that
// neighbours share an operand panel, and the workgroup -> tile map gives each
// of the 8 XCDs (which receive workgroups round-robin) a contiguous range of
// tiles, so a panel is fetched into one XCD's L2 and reused there.

#include "qn_internal.h"
#include "qn_mfma.h"

namespace qn {

// Padded row r = (c * pz + z) * py + y of a form-R product -> offset of the
// dense caller row (c, z, y); false for padding rows.
__device__ inline bool dense_row(const EpiArgs& ep, int r, long long& base) {
  const int y = r % ep.py;
  const int zc = r / ep.py;
  const int z = zc % ep.pz;
  const int c = zc / ep.pz;
  base = (((long long)c * ep.nz + z) * ep.ny + y) * ep.nx;
  return y < ep.ny && z < ep.nz;
}

template <typename T, int TM, int TN, int EPI>
__global__ __launch_bounds__(256, 2) void k_gemm_left(const T* __restrict__ S,
                                                      const T* __restrict__ B,
                                                      T* __restrict__ C, int M, int ncols,
                                                      int batch, long long bstride, EpiArgs ep) {
  using MF = Mfma<T>;
  constexpr int TK = MF::TK;
  constexpr int VE = 16 / sizeof(T);
  typedef T V __attribute__((ext_vector_type(VE)));
  constexpr int WM = TM / 2, WN = TN / 2, BM = WM / 16, BN = WN / 16;
  constexpr int NA = TK * TM / (VE * 256), NB = TK * TN / (VE * 256);
  static_assert(NA >= 1 && NB >= 1, "tile too small for 256 threads");
  __shared__ __attribute__((aligned(16))) T As[2][TK][TM];
  __shared__ __attribute__((aligned(16))) T Bs[2][TK][TN];

  const int MT = M / TM, NT = ncols / TN;
  const int t = xcd_tile(blockIdx.x, batch * MT * NT);
  const int mt = t % MT, rest = t / MT, nt = rest % NT, b = rest / NT;
  const int inst = b % ep.inst_mod;
  if (ep.skip && ep.skip[inst]) return;  // whole workgroup: finished instance
  const int m0 = mt * TM, n0 = nt * TN;
  const T* Bb = B + (long long)b * bstride;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;

  typename MF::v4 acc[BM][BN];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) acc[i][j] = typename MF::v4{0, 0, 0, 0};

  V ra[NA], rb[NB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int v = tid + 256 * i, kk = v / (TM / VE), mm = (v % (TM / VE)) * VE;
      // S[m][k] = S[k][m]: read row k of the symmetric matrix, contiguous in m.
      ra[i] = *reinterpret_cast<const V*>(S + (long long)(k0 + kk) * M + m0 + mm);
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int v = tid + 256 * i, kk = v / (TN / VE), nn = (v % (TN / VE)) * VE;
      rb[i] = *reinterpret_cast<const V*>(Bb + (long long)(k0 + kk) * ncols + n0 + nn);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int v = tid + 256 * i, kk = v / (TM / VE), mm = (v % (TM / VE)) * VE;
      *reinterpret_cast<V*>(&As[buf][kk][mm]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int v = tid + 256 * i, kk = v / (TN / VE), nn = (v % (TN / VE)) * VE;
      *reinterpret_cast<V*>(&Bs[buf][kk][nn]) = rb[i];
    }
  };

  const int nk = M / TK;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) gload((kc + 1) * TK);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      T a[BM], bb[BN];
#pragma unroll
      for (int i = 0; i < BM; ++i) a[i] = As[buf][ks + (lane >> 4)][wm + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < BN; ++j) bb[j] = Bs[buf][ks + (lane >> 4)][wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) acc[i][j] = MF::op(a[i], bb[j], acc[i][j]);
    }
    if (kc + 1 < nk) lstore(buf ^ 1);
    __syncthreads();
  }

  T* Cb = C + (long long)b * bstride;
  if (EPI == EPI_DIVIDE) {
    // d(m, n) = scale * (lamM[m] + lamX[n % px] + lamY[n / px]) + beta; the
    // column part depends on (j, lane) only, the row part on (i, q) only.
    const double* cf = ep.coef + (long long)inst * ep.coef_stride;
    const double scale = cf[0], beta = cf[1];
    double cn[BN];
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      const int n = n0 + wn + 16 * j + (lane & 15);
      const int ny_ = n / ep.px;
      cn[j] = ep.lamX[n - ny_ * ep.px] + (ep.lamY ? ep.lamY[ny_] : 0.0);
    }
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm + 16 * i + MF::row(lane, q);
        const double lm = ep.lamM[m];
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          const int n = n0 + wn + 16 * j + (lane & 15);
          const double d = scale * (lm + cn[j]) + beta;
          Cb[(long long)m * ncols + n] = (T)((double)acc[i][j][q] / d);
        }
      }
  } else {
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm + 16 * i + MF::row(lane, q);
#pragma unroll
        for (int j = 0; j < BN; ++j)
          Cb[(long long)m * ncols + n0 + wn + 16 * j + (lane & 15)] = acc[i][j][q];
      }
  }
}

template <typename T, int TM, int TN, int EPI>
__global__ __launch_bounds__(256, 2) void k_gemm_right(const T* __restrict__ A,
                                                       const T* __restrict__ S,
                                                       T* __restrict__ C, int rows, int K,
                                                       EpiArgs ep) {
  using MF = Mfma<T>;
  constexpr int TK = MF::TK;
  constexpr int VE = 16 / sizeof(T);
  typedef T V __attribute__((ext_vector_type(VE)));
  constexpr int WM = TM / 2, WN = TN / 2, BM = WM / 16, BN = WN / 16;
  constexpr int NA = TK * TM / (VE * 256), NB = TK * TN / (VE * 256);
  static_assert(NA >= 1 && NB >= 1, "tile too small for 256 threads");
  // The A chunk keeps its natural [r][k] layout in LDS.  Rows are padded to
  // TK + 16/sizeof(T) elements (144 bytes for both types): vector stores stay
  // 16-byte aligned and the 16 rows read by a fragment fall on distinct banks.
  constexpr int AK = TK + VE;
  __shared__ __attribute__((aligned(16))) T As[2][TM][AK];
  __shared__ __attribute__((aligned(16))) T Bs[2][TK][TN];

  const int MT = rows / TM, NT = K / TN;
  const int t = xcd_tile(blockIdx.x, MT * NT);
  const int nt = t % NT, mt = t / NT;
  const int r0 = mt * TM, n0 = nt * TN;
  if (ep.skip && ep.skip[(r0 / ep.py / ep.pz) % ep.inst_mod]) return;  // finished instance
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;

  typename MF::v4 acc[BM][BN];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) acc[i][j] = typename MF::v4{0, 0, 0, 0};

  V ra[NA], rb[NB];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int v = tid + 256 * i, row = v / (TK / VE), kv = (v % (TK / VE)) * VE;
      ra[i] = *reinterpret_cast<const V*>(A + (long long)(r0 + row) * K + k0 + kv);
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int v = tid + 256 * i, kk = v / (TN / VE), nn = (v % (TN / VE)) * VE;
      rb[i] = *reinterpret_cast<const V*>(S + (long long)(k0 + kk) * K + n0 + nn);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int v = tid + 256 * i, row = v / (TK / VE), kv = (v % (TK / VE)) * VE;
      *reinterpret_cast<V*>(&As[buf][row][kv]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int v = tid + 256 * i, kk = v / (TN / VE), nn = (v % (TN / VE)) * VE;
      *reinterpret_cast<V*>(&Bs[buf][kk][nn]) = rb[i];
    }
  };

  const int nk = K / TK;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) gload((kc + 1) * TK);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      T a[BM], bb[BN];
#pragma unroll
      for (int i = 0; i < BM; ++i) a[i] = As[buf][wm + 16 * i + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < BN; ++j) bb[j] = Bs[buf][ks + (lane >> 4)][wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) acc[i][j] = MF::op(a[i], bb[j], acc[i][j]);
    }
    if (kc + 1 < nk) lstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = r0 + wm + 16 * i + MF::row(lane, q);
      if (EPI == EPI_STORE) {
#pragma unroll
        for (int j = 0; j < BN; ++j)
          C[(long long)r * K + n0 + wn + 16 * j + (lane & 15)] = acc[i][j][q];
      } else {
        long long base;
        if (dense_row(ep, r, base)) {
#pragma unroll
          for (int j = 0; j < BN; ++j) {
            const int n = n0 + wn + 16 * j + (lane & 15);
            if (n < ep.nx) {
              if (EPI == EPI_SUB_DENSE)
                ep.dense[base + n] -= (double)acc[i][j][q];
              else
                ep.dense[base + n] = (double)acc[i][j][q];
            }
          }
        }
      }
    }
}

// ---------------------------------------------------------------- dispatch

template <typename T, int TM, int TN>
static hipError_t left_tn(const T* S, const T* B, T* C, int M, int ncols, int batch,
                          long long bstride, int epi, const EpiArgs& ep, hipStream_t st) {
  const long long tiles = (long long)batch * (M / TM) * (ncols / TN);
  dim3 grid((unsigned)tiles), block(256);
  if (epi == EPI_DIVIDE)
    hipLaunchKernelGGL((k_gemm_left<T, TM, TN, EPI_DIVIDE>), grid, block, 0, st, S, B, C, M,
                       ncols, batch, bstride, ep);
  else
    hipLaunchKernelGGL((k_gemm_left<T, TM, TN, EPI_STORE>), grid, block, 0, st, S, B, C, M,
                       ncols, batch, bstride, ep);
  return hipGetLastError();
}

template <typename T, int TM, int TN>
static hipError_t right_tn(const T* A, const T* S, T* C, int rows, int K, int epi,
                           const EpiArgs& ep, hipStream_t st) {
  const long long tiles = (long long)(rows / TM) * (K / TN);
  dim3 grid((unsigned)tiles), block(256);
  switch (epi) {
    case EPI_SUB_DENSE:
      hipLaunchKernelGGL((k_gemm_right<T, TM, TN, EPI_SUB_DENSE>), grid, block, 0, st, A, S, C,
                         rows, K, ep);
      break;
    case EPI_STORE_DENSE:
      hipLaunchKernelGGL((k_gemm_right<T, TM, TN, EPI_STORE_DENSE>), grid, block, 0, st, A, S,
                         C, rows, K, ep);
      break;
    default:
      hipLaunchKernelGGL((k_gemm_right<T, TM, TN, EPI_STORE>), grid, block, 0, st, A, S, C, rows,
                         K, ep);
  }
  return hipGetLastError();
}

template <typename T, int TM>
static hipError_t left_tm(int tn, const T* S, const T* B, T* C, int M, int ncols, int batch,
                          long long bstride, int epi, const EpiArgs& ep, hipStream_t st) {
  switch (tn) {
    case 128: return left_tn<T, TM, 128>(S, B, C, M, ncols, batch, bstride, epi, ep, st);
    case 64: return left_tn<T, TM, 64>(S, B, C, M, ncols, batch, bstride, epi, ep, st);
    default: return left_tn<T, TM, 32>(S, B, C, M, ncols, batch, bstride, epi, ep, st);
  }
}

template <typename T, int TM>
static hipError_t right_tm(int tn, const T* A, const T* S, T* C, int rows, int K, int epi,
                           const EpiArgs& ep, hipStream_t st) {
  switch (tn) {
    case 128: return right_tn<T, TM, 128>(A, S, C, rows, K, epi, ep, st);
    case 64: return right_tn<T, TM, 64>(A, S, C, rows, K, epi, ep, st);
    default: return right_tn<T, TM, 32>(A, S, C, rows, K, epi, ep, st);
  }
}

template <typename T>
static hipError_t left_t(int tm, int tn, const T* S, const T* B, T* C, int M, int ncols,
                         int batch, long long bstride, int epi, const EpiArgs& ep,
                         hipStream_t st) {
  switch (tm) {
    case 128: return left_tm<T, 128>(tn, S, B, C, M, ncols, batch, bstride, epi, ep, st);
    case 64: return left_tm<T, 64>(tn, S, B, C, M, ncols, batch, bstride, epi, ep, st);
    default: return left_tm<T, 32>(tn, S, B, C, M, ncols, batch, bstride, epi, ep, st);
  }
}

template <typename T>
static hipError_t right_t(int tm, int tn, const T* A, const T* S, T* C, int rows, int K,
                          int epi, const EpiArgs& ep, hipStream_t st) {
  switch (tm) {
    case 128: return right_tm<T, 128>(tn, A, S, C, rows, K, epi, ep, st);
    case 64: return right_tm<T, 64>(tn, A, S, C, rows, K, epi, ep, st);
    default: return right_tm<T, 32>(tn, A, S, C, rows, K, epi, ep, st);
  }
}

hipError_t launch_gemm_bf16x3_left(const GemmOperands& s, const float* B, float* C, int M,
                                   int ncols, int batch, long long bstride, int epi,
                                   const EpiArgs& ep, int tm, int tn, hipStream_t st);
hipError_t launch_gemm_bf16x3_right(const GemmOperands& s, const float* A, float* C, int rows,
                                    int K, int epi, const EpiArgs& ep, int tm, int tn,
                                    hipStream_t st);

hipError_t launch_gemm_left(int prec, const GemmOperands& s, const void* B, void* C, int M,
                            int ncols, int batch, long long bstride, int epi, const EpiArgs& ep,
                            int tm, int tn, hipStream_t st) {
  if (prec == 0)
    return left_t<double>(tm, tn, (const double*)s.S, (const double*)B, (double*)C, M, ncols,
                          batch, bstride, epi, ep, st);
  if (prec == 1)
    return left_t<float>(tm, tn, (const float*)s.S, (const float*)B, (float*)C, M, ncols, batch,
                         bstride, epi, ep, st);
  return launch_gemm_bf16x3_left(s, (const float*)B, (float*)C, M, ncols, batch, bstride, epi, ep,
                                 tm, tn, st);
}

hipError_t launch_gemm_right(int prec, const GemmOperands& s, const void* A, void* C, int rows,
                             int K, int epi, const EpiArgs& ep, int tm, int tn, hipStream_t st) {
  if (prec == 0)
    return right_t<double>(tm, tn, (const double*)A, (const double*)s.S, (double*)C, rows, K, epi,
                           ep, st);
  if (prec == 1)
    return right_t<float>(tm, tn, (const float*)A, (const float*)s.S, (float*)C, rows, K, epi, ep,
                          st);
  return launch_gemm_bf16x3_right(s, (const float*)A, (float*)C, rows, K, epi, ep, tm, tn, st);
}

}  // namespace qn
