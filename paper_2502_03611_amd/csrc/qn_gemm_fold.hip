// Mode products with the reflection-folded eigenvector matrix.
//
// The sine eigenvectors of the 1D stiffness matrix (Section 3.2 eq. Sy) are
// symmetric or antisymmetric about the grid centre: S[n-1-j][k] = (-1)^k S[j][k]
// (0-based).  The forward transform y = S^T x therefore splits into
//   y[2i]   = sum_{j<h} S[j][2i]   (x[j] + x[n-1-j]) + [n odd] S[h][2i] x[h]
//   y[2i+1] = sum_{j<h} S[j][2i+1] (x[j] - x[n-1-j])
// (h = n/2), and the inverse x = S y into p = S_even y_even, q = S_odd y_odd,
// x[j] = p[j] + q[j], x[n-1-j] = p[j] - q[j], x[h] = p[h].  Each mode product
// of Section 4.1 (eq. fin_inverse) is thus two GEMMs of half the contraction
// length: the same result with half the matrix-core work.
//
// Storage: along a folded axis the spectral index is kept split, even modes
// in [0, bk) and odd modes in [bk, 2 bk) (bk = ceil(n/2) rounded up to 32);
// spatial layout is natural with padded extent 2 bk.  Matrices (bk x bk each):
//   FeT[k][i] = S[k][2i], FoT[k][i] = S[k][2i+1]   (forward: rows k contiguous in i)
//   Fe[i][k]  = S[k][2i], Fo[i][k]  = S[k][2i+1]   (inverse: rows i contiguous in k)
// zero outside the valid block.  Forward loaders fold the contracted operand
// on the fly (two loads per element); inverse kernels keep p and q
// accumulators for the same fold rows and write both mirrored outputs.  Only
// rows / columns below n of a spatial axis are ever read or written.
//
// Work decomposition: a 256-thread workgroup (four wave64s in a 2 x 2 grid)
// owns an output tile and walks the contraction in chunks staged in LDS
// (double-buffered, one barrier per chunk; the global loads of the next chunk
// are issued before the current chunk's matrix-core work).  Two forms cover
// the three axes of a C-order (.., z, y, x) tensor: form L (y and z products,
// contraction over the rows of slabs whose rows are contiguous) and form R
// (x product, contraction along contiguous rows).  Each XCD (workgroups are
// dealt round-robin) walks a contiguous range of tiles, so operand panels
// are reused in its L2.  FP64 uses v_mfma_f64_16x16x4f64, FP32
// v_mfma_f32_16x16x4f32.

#include "qn_internal.h"
#include "qn_mfma.h"

namespace qn {

// Row-major LDS tiles whose rows are the contraction (k) and whose readers
// take one k column of 16 consecutive rows per quarter wave: the 16-byte
// chunks of a row are permuted by an XOR with the row's index within its
// bank group, so both those column reads and the row-wise 16-byte stores hit
// 16 distinct chunks of the LDS banks.  The row's 16-row block (bits 4-5)
// enters the XOR as well: fragment rows 16 apart then sit at a lane-dependent
// distance, which keeps the compiler from pairing their reads into one
// two-address LDS read whose halves fall on the same banks (measured: 8
// conflict cycles per such read).  RB: bytes per row (a power of two).
template <int RB>
__device__ __forceinline__ int swz(int row, int col_bytes) {
  constexpr int NCH = RB / 16, SR = RB >= 256 ? 1 : 256 / RB;
  const int t = ((row / SR) % NCH) ^ ((row >> 4) & 3);
  return row * RB + ((((col_bytes >> 4) ^ t) << 4) | (col_bytes & 15));
}

// The spectral divide x / (scale * lam + beta) of a product result stored as
// T: FP64 in FP64; FP32 results take the denominator and the quotient in FP32
// (the stored value is rounded to FP32 anyway).
template <typename T>
__device__ __forceinline__ T divide_to(T x, double scale, double lam, double beta) {
  if constexpr (sizeof(T) == 4)
    return quotf(x, __builtin_fmaf((float)scale, (float)lam, (float)beta));
  else
    return quot(x, scale * lam + beta);
}

// ------------------------------------------------------------------ form L

// Forward, contraction over the slab rows (the folded axis):
// C[b][m][c] (m in [0, 2 bk)) = sum_{k<bk} F^T_blk[k][i] * fold_blk(B[b])[k][c],
// blk = m / bk, i = m % bk.
template <typename T, int TM, int TN, int EPI, int TKS>
__global__ __launch_bounds__(256, 2) void k_fold_left_fwd(const T* __restrict__ FeT,
                                                          const T* __restrict__ FoT,
                                                          const T* __restrict__ B,
                                                          T* __restrict__ C, FoldAxis ax, int ncols,
                                                          int batch, long long bstride, EpiArgs ep) {
  using MF = Mfma<T>;
  constexpr int TK = TKS ? TKS : MF::TK;
  constexpr int VE = 16 / sizeof(T);
  typedef T V __attribute__((ext_vector_type(VE)));
  constexpr int WM = TM / 2, WN = TN / 2, BM = WM / 16, BN = WN / 16;
  constexpr int NA = (TK * TM / VE + 255) / 256, NB = (TK * TN / VE + 255) / 256;
  __shared__ __attribute__((aligned(16))) T As[2][TK][TM];
  __shared__ __attribute__((aligned(16))) T Bs[2][TK][TN];

  const int bk = ax.bk, P2 = 2 * bk, na = ax.n, h = ax.h;
  const int MT = P2 / TM, NT = ncols / TN;
  const int t = xcd_tile(blockIdx.x, batch * MT * NT);
  const int mt = t % MT, rest = t / MT, nt = rest % NT, b = rest / NT;
  const int inst = b % ep.inst_mod;
  if (ep.skip && ep.skip[inst]) return;
  const int m0 = mt * TM, n0 = nt * TN;
  const int blk = m0 / bk, i0 = m0 - blk * bk;
  const T* F = blk ? FoT : FeT;
  const T* Bb = B + (long long)b * bstride;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;

  typename MF::v4 acc[BM][BN];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) acc[i][j] = typename MF::v4{0, 0, 0, 0};

  // The prefetch keeps the raw row pair; the fold (lo +- hi) happens at the LDS
  // store, so the global loads stay in flight across the MFMA phase.
  V ra[NA], rlo[NB], rhi[NB];
  int kpre = 0;
  auto gload = [&](int k0) {
    kpre = k0;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int v = tid + 256 * i;
      if (v < TK * TM / VE) {
        const int kk = v / (TM / VE), mm = (v % (TM / VE)) * VE;
        ra[i] = *reinterpret_cast<const V*>(F + (long long)(k0 + kk) * bk + i0 + mm);
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int v = tid + 256 * i;
      if (v < TK * TN / VE) {
        const int kk = v / (TN / VE), nn = (v % (TN / VE)) * VE;
        const int k = k0 + kk;
        // rows k and n-1-k (the centre row pairs with itself); clamped for k > h
        const int kl = k <= h ? k : h, kh = k < h ? na - 1 - k : h;
        rlo[i] = *reinterpret_cast<const V*>(Bb + (long long)kl * ncols + n0 + nn);
        rhi[i] = *reinterpret_cast<const V*>(Bb + (long long)kh * ncols + n0 + nn);
      }
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int v = tid + 256 * i;
      if (v < TK * TM / VE) {
        const int kk = v / (TM / VE), mm = (v % (TM / VE)) * VE;
        *reinterpret_cast<V*>(&As[buf][kk][mm]) = ra[i];
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int v = tid + 256 * i;
      if (v < TK * TN / VE) {
        const int kk = v / (TN / VE), nn = (v % (TN / VE)) * VE;
        const int k = kpre + kk;
        V val = V{};
        if (k < h)
          val = blk ? rlo[i] - rhi[i] : rlo[i] + rhi[i];
        else if (k == h && ax.odd && !blk)
          val = rlo[i];
        *reinterpret_cast<V*>(&Bs[buf][kk][nn]) = val;
      }
    }
  };

  // Fold rows at or beyond ne = h + odd contribute nothing: stop the K loop there.
  const int kmax = ((h + ax.odd + TK - 1) / TK) * TK;
  const int nk = kmax / TK;
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
    const double* cf = ep.coef + (long long)inst * ep.coef_stride;
    const double scale = cf[0] * (ep.cscale ? ep.cscale[b / ep.comp_div] : 1.0), beta = cf[1];
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
          Cb[(long long)m * ncols + n] = divide_to<T>(acc[i][j][q], scale, lm + cn[j], beta);
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

// Forward, paired: one tile computes the even spectral rows i and the odd
// rows bk + i (i in [i0, i0 + TMF)) of the same columns, so the raw rows k and
// n-1-k are loaded once for both halves:
//   C[b][i][c]      = sum_{k<ne} FeT[k][i] (B[b][k][c] + B[b][n-1-k][c])
//   C[b][bk + i][c] = sum_{k<h}  FoT[k][i] (B[b][k][c] - B[b][n-1-k][c])
// (the centre row k = h of odd n enters the even half alone).
template <typename T, int TMF, int TN, int EPI, int TKS>
__global__ __launch_bounds__(256, 2) void k_fold_left_fwd2(const T* __restrict__ FeT,
                                                           const T* __restrict__ FoT,
                                                           const T* __restrict__ B,
                                                           T* __restrict__ C, FoldAxis ax, int ncols,
                                                           int batch, long long bstride, EpiArgs ep) {
  using MF = Mfma<T>;
  constexpr int TK = TKS ? TKS : MF::TK / 2;
  constexpr int VE = 16 / sizeof(T);
  typedef T V __attribute__((ext_vector_type(VE)));
  constexpr int WM = TMF / 2, WN = TN / 2, BM = WM / 16, BN = WN / 16;
  constexpr int NA = (TK * TMF / VE + 255) / 256, NB = (TK * TN / VE + 255) / 256;
  __shared__ __attribute__((aligned(16))) T Ae[2][TK][TMF];
  __shared__ __attribute__((aligned(16))) T Ao[2][TK][TMF];
  __shared__ __attribute__((aligned(16))) T Bs[2][TK][TN];
  __shared__ __attribute__((aligned(16))) T Bd[2][TK][TN];

  const int bk = ax.bk, na = ax.n, h = ax.h;
  const int MT = bk / TMF, NT = ncols / TN;
  const int t = xcd_tile(blockIdx.x, batch * MT * NT);
  const int mt = t % MT, rest = t / MT, nt = rest % NT, b = rest / NT;
  const int inst = b % ep.inst_mod;
  if (ep.skip && ep.skip[inst]) return;
  const int i0 = mt * TMF, n0 = nt * TN;
  const T* Bb = B + (long long)b * bstride;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;

  typename MF::v4 acce[BM][BN], acco[BM][BN];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) acce[i][j] = acco[i][j] = typename MF::v4{0, 0, 0, 0};

  V rae[NA], rao[NA], rlo[NB], rhi[NB];
  int kpre = 0;
  auto gload = [&](int k0) {
    kpre = k0;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int v = tid + 256 * i;
      if (v < TK * TMF / VE) {
        const int kk = v / (TMF / VE), mm = (v % (TMF / VE)) * VE;
        rae[i] = *reinterpret_cast<const V*>(FeT + (long long)(k0 + kk) * bk + i0 + mm);
        rao[i] = *reinterpret_cast<const V*>(FoT + (long long)(k0 + kk) * bk + i0 + mm);
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int v = tid + 256 * i;
      if (v < TK * TN / VE) {
        const int kk = v / (TN / VE), nn = (v % (TN / VE)) * VE;
        const int k = k0 + kk;
        // rows k and n-1-k (the centre row pairs with itself); clamped for k > h
        const int kl = k <= h ? k : h, kh = k < h ? na - 1 - k : h;
        rlo[i] = *reinterpret_cast<const V*>(Bb + (long long)kl * ncols + n0 + nn);
        rhi[i] = *reinterpret_cast<const V*>(Bb + (long long)kh * ncols + n0 + nn);
      }
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int v = tid + 256 * i;
      if (v < TK * TMF / VE) {
        const int kk = v / (TMF / VE), mm = (v % (TMF / VE)) * VE;
        *reinterpret_cast<V*>(&Ae[buf][kk][mm]) = rae[i];
        *reinterpret_cast<V*>(&Ao[buf][kk][mm]) = rao[i];
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int v = tid + 256 * i;
      if (v < TK * TN / VE) {
        const int kk = v / (TN / VE), nn = (v % (TN / VE)) * VE;
        const int k = kpre + kk;
        V sum = V{}, dif = V{};
        if (k < h) {
          sum = rlo[i] + rhi[i];
          dif = rlo[i] - rhi[i];
        } else if (k == h && ax.odd) {
          sum = rlo[i];
        }
        *reinterpret_cast<V*>(&Bs[buf][kk][nn]) = sum;
        *reinterpret_cast<V*>(&Bd[buf][kk][nn]) = dif;
      }
    }
  };

  // Fold rows at or beyond ne = h + odd contribute nothing: stop the K loop there.
  const int kmax = ((h + ax.odd + TK - 1) / TK) * TK;
  const int nk = kmax / TK;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) gload((kc + 1) * TK);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      T ae[BM], ao[BM], bs[BN], bd[BN];
#pragma unroll
      for (int i = 0; i < BM; ++i) {
        ae[i] = Ae[buf][ks + (lane >> 4)][wm + 16 * i + (lane & 15)];
        ao[i] = Ao[buf][ks + (lane >> 4)][wm + 16 * i + (lane & 15)];
      }
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        bs[j] = Bs[buf][ks + (lane >> 4)][wn + 16 * j + (lane & 15)];
        bd[j] = Bd[buf][ks + (lane >> 4)][wn + 16 * j + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          acce[i][j] = MF::op(ae[i], bs[j], acce[i][j]);
          acco[i][j] = MF::op(ao[i], bd[j], acco[i][j]);
        }
    }
    if (kc + 1 < nk) lstore(buf ^ 1);
    __syncthreads();
  }

  T* Cb = C + (long long)b * bstride;
  double scale = 1.0, beta = 0.0, cn[BN];
  if (EPI == EPI_DIVIDE) {
    const double* cf = ep.coef + (long long)inst * ep.coef_stride;
    scale = cf[0] * (ep.cscale ? ep.cscale[b / ep.comp_div] : 1.0);
    beta = cf[1];
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      const int n = n0 + wn + 16 * j + (lane & 15);
      const int ny_ = n / ep.px;
      cn[j] = ep.lamX[n - ny_ * ep.px] + (ep.lamY ? ep.lamY[ny_] : 0.0);
    }
  }
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = i0 + wm + 16 * i + MF::row(lane, q);
      double le = 0.0, lo = 0.0;
      if (EPI == EPI_DIVIDE) {
        le = ep.lamM[m];
        lo = ep.lamM[bk + m];
      }
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (EPI == EPI_DIVIDE) {
          Cb[(long long)m * ncols + n] = divide_to<T>(acce[i][j][q], scale, le + cn[j], beta);
          Cb[(long long)(bk + m) * ncols + n] =
              divide_to<T>(acco[i][j][q], scale, lo + cn[j], beta);
        } else {
          Cb[(long long)m * ncols + n] = acce[i][j][q];
          Cb[(long long)(bk + m) * ncols + n] = acco[i][j][q];
        }
      }
    }
}

// Inverse, contraction over the split spectral rows, output spatial rows:
// p[k][c] = sum_{i<bk} Fe[i][k] Y[b][i][c], q[k][c] = sum_{i<bk} Fo[i][k] Y[b][bk+i][c];
// C[b][k] = p + q, C[b][n-1-k] = p - q (k < h), C[b][h] = p (n odd).
// A tile owns TMF fold rows (2 TMF output rows) x TN columns.
template <typename T, int TMF, int TN, int TKS>
__global__ __launch_bounds__(256, 2) void k_fold_left_inv(const T* __restrict__ Fe,
                                                          const T* __restrict__ Fo,
                                                          const T* __restrict__ Y,
                                                          T* __restrict__ C, FoldAxis ax, int ncols,
                                                          int batch, long long bstride, EpiArgs ep) {
  using MF = Mfma<T>;
  constexpr int TK = TKS ? TKS : MF::TK / 2;
  constexpr int VE = 16 / sizeof(T);
  typedef T V __attribute__((ext_vector_type(VE)));
  constexpr int WM = TMF / 2, WN = TN / 2, BM = WM / 16, BN = WN / 16;
  constexpr int NA = (TK * TMF / VE + 255) / 256, NB = (TK * TN / VE + 255) / 256;
  __shared__ __attribute__((aligned(16))) T Ap[2][TK][TMF];
  __shared__ __attribute__((aligned(16))) T Aq[2][TK][TMF];
  __shared__ __attribute__((aligned(16))) T Bp[2][TK][TN];
  __shared__ __attribute__((aligned(16))) T Bq[2][TK][TN];

  const int bk = ax.bk, na = ax.n, h = ax.h;
  const int MT = bk / TMF, NT = ncols / TN;
  const int t = xcd_tile(blockIdx.x, batch * MT * NT);
  const int mt = t % MT, rest = t / MT, nt = rest % NT, b = rest / NT;
  const int inst = b % ep.inst_mod;
  if (ep.skip && ep.skip[inst]) return;
  const int k0 = mt * TMF, n0 = nt * TN;
  if (k0 > h) return;  // only padding fold rows: nothing to write
  const T* Yb = Y + (long long)b * bstride;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;

  typename MF::v4 accp[BM][BN], accq[BM][BN];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) accp[i][j] = accq[i][j] = typename MF::v4{0, 0, 0, 0};

  V rap[NA], raq[NA], rbp[NB], rbq[NB];
  auto gload = [&](int i0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int v = tid + 256 * i;
      if (v < TK * TMF / VE) {
        const int ii = v / (TMF / VE), mm = (v % (TMF / VE)) * VE;
        rap[i] = *reinterpret_cast<const V*>(Fe + (long long)(i0 + ii) * bk + k0 + mm);
        raq[i] = *reinterpret_cast<const V*>(Fo + (long long)(i0 + ii) * bk + k0 + mm);
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int v = tid + 256 * i;
      if (v < TK * TN / VE) {
        const int ii = v / (TN / VE), nn = (v % (TN / VE)) * VE;
        rbp[i] = *reinterpret_cast<const V*>(Yb + (long long)(i0 + ii) * ncols + n0 + nn);
        rbq[i] = *reinterpret_cast<const V*>(Yb + (long long)(bk + i0 + ii) * ncols + n0 + nn);
      }
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int v = tid + 256 * i;
      if (v < TK * TMF / VE) {
        const int ii = v / (TMF / VE), mm = (v % (TMF / VE)) * VE;
        *reinterpret_cast<V*>(&Ap[buf][ii][mm]) = rap[i];
        *reinterpret_cast<V*>(&Aq[buf][ii][mm]) = raq[i];
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int v = tid + 256 * i;
      if (v < TK * TN / VE) {
        const int ii = v / (TN / VE), nn = (v % (TN / VE)) * VE;
        *reinterpret_cast<V*>(&Bp[buf][ii][nn]) = rbp[i];
        *reinterpret_cast<V*>(&Bq[buf][ii][nn]) = rbq[i];
      }
    }
  };

  // Spectral rows at or beyond ne (even) are exactly zero in both operands.
  const int imax = ((h + ax.odd + TK - 1) / TK) * TK;
  const int nk = imax / TK;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) gload((kc + 1) * TK);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      T ap[BM], aq[BM], bp[BN], bq[BN];
#pragma unroll
      for (int i = 0; i < BM; ++i) {
        ap[i] = Ap[buf][ks + (lane >> 4)][wm + 16 * i + (lane & 15)];
        aq[i] = Aq[buf][ks + (lane >> 4)][wm + 16 * i + (lane & 15)];
      }
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        bp[j] = Bp[buf][ks + (lane >> 4)][wn + 16 * j + (lane & 15)];
        bq[j] = Bq[buf][ks + (lane >> 4)][wn + 16 * j + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          accp[i][j] = MF::op(ap[i], bp[j], accp[i][j]);
          accq[i][j] = MF::op(aq[i], bq[j], accq[i][j]);
        }
    }
    if (kc + 1 < nk) lstore(buf ^ 1);
    __syncthreads();
  }

  T* Cb = C + (long long)b * bstride;
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + wm + 16 * i + MF::row(lane, q);
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        const int n = n0 + wn + 16 * j + (lane & 15);
        const T p = accp[i][j][q], qq = accq[i][j][q];
        if (k < h) {
          Cb[(long long)k * ncols + n] = p + qq;
          Cb[(long long)(na - 1 - k) * ncols + n] = p - qq;
        } else if (k == h && ax.odd) {
          Cb[(long long)k * ncols + n] = p;
        }
      }
    }
}

// ------------------------------------------------------------------ form R

// Forward along x (contraction over the columns of A's rows):
// C[r][m] = sum_{k<bk} fold_blk(A[r])[k] F^T_blk[k][i], blk = m / bk, i = m % bk.
template <typename T, int TM, int TN, int TKS>
__global__ __launch_bounds__(256, 2) void k_fold_right_fwd(const T* __restrict__ A,
                                                           const T* __restrict__ FeT,
                                                           const T* __restrict__ FoT,
                                                           T* __restrict__ C, FoldAxis ax, int rows,
                                                           EpiArgs ep) {
  using MF = Mfma<T>;
  constexpr int TK = TKS ? TKS : MF::TK;
  constexpr int VE = 16 / sizeof(T);
  typedef T V __attribute__((ext_vector_type(VE)));
  constexpr int WM = TM / 2, WN = TN / 2, BM = WM / 16, BN = WN / 16;
  constexpr int NA = (TK * TM / VE + 255) / 256, NB = (TK * TN / VE + 255) / 256;
  constexpr int RB = TK * (int)sizeof(T);  // bytes per A row (swizzled chunks)
  __shared__ __attribute__((aligned(16))) char As[2][TM * RB];
  __shared__ __attribute__((aligned(16))) T Bs[2][TK][TN];

  const int bk = ax.bk, P2 = 2 * bk, na = ax.n, h = ax.h;
  const int MT = rows / TM, NT = P2 / TN;
  const int t = xcd_tile(blockIdx.x, MT * NT);
  const int nt = t % NT, mt = t / NT;
  const int r0 = mt * TM, n0 = nt * TN;
  if (ep.skip && ep.skip[(r0 / ep.py / ep.pz) % ep.inst_mod]) return;
  const int blk = n0 / bk, i0 = n0 - blk * bk;
  const T* F = blk ? FoT : FeT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;

  typename MF::v4 acc[BM][BN];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) acc[i][j] = typename MF::v4{0, 0, 0, 0};

  // Raw pairs (row element k and its mirror n-1-k) are prefetched; the fold
  // happens at the LDS store so the loads overlap the MFMA phase.
  V rlo[NA], rhi[NA], rb[NB];
  int kpre = 0;
  auto gload = [&](int k0) {
    kpre = k0;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int v = tid + 256 * i;
      if (v < TM * TK / VE) {
        const int row = v / (TK / VE), kv = (v % (TK / VE)) * VE;
        const T* src = A + (long long)(r0 + row) * P2;
        rlo[i] = *reinterpret_cast<const V*>(src + k0 + kv);
#pragma unroll
        for (int e = 0; e < VE; ++e) {
          const int k = k0 + kv + e;
          rhi[i][e] = src[k < h ? na - 1 - k : 0];
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int v = tid + 256 * i;
      if (v < TK * TN / VE) {
        const int kk = v / (TN / VE), nn = (v % (TN / VE)) * VE;
        rb[i] = *reinterpret_cast<const V*>(F + (long long)(k0 + kk) * bk + i0 + nn);
      }
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int v = tid + 256 * i;
      if (v < TM * TK / VE) {
        const int row = v / (TK / VE), kv = (v % (TK / VE)) * VE;
        V val;
#pragma unroll
        for (int e = 0; e < VE; ++e) {
          const int k = kpre + kv + e;
          T x = 0;
          if (k < h)
            x = blk ? rlo[i][e] - rhi[i][e] : rlo[i][e] + rhi[i][e];
          else if (k == h && ax.odd && !blk)
            x = rlo[i][e];
          val[e] = x;
        }
        *reinterpret_cast<V*>(&As[buf][swz<RB>(row, kv * (int)sizeof(T))]) = val;
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int v = tid + 256 * i;
      if (v < TK * TN / VE) {
        const int kk = v / (TN / VE), nn = (v % (TN / VE)) * VE;
        *reinterpret_cast<V*>(&Bs[buf][kk][nn]) = rb[i];
      }
    }
  };

  const int kmax = ((h + ax.odd + TK - 1) / TK) * TK;
  const int nk = kmax / TK;
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
      for (int i = 0; i < BM; ++i)
        a[i] = *reinterpret_cast<const T*>(
            &As[buf][swz<RB>(wm + 16 * i + (lane & 15), (ks + (lane >> 4)) * (int)sizeof(T))]);
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
#pragma unroll
      for (int j = 0; j < BN; ++j)
        C[(long long)r * P2 + n0 + wn + 16 * j + (lane & 15)] = acc[i][j][q];
    }
}

// Inverse along x: p[r][k] = sum_i Y[r][i] Fe[i][k], q[r][k] = sum_i Y[r][bk+i] Fo[i][k];
// output columns k and n-1-k (p + q, p - q), or h (p).  EPI: store into C
// (row length 2 bk) or the dense epilogues (U -= dU / X = dU) on ep.dense.
template <typename T, int TM, int TNF, int EPI, int TKS>
__global__ __launch_bounds__(256, 2) void k_fold_right_inv(const T* __restrict__ Y,
                                                           const T* __restrict__ Fe,
                                                           const T* __restrict__ Fo,
                                                           T* __restrict__ C, FoldAxis ax, int rows,
                                                           EpiArgs ep) {
  using MF = Mfma<T>;
  constexpr int TK = TKS ? TKS : MF::TK / 2;
  constexpr int VE = 16 / sizeof(T);
  typedef T V __attribute__((ext_vector_type(VE)));
  constexpr int WM = TM / 2, WN = TNF / 2, BM = WM / 16, BN = WN / 16;
  constexpr int NA = (TM * TK / VE + 255) / 256, NB = (TK * TNF / VE + 255) / 256;
  constexpr int RB = TK * (int)sizeof(T);  // bytes per A row (swizzled chunks)
  __shared__ __attribute__((aligned(16))) char Ap[2][TM * RB];
  __shared__ __attribute__((aligned(16))) char Aq[2][TM * RB];
  __shared__ __attribute__((aligned(16))) T Bp[2][TK][TNF];
  __shared__ __attribute__((aligned(16))) T Bq[2][TK][TNF];

  const int bk = ax.bk, P2 = 2 * bk, na = ax.n, h = ax.h;
  const int MT = rows / TM, NT = bk / TNF;
  const int t = xcd_tile(blockIdx.x, MT * NT);
  const int nt = t % NT, mt = t / NT;
  const int r0 = mt * TM, k0 = nt * TNF;
  if (ep.skip && ep.skip[(r0 / ep.py / ep.pz) % ep.inst_mod]) return;
  if (k0 > h) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;

  typename MF::v4 accp[BM][BN], accq[BM][BN];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) accp[i][j] = accq[i][j] = typename MF::v4{0, 0, 0, 0};

  V rap[NA], raq[NA], rbp[NB], rbq[NB];
  auto gload = [&](int i0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int v = tid + 256 * i;
      if (v < TM * TK / VE) {
        const int row = v / (TK / VE), kv = (v % (TK / VE)) * VE;
        const T* src = Y + (long long)(r0 + row) * P2 + i0 + kv;
        rap[i] = *reinterpret_cast<const V*>(src);
        raq[i] = *reinterpret_cast<const V*>(src + bk);
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int v = tid + 256 * i;
      if (v < TK * TNF / VE) {
        const int ii = v / (TNF / VE), nn = (v % (TNF / VE)) * VE;
        rbp[i] = *reinterpret_cast<const V*>(Fe + (long long)(i0 + ii) * bk + k0 + nn);
        rbq[i] = *reinterpret_cast<const V*>(Fo + (long long)(i0 + ii) * bk + k0 + nn);
      }
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int v = tid + 256 * i;
      if (v < TM * TK / VE) {
        const int row = v / (TK / VE), kv = (v % (TK / VE)) * VE;
        *reinterpret_cast<V*>(&Ap[buf][swz<RB>(row, kv * (int)sizeof(T))]) = rap[i];
        *reinterpret_cast<V*>(&Aq[buf][swz<RB>(row, kv * (int)sizeof(T))]) = raq[i];
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int v = tid + 256 * i;
      if (v < TK * TNF / VE) {
        const int ii = v / (TNF / VE), nn = (v % (TNF / VE)) * VE;
        *reinterpret_cast<V*>(&Bp[buf][ii][nn]) = rbp[i];
        *reinterpret_cast<V*>(&Bq[buf][ii][nn]) = rbq[i];
      }
    }
  };

  const int imax = ((h + ax.odd + TK - 1) / TK) * TK;
  const int nk = imax / TK;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nk) gload((kc + 1) * TK);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      T ap[BM], aq[BM], bp[BN], bq[BN];
#pragma unroll
      for (int i = 0; i < BM; ++i) {
        const int off = swz<RB>(wm + 16 * i + (lane & 15), (ks + (lane >> 4)) * (int)sizeof(T));
        ap[i] = *reinterpret_cast<const T*>(&Ap[buf][off]);
        aq[i] = *reinterpret_cast<const T*>(&Aq[buf][off]);
      }
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        bp[j] = Bp[buf][ks + (lane >> 4)][wn + 16 * j + (lane & 15)];
        bq[j] = Bq[buf][ks + (lane >> 4)][wn + 16 * j + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          accp[i][j] = MF::op(ap[i], bp[j], accp[i][j]);
          accq[i][j] = MF::op(aq[i], bq[j], accq[i][j]);
        }
    }
    if (kc + 1 < nk) lstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < BM; ++i) {
    // Row bases of this fragment row block; for U -= dU every old value of the
    // block is loaded before the first store, so the loads overlap instead of
    // each waiting behind the previous store to the same array.
    long long base[4];
    bool row_ok[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = r0 + wm + 16 * i + MF::row(lane, q);
      base[q] = (long long)r * P2;
      row_ok[q] = true;
      if (EPI != EPI_STORE) {
        const int y = r % ep.py, zc = r / ep.py, z = zc % ep.pz, c = zc / ep.pz;
        base[q] = (((long long)c * ep.nz + z) * ep.ny + y) * ep.nx;
        row_ok[q] = y < ep.ny && z < ep.nz;
      }
    }
    double old1[4][BN], old2[4][BN];
    const double us = (EPI == EPI_SUB_DENSE && ep.uscale) ? *ep.uscale : 1.0;
    const double st = (EPI == EPI_SUB_DENSE && ep.step != 0.0) ? ep.step : 1.0;
    if (EPI == EPI_SUB_DENSE) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          const int k = k0 + wn + 16 * j + (lane & 15);
          const bool pair = k < h, centre = (k == h) && ax.odd;
          old1[q][j] = (row_ok[q] && (pair || centre)) ? ep.dense[base[q] + k] : 0.0;
          old2[q][j] = (row_ok[q] && pair) ? ep.dense[base[q] + na - 1 - k] : 0.0;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!row_ok[q]) continue;
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        const int k = k0 + wn + 16 * j + (lane & 15);
        const T p = accp[i][j][q], qq = accq[i][j][q];
        const bool pair = k < h, centre = (k == h) && ax.odd;
        if (!pair && !centre) continue;
        const T v1 = pair ? p + qq : p;
        if (EPI == EPI_STORE) {
          C[base[q] + k] = v1;
          if (pair) C[base[q] + na - 1 - k] = p - qq;
        } else if (EPI == EPI_SUB_DENSE) {
          ep.dense[base[q] + k] = us * old1[q][j] - st * (double)v1;
          if (pair) ep.dense[base[q] + na - 1 - k] = us * old2[q][j] - st * (double)(p - qq);
        } else {
          ep.dense[base[q] + k] = (double)v1;
          if (pair) ep.dense[base[q] + na - 1 - k] = (double)(p - qq);
        }
      }
    }
  }
}

// ------------------------------------------------------------------ dispatch

namespace {

// Stage depths of the deep tiles: one LDS stage spans 64 contraction rows in
// the forward kernels and 32 fold rows in the inverse and paired kernels
// (against 16 / 8 in FP64 and 32 / 16 in FP32 otherwise), so a short
// contraction (small grids) waits on two to four global-load round trips
// instead of eight to sixteen.  (On large grids deeper stages of the 64-wide
// tiles measured no faster than the defaults.)
constexpr int kDeepFwd = 64, kDeepInv = 32;

template <typename T>
hipError_t lfwd(const FoldOperands& f, const T* B, T* C, const FoldAxis& ax, int ncols, int batch,
                long long bstride, int epi, const EpiArgs& ep, const FoldTile& t, hipStream_t st) {
  const T* FeT = (const T*)f.FeT;
  const T* FoT = (const T*)f.FoT;
#define QN_LFWD(TM_, TN_, TK_)                                                                  \
  if (t.tm == TM_ && t.tn == TN_ && t.tk == TK_) {                                              \
    const unsigned g = (unsigned)((long long)batch * (2 * ax.bk / TM_) * (ncols / TN_));        \
    if (epi == EPI_DIVIDE)                                                                      \
      hipLaunchKernelGGL((k_fold_left_fwd<T, TM_, TN_, EPI_DIVIDE, TK_>), dim3(g), dim3(256), 0, \
                         st, FeT, FoT, B, C, ax, ncols, batch, bstride, ep);                    \
    else                                                                                        \
      hipLaunchKernelGGL((k_fold_left_fwd<T, TM_, TN_, EPI_STORE, TK_>), dim3(g), dim3(256), 0, \
                         st, FeT, FoT, B, C, ax, ncols, batch, bstride, ep);                    \
    return hipGetLastError();                                                                   \
  }
  QN_LFWD(128, 128, 0)
  QN_LFWD(64, 128, 0)
  QN_LFWD(64, 64, 0)
  QN_LFWD(32, 64, 0)
  QN_LFWD(32, 32, 0)
  QN_LFWD(32, 32, kDeepFwd)
#undef QN_LFWD
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t lfwd2(const FoldOperands& f, const T* B, T* C, const FoldAxis& ax, int ncols, int batch,
                 long long bstride, int epi, const EpiArgs& ep, const FoldTile& t, hipStream_t st) {
  const T* FeT = (const T*)f.FeT;
  const T* FoT = (const T*)f.FoT;
#define QN_LFWD2(TM_, TN_, TK_)                                                                  \
  if (t.tm == TM_ && t.tn == TN_ && t.tk == TK_) {                                               \
    const unsigned g = (unsigned)((long long)batch * (ax.bk / TM_) * (ncols / TN_));             \
    if (epi == EPI_DIVIDE)                                                                       \
      hipLaunchKernelGGL((k_fold_left_fwd2<T, TM_, TN_, EPI_DIVIDE, TK_>), dim3(g), dim3(256), 0, \
                         st, FeT, FoT, B, C, ax, ncols, batch, bstride, ep);                     \
    else                                                                                         \
      hipLaunchKernelGGL((k_fold_left_fwd2<T, TM_, TN_, EPI_STORE, TK_>), dim3(g), dim3(256), 0, \
                         st, FeT, FoT, B, C, ax, ncols, batch, bstride, ep);                     \
    return hipGetLastError();                                                                    \
  }
  QN_LFWD2(64, 64, 0)
  QN_LFWD2(128, 64, 0)
  QN_LFWD2(32, 64, 0)
  QN_LFWD2(64, 128, 0)
  QN_LFWD2(32, 128, 0)
  QN_LFWD2(32, 32, kDeepInv)
#undef QN_LFWD2
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t linv(const FoldOperands& f, const T* Y, T* C, const FoldAxis& ax, int ncols, int batch,
                long long bstride, const EpiArgs& ep, const FoldTile& t, hipStream_t st) {
  const T* Fe = (const T*)f.Fe;
  const T* Fo = (const T*)f.Fo;
#define QN_LINV(TM_, TN_, TK_)                                                                  \
  if (t.tm == TM_ && t.tn == TN_ && t.tk == TK_) {                                              \
    const unsigned g = (unsigned)((long long)batch * (ax.bk / TM_) * (ncols / TN_));            \
    hipLaunchKernelGGL((k_fold_left_inv<T, TM_, TN_, TK_>), dim3(g), dim3(256), 0, st, Fe, Fo, \
                       Y, C, ax, ncols, batch, bstride, ep);                                    \
    return hipGetLastError();                                                                   \
  }
  QN_LINV(64, 128, 0)
  QN_LINV(64, 64, 0)
  QN_LINV(32, 64, 0)
  QN_LINV(32, 32, 0)
  QN_LINV(32, 128, 0)
  QN_LINV(32, 32, kDeepInv)
  QN_LINV(32, 64, kDeepInv)
#undef QN_LINV
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t rfwd(const FoldOperands& f, const T* A, T* C, const FoldAxis& ax, int rows,
                const EpiArgs& ep, const FoldTile& t, hipStream_t st) {
  const T* FeT = (const T*)f.FeT;
  const T* FoT = (const T*)f.FoT;
#define QN_RFWD(TM_, TN_, TK_)                                                                   \
  if (t.tm == TM_ && t.tn == TN_ && t.tk == TK_) {                                               \
    const unsigned g = (unsigned)((long long)(rows / TM_) * (2 * ax.bk / TN_));                  \
    hipLaunchKernelGGL((k_fold_right_fwd<T, TM_, TN_, TK_>), dim3(g), dim3(256), 0, st, A, FeT, \
                       FoT, C, ax, rows, ep);                                                    \
    return hipGetLastError();                                                                    \
  }
  QN_RFWD(128, 128, 0)
  QN_RFWD(128, 64, 0)
  QN_RFWD(64, 64, 0)
  QN_RFWD(64, 32, 0)
  QN_RFWD(32, 32, 0)
  QN_RFWD(64, 128, 0)
  QN_RFWD(32, 64, 0)
  QN_RFWD(32, 32, kDeepFwd)
#undef QN_RFWD
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t rinv(const FoldOperands& f, const T* Y, T* C, const FoldAxis& ax, int rows, int epi,
                const EpiArgs& ep, const FoldTile& t, hipStream_t st) {
  const T* Fe = (const T*)f.Fe;
  const T* Fo = (const T*)f.Fo;
#define QN_RINV(TM_, TN_, TK_)                                                                   \
  if (t.tm == TM_ && t.tn == TN_ && t.tk == TK_) {                                               \
    const unsigned g = (unsigned)((long long)(rows / TM_) * (ax.bk / TN_));                      \
    if (epi == EPI_SUB_DENSE)                                                                    \
      hipLaunchKernelGGL((k_fold_right_inv<T, TM_, TN_, EPI_SUB_DENSE, TK_>), dim3(g), dim3(256), \
                         0, st, Y, Fe, Fo, C, ax, rows, ep);                                     \
    else if (epi == EPI_STORE_DENSE)                                                             \
      hipLaunchKernelGGL((k_fold_right_inv<T, TM_, TN_, EPI_STORE_DENSE, TK_>), dim3(g),         \
                         dim3(256), 0, st, Y, Fe, Fo, C, ax, rows, ep);                          \
    else                                                                                         \
      hipLaunchKernelGGL((k_fold_right_inv<T, TM_, TN_, EPI_STORE, TK_>), dim3(g), dim3(256), 0, \
                         st, Y, Fe, Fo, C, ax, rows, ep);                                        \
    return hipGetLastError();                                                                    \
  }
  QN_RINV(128, 64, 0)
  QN_RINV(64, 64, 0)
  QN_RINV(64, 32, 0)
  QN_RINV(32, 32, 0)
  QN_RINV(64, 128, 0)
  QN_RINV(32, 64, 0)
  QN_RINV(32, 32, kDeepInv)
  QN_RINV(64, 32, kDeepInv)
#undef QN_RINV
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t fold_typed(int kind, const FoldOperands& f, const void* in, void* out,
                      const FoldAxis& ax, int ncols, int batch, long long bstride, int rows,
                      int epi, const EpiArgs& ep, const FoldTile& t, hipStream_t st) {
  const T* src = (const T*)in;
  T* dst = (T*)out;
  switch (kind) {
    case FK_RFWD: return rfwd<T>(f, src, dst, ax, rows, ep, t, st);
    case FK_LFWD:
      if (t.paired) return lfwd2<T>(f, src, dst, ax, ncols, batch, bstride, epi, ep, t, st);
      return lfwd<T>(f, src, dst, ax, ncols, batch, bstride, epi, ep, t, st);
    case FK_LINV: return linv<T>(f, src, dst, ax, ncols, batch, bstride, ep, t, st);
    default: return rinv<T>(f, src, dst, ax, rows, epi, ep, t, st);
  }
}

// Instantiated shapes in order of preference.  The deep variants come right
// before the plain 32-wide shapes of the same extents, so the default rule
// (most workgroups when no shape fills the chip) prefers them on small grids.
const FoldTile kTilesRfwd[] = {{128, 128, 0, 0}, {128, 64, 0, 0},       {64, 128, 0, 0},
                               {64, 64, 0, 0},   {64, 32, 0, 0},        {32, 64, 0, 0},
                               {32, 32, 0, kDeepFwd}, {32, 32, 0, 0}};
const FoldTile kTilesLfwd[] = {{64, 64, 1, 0},  {128, 128, 0, 0},      {64, 128, 0, 0},
                               {128, 64, 1, 0}, {64, 128, 1, 0},       {32, 128, 1, 0},
                               {64, 64, 0, 0},  {32, 64, 1, 0},        {32, 64, 0, 0},
                               {32, 32, 1, kDeepInv}, {32, 32, 0, kDeepFwd}, {32, 32, 0, 0}};
const FoldTile kTilesLinv[] = {{64, 64, 0, 0},        {64, 128, 0, 0}, {32, 128, 0, 0},
                               {32, 64, 0, kDeepInv}, {32, 64, 0, 0},  {32, 32, 0, kDeepInv},
                               {32, 32, 0, 0}};
const FoldTile kTilesRinv[] = {{64, 64, 0, 0},        {128, 64, 0, 0}, {64, 128, 0, 0},
                               {64, 32, 0, kDeepInv}, {64, 32, 0, 0}, {32, 64, 0, 0},
                               {32, 32, 0, kDeepInv}, {32, 32, 0, 0}};
}  // namespace

int fold_tiles(int kind, const FoldTile** list) {
  switch (kind) {
    case FK_RFWD: *list = kTilesRfwd; return (int)(sizeof kTilesRfwd / sizeof kTilesRfwd[0]);
    case FK_LFWD: *list = kTilesLfwd; return (int)(sizeof kTilesLfwd / sizeof kTilesLfwd[0]);
    case FK_LINV: *list = kTilesLinv; return (int)(sizeof kTilesLinv / sizeof kTilesLinv[0]);
    default: *list = kTilesRinv; return (int)(sizeof kTilesRinv / sizeof kTilesRinv[0]);
  }
}

void fold_extents(int kind, int bk, int ncols, int rows, long long* mext, long long* next) {
  if (kind == FK_RFWD || kind == FK_RINV) {
    *mext = rows;
    *next = bk;
  } else {
    *mext = bk;
    *next = ncols;
  }
}

bool fold_tile_fits(int kind, const FoldTile& t, int bk, int ncols, int rows) {
  long long mext, next;
  fold_extents(kind, bk, ncols, rows, &mext, &next);
  // a deep stage may not run past the bk spectral rows of the fold matrices
  return mext % t.tm == 0 && next % t.tn == 0 && (t.tk == 0 || bk % t.tk == 0);
}

long long fold_blocks(int kind, const FoldTile& t, int bk, int ncols, int batch, int rows) {
  long long mext, next;
  fold_extents(kind, bk, ncols, rows, &mext, &next);
  // split forward kernels launch the even and odd halves as separate tiles
  const long long halves = ((kind == FK_RFWD || kind == FK_LFWD) && !t.paired) ? 2 : 1;
  const long long nb = (kind == FK_RFWD || kind == FK_RINV) ? 1 : batch;
  return halves * nb * (mext / t.tm) * (next / t.tn);
}

hipError_t launch_fold(int kind, int prec, const FoldOperands& f, const void* in, void* out,
                       const FoldAxis& ax, int ncols, int batch, long long bstride, int rows,
                       int epi, const EpiArgs& ep, const FoldTile& t, hipStream_t st) {
  if (prec == 0)
    return fold_typed<double>(kind, f, in, out, ax, ncols, batch, bstride, rows, epi, ep, t, st);
  return fold_typed<float>(kind, f, in, out, ax, ncols, batch, bstride, rows, epi, ep, t, st);
}

}  // namespace qn
