// Split-bf16 mode products of the tensor-product solve (Section 4.1,
// eq. fin_inverse) on the bf16 matrix cores, with the spectral divide and the
// quasi-Newton update fused into the epilogues.  The FP64 and FP32 forms use
// the reflection-folded kernels of qn_gemm_fold.hip.
//
// Every FP32 operand x is split into NP bf16 parts, x ~ x0 + x1 (+ x2),
// x0 = RNE(x), x1 = RNE(x - x0), x2 = RNE(x - x0 - x1), and a product keeps
// the part products x_i y_j with i + j < NP, accumulated in FP32 from the
// smallest terms up:
//   NP = 2 ("bf16x3"): x1 y0 + x0 y1 + x0 y0          (dropped: 2^-16 relative)
//   NP = 3 ("bf16x6"): x2 y0 + x0 y2 + x1 y1 + x1 y0 + x0 y1 + x0 y0
//                                                      (dropped: 2^-24 relative)
// The 1D eigenvector matrix S is split once at setup.  bf16x3 keeps every
// tensor between products as its two part planes (written by the residual,
// the pad copy and each product's epilogue), so both operands travel from
// global memory straight into LDS; bf16x6 keeps FP32 tensors and splits the
// tensor operand while staging it through registers.
//
// Two forms cover the three axes of a C-order (.., z, y, x) tensor:
//   form L  C[b][m][n] = sum_k S[m][k] B[b][k][n]   (y and z products; B rows
//           are contiguous in n, b runs over the batch of slabs)
//   form R  C[r][n]    = sum_k A[r][k] S[k][n]      (x product; A rows are the
//           x-lines of the tensor, contiguous in k)
// S is P x P (P = padded axis length, a multiple of 32), symmetric and zero
// outside the N x N block, so padded rows and columns stay exactly zero.
//
// bf16x3 inverse products run folded: the eigenvectors are symmetric or
// antisymmetric about the grid centre by mode parity, S[n-1-j][k] =
// (-1)^k S[j][k], so one tile computes output j (< ceil(n/2)) from the sums
// over the even modes (p) and the odd modes (q), taken by masking each
// fragment's 8 consecutive modes to its even or odd entries, and writes
// x[j] = p + q and x[n-1-j] = p - q: half the workgroups, each with twice the
// matrix-core work per staged chunk for the same loads.
//
// 3D bf16x3 solves whose y and z axes allow it (2 hp = P, hp = ceil(n / 2)
// rounded up to 32) also fold the forward y and z products, which contract
// over the spatial index: the producer of each one's input writes it folded
// along that axis, and the product takes the even modes from the sums and
// the odd modes from the differences:
//   - the x product writes its output folded along z: plane z < hp holds
//     X[z] + X[nz-1-z] and plane hp + z holds X[z] - X[nz-1-z] (the middle
//     plane of odd nz once, its difference zero; planes from ceil(nz / 2) to
//     hp zero), pairing the two planes' rows inside one tile;
//   - a forward product over a folded input contracts hp rows for each mode,
//     the sums for the even modes and the differences for the odd ones (S:
//     the even modes' rows, then the odd modes', hp columns): half the loads
//     and matrix-core work of the dense product, output in mode order; the z
//     product writes its output folded along y in the same way (pairing the
//     columns of rows y and ny-1-y in one tile);
//   - quasi-linear and 2-component problems whose residual tiles cover whole
//     rows also fold the x product: the residual (or the copy of a caller's
//     right-hand side) writes its output folded along x, and the x product
//     contracts half a row per mode (ZF = 2 below).
//
// Work decomposition: a 256-thread workgroup (four wave64s in a 2 x 2 grid)
// owns a TM x TN output tile and walks K in chunks of 32 (one matrix-core
// step), double-buffered in LDS with one barrier per chunk (the next chunk's
// direct-to-LDS loads, or global loads into registers, are issued before the
// current chunk's matrix-core work).
// v_mfma_f32_16x16x32_bf16 takes, per lane, 8 consecutive k values of one row
// of A (row = lane % 16, k = 8 * (lane / 16) ..) and of one column of B;
// the S parts and the x-product data are staged k-contiguous, [row][k], and
// the y/z-product data keeps its [k][n] layout and is read k-wise with the
// transposing LDS load; both layouts are XOR-swizzled (kswz, tswz).  Each XCD
// (workgroups are dealt round-robin) walks a contiguous range of tiles, so
// operand panels are reused in its L2.

#include "qn_internal.h"
#include "qn_mfma.h"

namespace qn {

namespace {

typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef unsigned u4v_t __attribute__((ext_vector_type(4)));

// A fragment's 8 consecutive modes k0 + 8 g + e (k0 + 8 g even) kept at the
// even modes (e even: the low half of each 32-bit word) or at the odd ones.
__device__ __forceinline__ bf8_t even_modes(bf8_t v) {
  return __builtin_bit_cast(bf8_t, __builtin_bit_cast(u4v_t, v) & 0x0000FFFFu);
}
__device__ __forceinline__ bf8_t odd_modes(bf8_t v) {
  return __builtin_bit_cast(bf8_t, __builtin_bit_cast(u4v_t, v) & 0xFFFF0000u);
}

constexpr int BTK = 32;  // k per chunk = one matrix-core step
constexpr int RBK = BTK * 2;  // bytes of the 32 k values of one row of a part

// LDS tiles of rows with 32 k values ([row][k]: the S parts, and the
// x-product data; 64 bytes per row and part): the four 16-byte chunks of a
// row are XOR-permuted by the row's index within its 256-byte bank line, so
// the row-wise staging stores and the fragment reads (chunk c of 16
// consecutive rows) spread over all 16 chunks of a bank line.  (A
// chunk-major layout, whose fragment reads are free of bank conflicts, was
// measured slower: its staging threads, mapped row-fastest, lose the
// coalescing of the global loads.)
__device__ __forceinline__ int kswz(int row, int col_bytes) {
  return row * RBK + ((((col_bytes >> 4) ^ ((row >> 2) & 3)) << 4) | (col_bytes & 15));
}

// The y/z products' data tile stays in its global layout, [k][n] with n
// contiguous (TN bf16 per k-row), and the MFMA B fragments (8 consecutive k of
// one column n per lane) are read with the transposing LDS load: in each group
// of 16 lanes, lane 4a + e receives element e of the 8-byte words of lanes
// a, a + 4, a + 8, a + 12.  Lane i of group g therefore addresses row
// 8 g + 4 h + i / 4, columns n0 + 4 (i % 4) .. + 3 (h = 0, 1: k 0-3 and 4-7 of
// the group).  Its 32-byte segments are XOR-permuted per row so that the
// four rows of a group, and the rows of the group read in the same cycle,
// fall on distinct banks.
template <int TN>
__device__ __forceinline__ int tperm(int k) {
  constexpr int RB = TN * 2;  // bytes per k-row
  if constexpr (RB >= 256)
    return (k & 3) | (((k >> 3) & 1) << 2);
  else if constexpr (RB == 128)
    return ((k >> 1) & 1) | (((k >> 3) & 1) << 1);
  else
    return (k >> 3) & 1;
}
template <int TN>
__device__ __forceinline__ int tswz(int k, int col_bytes) {
  return k * TN * 2 + ((((col_bytes >> 5) ^ tperm<TN>(k)) << 5) | (col_bytes & 31));
}

// bf16x3 keeps every intermediate tensor of the solve as its two bf16 parts,
// hi = RNE(x) and lo = RNE(x - hi) of the FP32 value x, in two planes (hi at
// the tensor's base, lo one tensor size further): the parts a kernel would
// split from x, so the results are the same bits, while the products load
// both operands straight into LDS (global_load_lds: a wave fills 1 KiB of LDS
// per instruction, lane p the 16 bytes at p * 16, from a global address the
// lane chooses, so the lanes gather the swizzled layout) with no register
// staging and no split on the load path.
typedef __attribute__((address_space(3))) void lds_void;
__device__ __forceinline__ void put_pair(__bf16* hi, long long plane, long long idx, float v) {
  const __bf16 h = (__bf16)v;
  hi[idx] = h;
  hi[plane + idx] = (__bf16)(v - (float)h);
}
// One KiB block of a [row][k] tile (16 rows of 32 k): lane p fetches row
// row0 + p / 4, the logical chunk that the XOR permutation puts at slot p % 4.
__device__ __forceinline__ void dload_rows(const __bf16* src, long long ld, int row0, int k0, int lane,
                                           char* dst) {
  const int row = lane >> 2, c = (lane & 3) ^ (((row0 + row) >> 2) & 3);
  __builtin_amdgcn_global_load_lds(src + (long long)(row0 + row) * ld + k0 + 8 * c, (lds_void*)dst,
                                   16, 0, 0);
}

typedef short s4v_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ bf4_t lds_tr4(const char* base, int off) {
  const s4v_t v = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
      (__attribute__((address_space(3))) s4v_t*)(base + off));
  return __builtin_bit_cast(bf4_t, v);
}

template <int NP>
__device__ inline void split(float x, __bf16 (&p)[NP]) {
  p[0] = (__bf16)x;
  const float r = x - (float)p[0];
  p[1] = (__bf16)r;
  if constexpr (NP > 2) p[2] = (__bf16)(r - (float)p[1]);
}

// sum over part pairs i + j < NP, smallest terms first
template <int NP>
__device__ inline f4_t mfma_split(const bf8_t (&a)[NP], const bf8_t (&b)[NP], f4_t c) {
  if constexpr (NP == 3) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1], c, 0, 0, 0);
  }
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], c, 0, 0, 0);
  return c;
}

__device__ inline const __bf16* part(const GemmOperands& s, int i) {
  return (const __bf16*)(i == 0 ? s.Shi : i == 1 ? s.Slo : s.Slo2);
}

}  // namespace

// FWD (bf16x3, the 3D path with folded forward products; K = hp, M = 2 hp):
//   1  forward product from a folded input: tile rows t < hp contract the
//      mirror sums (B rows [0, hp)) into even mode 2 t, rows hp + t the
//      differences (B rows [hp, 2 hp)) into odd mode 2 t + 1 (S: the modes'
//      rows of S in that order, hp columns); output rows in mode order
//   2  the same, the output written folded along y (the z product: columns
//      y * px + x, hpo = the folded y layout's half extent)
// K is the contraction length and the leading dimension of S (M otherwise).
template <int NP, int TM, int TN, int EPI, bool FOLD = false, int FWD = 0>
__global__ __launch_bounds__(256, 2) void k_gemm_left_bf(GemmOperands S, const void* __restrict__ Bv,
                                                         void* __restrict__ Cv, int M, int K,
                                                         int ncols, int batch, long long bstride,
                                                         EpiArgs ep, int mh, int nmir, int hpo) {
  // NP = 2: B and C are bf16 part planes; NP = 3: FP32 tensors
  constexpr bool PS = NP == 2;
  constexpr bool FF = FWD >= 1, YF = FWD == 2;
  static_assert(!FOLD || (NP == 2 && EPI == EPI_STORE), "folded: the bf16x3 inverse products");
  static_assert(FWD == 0 || (NP == 2 && !FOLD), "folded forward: bf16x3 forward products");
  static_assert(!YF || (EPI == EPI_STORE && TN >= 64), "y-folded output: plain store, paired column halves");
  const float* B = (const float*)Bv;
  float* C = (float*)Cv;
  const long long plane = (long long)batch * bstride;
  constexpr int WM = TM / 2, WN = TN / 2, BM = WM / 16, BN = WN / 16;
  constexpr int NAV = TM * (BTK / 8);        // 16-byte vectors per S part
  constexpr int NBV = BTK * (TN / 4);        // float4 runs (4 consecutive n) of the tensor chunk
  constexpr int PA = (NAV + 255) / 256, PB = (NBV + 255) / 256;
  __shared__ __attribute__((aligned(16))) char As[NP][2][TM * RBK];
  __shared__ __attribute__((aligned(16))) char Bs[NP][2][BTK * TN * 2];

  // FOLD: output rows m < mh only (mh: ceil(nmir / 2) rounded up to TM), each
  // giving rows m and nmir - 1 - m.  YF: column tiles of TN / 2 x values at
  // rows y < hpo and ny-1-y.
  const int MT = (FOLD ? mh : M) / TM, NT = YF ? hpo * (ep.px / (TN / 2)) : ncols / TN;
  const int t = xcd_tile(blockIdx.x, batch * MT * NT);
  const int mt = t % MT, rest = t / MT, nt = rest % NT, b = rest / NT;
  const int inst = b % ep.inst_mod;
  if (ep.skip && ep.skip[inst]) return;  // whole workgroup: finished instance
  const int m0 = mt * TM, n0 = nt * TN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
  // FF: this tile's parity half of the folded input (all its rows have one
  // parity: TM divides K); YF: its row pair and x range
  const int krow0 = FF && m0 >= K ? K : 0;
  auto orow = [&](int m) { return FF ? 2 * (m - krow0) + (krow0 ? 1 : 0) : m; };  // output row
  int yf = 0, ybar = 0, x0 = 0;
  if constexpr (YF) {
    const int xt = ep.px / (TN / 2);
    yf = nt / xt;
    x0 = (nt % xt) * (TN / 2);
    ybar = max(ep.ny - 1 - yf, 0);
  }
  // global column of the tile's logical column l (a multiple of 8): YF puts
  // the x values of row y in the first half of each wave's WN columns and
  // those of row ny-1-y in the second, so a lane holds both of a pair
  auto bcol = [&](int l) -> long long {
    if constexpr (YF) {
      const int wh = l / WN, r = l % WN, mir = r >= WN / 2;
      return (long long)(mir ? ybar : yf) * ep.px + x0 + wh * (WN / 2) + r - (mir ? WN / 2 : 0);
    } else {
      return n0 + l;
    }
  };

  f4_t acc[BM][BN], accq[BM][BN];  // accq: the odd modes' sums (FOLD)
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) acc[i][j] = accq[i][j] = f4_t{0, 0, 0, 0};

  const int g = lane >> 4, li = lane & 15;
  // all matrix-core fragments of chunk buf: a[i][part], bj[j][part]
  auto read_frags = [&](int buf, bf8_t (&a)[BM][NP], bf8_t (&bj)[BN][NP]) {
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int q = 0; q < NP; ++q)
        a[i][q] = *reinterpret_cast<const bf8_t*>(&As[q][buf][kswz(wm + 16 * i + li, 16 * g)]);
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      const int ncol = wn + 16 * j + 4 * (li & 3);
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const bf4_t lo4 = lds_tr4(&Bs[q][buf][0], tswz<TN>(8 * g + (li >> 2), 2 * ncol));
        const bf4_t hi4 = lds_tr4(&Bs[q][buf][0], tswz<TN>(8 * g + 4 + (li >> 2), 2 * ncol));
        bj[j][q] = bf8_t{lo4[0], lo4[1], lo4[2], lo4[3], hi4[0], hi4[1], hi4[2], hi4[3]};
      }
    }
  };
  auto mma = [&](const bf8_t (&a)[BM][NP], const bf8_t (&bj)[BN][NP]) {
    if constexpr (FOLD) {
      // S[n-1-m][k] = (-1)^k S[m][k]: the even and odd modes' sums of row m
      // give rows m (p + q) and n-1-m (p - q)
#pragma unroll
      for (int i = 0; i < BM; ++i) {
        bf8_t ae[NP], ao[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          ae[q] = even_modes(a[i][q]);
          ao[q] = odd_modes(a[i][q]);
        }
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          acc[i][j] = mfma_split<NP>(ae, bj[j], acc[i][j]);
          accq[i][j] = mfma_split<NP>(ao, bj[j], accq[i][j]);
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < BN; ++j)
#pragma unroll
        for (int i = 0; i < BM; ++i) acc[i][j] = mfma_split<NP>(a[i], bj[j], acc[i][j]);
    }
  };
  const int nk = K / BTK;
  if constexpr (PS) {
    const __bf16* Bh = (const __bf16*)Bv + (long long)b * bstride;
    // chunk k0 into LDS buffer buf: the S parts' rows (TM / 16 KiB blocks per
    // part) and the data's k-rows (TN / 16 blocks per part, 512 / TN rows each)
    auto dload = [&](int k0, int buf) {
#pragma unroll
      for (int blk = wave; blk < TM / 16; blk += 4)
#pragma unroll
        for (int q = 0; q < NP; ++q) dload_rows(part(S, q), K, m0 + 16 * blk, k0, lane, &As[q][buf][blk * 1024]);
      constexpr int RPB = 512 / TN, SPR = TN / 8;  // rows per block, 16-byte slots per row
#pragma unroll
      for (int blk = wave; blk < BTK / RPB; blk += 4) {
        const int row = RPB * blk + lane / SPR, slot = lane % SPR;
        const int seg = (slot >> 1) ^ tperm<TN>(row);
        const long long off = (long long)(krow0 + k0 + row) * ncols + bcol(16 * seg + 8 * (slot & 1));
#pragma unroll
        for (int q = 0; q < NP; ++q)
          __builtin_amdgcn_global_load_lds(Bh + q * plane + off, (lds_void*)&Bs[q][buf][blk * 1024], 16, 0, 0);
      }
    };
    dload(0, 0);
    for (int kc = 0; kc < nk; ++kc) {
      const int buf = kc & 1;
      // this chunk's loads have landed and every wave is done reading the
      // buffer the next chunk overwrites
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      // fragments first: the compiler makes LDS reads wait for every
      // direct-to-LDS load in flight, so the next chunk's loads are issued
      // after them and overlap the matrix-core work
      bf8_t a[BM][NP], bj[BN][NP];
      read_frags(buf, a, bj);
      if (kc + 1 < nk) dload((kc + 1) * BTK, buf ^ 1);
      mma(a, bj);
    }
  } else {
    const float* Bb = B + (long long)b * bstride;
    bf8_t ra[NP][PA];
    f4_t rb[PB];
    auto gload = [&](int k0) {
#pragma unroll
      for (int p = 0; p < PA; ++p) {
        const int v = tid + 256 * p;
        if (v < NAV) {
          const int m = v / (BTK / 8), kv = (v % (BTK / 8)) * 8;
          // S[m][k] with S symmetric: row m, 8 consecutive k.
          const long long off = (long long)(m0 + m) * K + k0 + kv;
#pragma unroll
          for (int q = 0; q < NP; ++q) ra[q][p] = *reinterpret_cast<const bf8_t*>(part(S, q) + off);
        }
      }
#pragma unroll
      for (int p = 0; p < PB; ++p) {
        const int v = tid + 256 * p;
        if (v < NBV) {
          const int k = v / (TN / 4), nq = (v % (TN / 4)) * 4;
          rb[p] = *reinterpret_cast<const f4_t*>(Bb + (long long)(k0 + k) * ncols + n0 + nq);
        }
      }
    };
    auto lstore = [&](int buf) {
#pragma unroll
      for (int p = 0; p < PA; ++p) {
        const int v = tid + 256 * p;
        if (v < NAV) {
          const int m = v / (BTK / 8), kv = (v % (BTK / 8)) * 8;
#pragma unroll
          for (int q = 0; q < NP; ++q)
            *reinterpret_cast<bf8_t*>(&As[q][buf][kswz(m, 2 * kv)]) = ra[q][p];
        }
      }
#pragma unroll
      for (int p = 0; p < PB; ++p) {
        const int v = tid + 256 * p;
        if (v < NBV) {
          const int k = v / (TN / 4), nq = (v % (TN / 4)) * 4;
          bf4_t w[NP];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            __bf16 x[NP];
            split<NP>(rb[p][e], x);
#pragma unroll
            for (int q = 0; q < NP; ++q) w[q][e] = x[q];
          }
#pragma unroll
          for (int q = 0; q < NP; ++q)
            *reinterpret_cast<bf4_t*>(&Bs[q][buf][tswz<TN>(k, 2 * nq)]) = w[q];
        }
      }
    };

    gload(0);
    lstore(0);
    __syncthreads();
    for (int kc = 0; kc < nk; ++kc) {
      const int buf = kc & 1;
      if (kc + 1 < nk) gload((kc + 1) * BTK);
      {
        bf8_t a[BM][NP], bj[BN][NP];
        read_frags(buf, a, bj);
        mma(a, bj);
      }
      if (kc + 1 < nk) lstore(buf ^ 1);
      __syncthreads();
    }
  }

  const long long cbase = (long long)b * bstride;
  auto put = [&](long long idx, float v) {
    if constexpr (PS)
      put_pair((__bf16*)Cv, plane, cbase + idx, v);
    else
      C[cbase + idx] = v;
  };
  if (EPI == EPI_DIVIDE) {
    // denominator scale (lam_m + lam_x + lam_y) + beta: the column part once
    // per column block, the row part once per row, one divide per entry
    const double* cf = ep.coef + (long long)inst * ep.coef_stride;
    const double scale = cf[0], beta = cf[1];
    double cn[BN];
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      const int n = n0 + wn + 16 * j + (lane & 15);
      const int ny_ = n / ep.px;
      cn[j] = ep.lamX[n - ny_ * ep.px] + (ep.lamY ? ep.lamY[ny_] : 0.0);
    }
    // bf16x3 rounds the quotient to FP32 and keeps it as two bf16 parts (a
    // 2^-16 relative split): the denominator and the quotient in FP32 lose
    // nothing at that precision and cost half the FP64 operations
    const float sf = (float)scale, bf = (float)beta;
    const double lb = ep.lamB ? ep.lamB[b % ep.pz] : 0.0;  // slab's own mode (z)
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = orow(m0 + wm + 16 * i + 4 * (lane >> 4) + q);
        const double lm = ep.lamM[m] + lb;
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          const int n = n0 + wn + 16 * j + (lane & 15);
          if constexpr (NP == 2)
            put((long long)m * ncols + n,
                quotf(acc[i][j][q], __builtin_fmaf(sf, (float)(lm + cn[j]), bf)));
          else
            put((long long)m * ncols + n, (float)quot((double)acc[i][j][q], scale * (lm + cn[j]) + beta));
        }
      }
  } else if constexpr (FOLD) {
    const int half = (nmir + 1) / 2;
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + q;
        if (m >= half) continue;
        const int mm = nmir - 1 - m;
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          const int n = n0 + wn + 16 * j + (lane & 15);
          const float p = acc[i][j][q], qq = accq[i][j][q];
          put((long long)m * ncols + n, p + qq);
          if (mm != m) put((long long)mm * ncols + n, p - qq);
        }
      }
  } else if constexpr (YF) {
    // plane m of the y-folded output: row y < hpo the pair's sum, row hpo + y
    // its difference (the middle row of odd ny once; rows from ceil(ny / 2)
    // to hpo zero)
    const int hy = (ep.ny + 1) / 2;
    const int xw = x0 + (wave & 1) * (WN / 2);
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = orow(m0 + wm + 16 * i + 4 * (lane >> 4) + q);
#pragma unroll
        for (int j = 0; j < BN / 2; ++j) {
          const int x = xw + 16 * j + (lane & 15);
          const float d = acc[i][j][q], e = acc[i][j + BN / 2][q];
          const float vp = yf >= hy ? 0.0f : ybar == yf ? d : d + e;
          const float vm = (yf >= hy || ybar == yf) ? 0.0f : d - e;
          put((long long)m * ncols + (long long)yf * ep.px + x, vp);
          put((long long)m * ncols + (long long)(hpo + yf) * ep.px + x, vm);
        }
      }
  } else {
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = orow(m0 + wm + 16 * i + 4 * (lane >> 4) + q);
#pragma unroll
        for (int j = 0; j < BN; ++j)
          put((long long)m * ncols + n0 + wn + 16 * j + (lane & 15), acc[i][j][q]);
      }
  }
}

// ZF (bf16x3, the 3D path with folded forward products): the output written folded along z,
// hpo = the folded z layout's half extent.  A tile's rows are TM / 2 rows y of
// plane z < hpo and the same rows of plane nz-1-z, each wave's fragment row
// blocks split in halves so that a lane holds both values of a pair.
// ZF = 2: the input is folded along x as well (row positions [0, kc) the
// mirror sums, [kc, 2 kc) the differences, K = 2 kc): tile columns below kc
// are the even modes 2 t, contracting the sums, the others the odd modes
// 2 t + 1, contracting the differences (S: the even modes' rows of S then the
// odd modes', kc columns); output columns in mode order.
template <int NP, int TM, int TN, int EPI, bool FOLD = false, int ZF = 0>
__global__ __launch_bounds__(256, 2) void k_gemm_right_bf(const void* __restrict__ Av,
                                                          GemmOperands S, void* __restrict__ Cv,
                                                          int rows, int K, EpiArgs ep, int nh,
                                                          int nmir, int hpo, int kc) {
  // NP = 2: A and C (with EPI_STORE) are bf16 part planes; NP = 3: FP32 tensors
  constexpr bool PS = NP == 2;
  static_assert(!FOLD || NP == 2, "folded: the bf16x3 inverse products");
  static_assert(ZF >= 0 && ZF <= 2, "ZF: 0 plain, 1 z-folded output, 2 with an x-folded input");
  static_assert(!ZF || (NP == 2 && !FOLD && EPI == EPI_STORE && TM >= 64),
                "z-folded output: bf16x3 forward x product, paired row halves");
  const float* A = (const float*)Av;
  float* C = (float*)Cv;
  const long long plane = (long long)rows * K;
  constexpr int WM = TM / 2, WN = TN / 2, BM = WM / 16, BN = WN / 16;
  constexpr int NAV = TM * (BTK / 8);  // (row, 8 consecutive k) groups of the tensor chunk
  constexpr int NBV = TN * (BTK / 8);  // 16-byte vectors per S part
  constexpr int PA = (NAV + 255) / 256, PB = (NBV + 255) / 256;
  __shared__ __attribute__((aligned(16))) char As[NP][2][TM * RBK];
  __shared__ __attribute__((aligned(16))) char Bs[NP][2][TN * RBK];

  // FOLD: output columns n < nh only (nh: ceil(nmir / 2) rounded up to TN),
  // each giving columns n and nmir - 1 - n
  constexpr int HB = BM / 2;  // ZF: fragment row blocks per wave of each plane
  const int ytiles = ZF ? ep.py / (TM / 2) : 1;
  const int MT = ZF ? rows / (ep.pz * ep.py) * hpo * ytiles : rows / TM, NT = (FOLD ? nh : K) / TN;
  const int t = xcd_tile(blockIdx.x, MT * NT);
  const int nt = t % NT, mt = t / NT;
  const int r0 = mt * TM, n0 = nt * TN;
  // ZF: component, plane pair and first row of the tile
  const int zc = ZF ? mt / ytiles : 0, zf = ZF ? zc % hpo : 0, zcomp = ZF ? zc / hpo : 0;
  const int zbar = ZF ? max(ep.nz - 1 - zf, 0) : 0, y0 = ZF ? (mt % ytiles) * (TM / 2) : 0;
  if (ep.skip && ep.skip[(ZF ? zcomp : r0 / ep.py / ep.pz) % ep.inst_mod]) return;  // finished instance
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
  // ZF = 2: this tile's parity half of the x-folded input (TN divides kc) and
  // the output column of a tile column
  const int acol0 = ZF == 2 && n0 >= kc ? kc : 0;
  auto ocol = [&](int n) { return ZF == 2 ? 2 * (n - acol0) + (acol0 ? 1 : 0) : n; };
  // first data row of the tile's 16-row LDS block blk
  auto arow = [&](int blk) -> int {
    if constexpr (ZF) {
      const int a = blk / BM, i = blk % BM;
      return ((zcomp * ep.pz + (i < HB ? zf : zbar)) * ep.py) + y0 + a * (WM / 2) + 16 * (i % HB);
    } else {
      return r0 + 16 * blk;
    }
  };

  f4_t acc[BM][BN], accq[BM][BN];  // accq: the odd modes' sums (FOLD)
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) acc[i][j] = accq[i][j] = f4_t{0, 0, 0, 0};

  auto read_frags = [&](int buf, bf8_t (&a)[BM][NP], bf8_t (&bj)[BN][NP]) {
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int q = 0; q < NP; ++q)
        a[i][q] = *reinterpret_cast<const bf8_t*>(&As[q][buf][kswz(wm + 16 * i + (lane & 15), 16 * (lane >> 4))]);
#pragma unroll
    for (int j = 0; j < BN; ++j)
#pragma unroll
      for (int q = 0; q < NP; ++q)
        bj[j][q] = *reinterpret_cast<const bf8_t*>(&Bs[q][buf][kswz(wn + 16 * j + (lane & 15), 16 * (lane >> 4))]);
  };
  auto mma = [&](const bf8_t (&a)[BM][NP], const bf8_t (&bj)[BN][NP]) {
    if constexpr (FOLD) {
      // S[n-1-j][k] = (-1)^k S[j][k]: the even and odd modes' sums of column
      // j give columns j (p + q) and n-1-j (p - q)
#pragma unroll
      for (int i = 0; i < BM; ++i) {
        bf8_t ae[NP], ao[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          ae[q] = even_modes(a[i][q]);
          ao[q] = odd_modes(a[i][q]);
        }
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          acc[i][j] = mfma_split<NP>(ae, bj[j], acc[i][j]);
          accq[i][j] = mfma_split<NP>(ao, bj[j], accq[i][j]);
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < BN; ++j)
#pragma unroll
        for (int i = 0; i < BM; ++i) acc[i][j] = mfma_split<NP>(a[i], bj[j], acc[i][j]);
    }
  };
  const int nk = (ZF == 2 ? kc : K) / BTK;
  if constexpr (PS) {
    const __bf16* Ah = (const __bf16*)Av;
    // chunk k0 into LDS buffer buf: TM / 16 KiB blocks of data rows and TN / 16
    // of S rows (S[k][n] = S[n][k]) per part
    auto dload = [&](int k0, int buf) {
#pragma unroll
      for (int blk = wave; blk < TM / 16; blk += 4)
#pragma unroll
        for (int q = 0; q < NP; ++q) dload_rows(Ah + q * plane, K, arow(blk), acol0 + k0, lane, &As[q][buf][blk * 1024]);
#pragma unroll
      for (int blk = wave; blk < TN / 16; blk += 4)
#pragma unroll
        for (int q = 0; q < NP; ++q) dload_rows(part(S, q), ZF == 2 ? kc : K, n0 + 16 * blk, k0, lane, &Bs[q][buf][blk * 1024]);
    };
    dload(0, 0);
    for (int kc = 0; kc < nk; ++kc) {
      const int buf = kc & 1;
      // this chunk's loads have landed and every wave is done reading the
      // buffer the next chunk overwrites
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      bf8_t a[BM][NP], bj[BN][NP];
      read_frags(buf, a, bj);
      if (kc + 1 < nk) dload((kc + 1) * BTK, buf ^ 1);
      mma(a, bj);
    }
  } else {
    f4_t ra[PA][2];
    bf8_t rb[NP][PB];
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
#pragma unroll
          for (int q = 0; q < NP; ++q) rb[q][p] = *reinterpret_cast<const bf8_t*>(part(S, q) + off);
        }
      }
    };
    auto lstore = [&](int buf) {
#pragma unroll
      for (int p = 0; p < PA; ++p) {
        const int v = tid + 256 * p;
        if (v < NAV) {
          const int r = v / (BTK / 8), kv = (v % (BTK / 8)) * 8;
          bf8_t w[NP];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            __bf16 x[NP];
            split<NP>(ra[p][e >> 2][e & 3], x);
#pragma unroll
            for (int q = 0; q < NP; ++q) w[q][e] = x[q];
          }
#pragma unroll
          for (int q = 0; q < NP; ++q)
            *reinterpret_cast<bf8_t*>(&As[q][buf][kswz(r, 2 * kv)]) = w[q];
        }
      }
#pragma unroll
      for (int p = 0; p < PB; ++p) {
        const int v = tid + 256 * p;
        if (v < NBV) {
          const int n = v / (BTK / 8), kv = (v % (BTK / 8)) * 8;
#pragma unroll
          for (int q = 0; q < NP; ++q)
            *reinterpret_cast<bf8_t*>(&Bs[q][buf][kswz(n, 2 * kv)]) = rb[q][p];
        }
      }
    };

    gload(0);
    lstore(0);
    __syncthreads();
    for (int kc = 0; kc < nk; ++kc) {
      const int buf = kc & 1;
      if (kc + 1 < nk) gload((kc + 1) * BTK);
      {
        bf8_t a[BM][NP], bj[BN][NP];
        read_frags(buf, a, bj);
        mma(a, bj);
      }
      if (kc + 1 < nk) lstore(buf ^ 1);
      __syncthreads();
    }
  }

  if constexpr (ZF) {
    // plane zf of the z-folded output holds the pair's sum, plane hpo + zf its
    // difference (the middle plane of odd nz once; planes from ceil(nz / 2)
    // to hpo zero)
    const int hz = (ep.nz + 1) / 2;
    const int yw = y0 + (wave >> 1) * (WM / 2);
    const long long pp = (long long)(zcomp * ep.pz + zf) * ep.py, pm = pp + (long long)hpo * ep.py;
#pragma unroll
    for (int i = 0; i < HB; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int y = yw + 16 * i + 4 * (lane >> 4) + q;
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          const int n = ocol(n0 + wn + 16 * j + (lane & 15));
          const float d = acc[i][j][q], e = acc[i + HB][j][q];
          const float vp = zf >= hz ? 0.0f : zbar == zf ? d : d + e;
          const float vm = (zf >= hz || zbar == zf) ? 0.0f : d - e;
          put_pair((__bf16*)Cv, plane, (pp + y) * K + n, vp);
          put_pair((__bf16*)Cv, plane, (pm + y) * K + n, vm);
        }
      }
    return;
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
      const int r = r0 + wm + 16 * i + 4 * (lane >> 4) + q;
      base[q] = (long long)r * K;
      row_ok[q] = true;
      if (EPI != EPI_STORE) {
        const int y = r % ep.py, zc = r / ep.py, z = zc % ep.pz, c = zc / ep.pz;
        base[q] = (((long long)c * ep.nz + z) * ep.ny + y) * ep.nx;
        row_ok[q] = y < ep.ny && z < ep.nz;
      }
    }
    const double st = ep.step != 0 ? ep.step : 1.0;  // U -= step dU
    if constexpr (FOLD) {
      const int half = (nmir + 1) / 2;
      double old1[4][BN], old2[4][BN];
      if (EPI == EPI_SUB_DENSE) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int j = 0; j < BN; ++j) {
            const int n = n0 + wn + 16 * j + (lane & 15), nm = nmir - 1 - n;
            const bool in = row_ok[q] && n < half;
            old1[q][j] = in ? ep.dense[base[q] + n] : 0.0;
            old2[q][j] = (in && nm != n) ? ep.dense[base[q] + nm] : 0.0;
          }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (!row_ok[q]) continue;
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          const int n = n0 + wn + 16 * j + (lane & 15), nm = nmir - 1 - n;
          if (n >= half) continue;
          const float p = acc[i][j][q], qq = accq[i][j][q];
          const float v1 = p + qq, v2 = p - qq;
          if (EPI == EPI_STORE) {
            put_pair((__bf16*)Cv, plane, base[q] + n, v1);
            if (nm != n) put_pair((__bf16*)Cv, plane, base[q] + nm, v2);
          } else if (EPI == EPI_SUB_DENSE) {
            ep.dense[base[q] + n] = old1[q][j] - st * (double)v1;
            if (nm != n) ep.dense[base[q] + nm] = old2[q][j] - st * (double)v2;
          } else {
            ep.dense[base[q] + n] = (double)v1;
            if (nm != n) ep.dense[base[q] + nm] = (double)v2;
          }
        }
      }
      continue;
    }
    double old[4][BN];
    if (EPI == EPI_SUB_DENSE) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          const int n = n0 + wn + 16 * j + (lane & 15);
          old[q][j] = (row_ok[q] && n < ep.nx) ? ep.dense[base[q] + n] : 0.0;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        const int n = n0 + wn + 16 * j + (lane & 15);
        const float v = acc[i][j][q];
        if (EPI == EPI_STORE) {
          if constexpr (PS)
            put_pair((__bf16*)Cv, plane, base[q] + n, v);
          else
            C[base[q] + n] = v;
        } else if (row_ok[q] && n < ep.nx) {
          if (EPI == EPI_SUB_DENSE)
            ep.dense[base[q] + n] = old[q][j] - st * (double)v;
          else
            ep.dense[base[q] + n] = (double)v;
        }
      }
  }
}

namespace {

int parts_of(int prec) { return prec == 3 ? 3 : 2; }  // 3: bf16x6, else bf16x3

// fold > 0: the reflection-folded inverse product (bf16x3 only), output rows
// (form L) or columns (form R) [0, fold) of the axis of length nmir, fold a
// multiple of the tile side.  sp: the folded forward products of the 3D path.
template <int NP, int TM, int TN>
hipError_t left_tile(const GemmOperands& s, const void* B, void* C, int M, int ncols, int batch,
                     long long bstride, int epi, const EpiArgs& ep, hipStream_t st, int fold,
                     int nmir, const BfSplit* sp) {
  const int fwd = sp ? sp->mode : 0;
  if (fwd) {
    if constexpr (NP == 2) {
      const int K = sp->K;
      if (K <= 0 || K % BTK != 0) return hipErrorInvalidValue;
      if (fold > 0) return hipErrorInvalidValue;
      if (M != 2 * K || K % TM != 0) return hipErrorInvalidValue;
      if (fwd == 1) {  // forward from a folded input
        if (ncols % TN != 0 || (epi != EPI_STORE && epi != EPI_DIVIDE)) return hipErrorInvalidValue;
        const unsigned g = (unsigned)((long long)batch * (M / TM) * (ncols / TN));
        if (epi == EPI_DIVIDE)
          hipLaunchKernelGGL((k_gemm_left_bf<NP, TM, TN, EPI_DIVIDE, false, 1>), dim3(g), dim3(256), 0,
                             st, s, B, C, M, K, ncols, batch, bstride, ep, 0, 0, 0);
        else
          hipLaunchKernelGGL((k_gemm_left_bf<NP, TM, TN, EPI_STORE, false, 1>), dim3(g), dim3(256), 0,
                             st, s, B, C, M, K, ncols, batch, bstride, ep, 0, 0, 0);
        return hipGetLastError();
      }
      if constexpr (TN >= 64) {
        const int hpo = sp->hpo;  // forward, output folded along y
        if (fwd != 2 || epi != EPI_STORE || hpo <= 0 || ep.px % (TN / 2) != 0 ||
            (long long)ncols != (long long)ep.py * ep.px || 2 * hpo > ep.py || hpo > ep.ny)
          return hipErrorInvalidValue;
        const unsigned g = (unsigned)((long long)batch * (M / TM) * hpo * (ep.px / (TN / 2)));
        hipLaunchKernelGGL((k_gemm_left_bf<NP, TM, TN, EPI_STORE, false, 2>), dim3(g), dim3(256), 0, st,
                           s, B, C, M, K, ncols, batch, bstride, ep, 0, 0, hpo);
        return hipGetLastError();
      }
    }
    return hipErrorInvalidValue;
  }
  if (fold > 0) {
    if constexpr (NP == 2) {
      if (epi != EPI_STORE || fold % TM != 0 || fold > M || 2 * fold < nmir) return hipErrorInvalidValue;
      const unsigned g = (unsigned)((long long)batch * (fold / TM) * (ncols / TN));
      hipLaunchKernelGGL((k_gemm_left_bf<NP, TM, TN, EPI_STORE, true>), dim3(g), dim3(256), 0, st, s,
                         B, C, M, M, ncols, batch, bstride, ep, fold, nmir, 0);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  const unsigned g = (unsigned)((long long)batch * (M / TM) * (ncols / TN));
  if (epi == EPI_DIVIDE)
    hipLaunchKernelGGL((k_gemm_left_bf<NP, TM, TN, EPI_DIVIDE>), dim3(g), dim3(256), 0, st, s, B, C,
                       M, M, ncols, batch, bstride, ep, 0, 0, 0);
  else
    hipLaunchKernelGGL((k_gemm_left_bf<NP, TM, TN, EPI_STORE>), dim3(g), dim3(256), 0, st, s, B, C,
                       M, M, ncols, batch, bstride, ep, 0, 0, 0);
  return hipGetLastError();
}

template <int NP, int TM, int TN, bool FOLD>
hipError_t right_launch(const GemmOperands& s, const void* A, void* C, int rows, int K, int epi,
                        const EpiArgs& ep, hipStream_t st, int nout, int nmir) {
  const unsigned g = (unsigned)((long long)(rows / TM) * (nout / TN));
  switch (epi) {
    case EPI_SUB_DENSE:
      hipLaunchKernelGGL((k_gemm_right_bf<NP, TM, TN, EPI_SUB_DENSE, FOLD>), dim3(g), dim3(256), 0,
                         st, A, s, C, rows, K, ep, nout, nmir, 0, 0);
      break;
    case EPI_STORE_DENSE:
      hipLaunchKernelGGL((k_gemm_right_bf<NP, TM, TN, EPI_STORE_DENSE, FOLD>), dim3(g), dim3(256), 0,
                         st, A, s, C, rows, K, ep, nout, nmir, 0, 0);
      break;
    default:
      hipLaunchKernelGGL((k_gemm_right_bf<NP, TM, TN, EPI_STORE, FOLD>), dim3(g), dim3(256), 0, st,
                         A, s, C, rows, K, ep, nout, nmir, 0, 0);
  }
  return hipGetLastError();
}

template <int NP, int TM, int TN>
hipError_t right_tile(const GemmOperands& s, const void* A, void* C, int rows, int K, int epi,
                      const EpiArgs& ep, hipStream_t st, int fold, int nmir, const BfSplit* sp) {
  if (sp && sp->mode) {
    if constexpr (NP == 2 && TM >= 64) {
      // dense x product (or, with sp->K = kc > 0, from an input folded along
      // x), output folded along z
      const int hpo = sp->hpo, kc = sp->K;
      if (sp->mode != 3 || fold > 0 || epi != EPI_STORE || hpo <= 0 || K % TN != 0 ||
          ep.py % (TM / 2) != 0 || rows % (ep.pz * ep.py) != 0 || 2 * hpo > ep.pz || hpo > ep.nz ||
          (kc > 0 && (K != 2 * kc || kc % TN != 0 || 2 * kc < ep.nx)))
        return hipErrorInvalidValue;
      const unsigned g =
          (unsigned)((long long)(rows / (ep.pz * ep.py)) * hpo * (ep.py / (TM / 2)) * (K / TN));
      if (kc > 0)
        hipLaunchKernelGGL((k_gemm_right_bf<NP, TM, TN, EPI_STORE, false, 2>), dim3(g), dim3(256), 0,
                           st, A, s, C, rows, K, ep, K, 0, hpo, kc);
      else
        hipLaunchKernelGGL((k_gemm_right_bf<NP, TM, TN, EPI_STORE, false, 1>), dim3(g), dim3(256), 0,
                           st, A, s, C, rows, K, ep, K, 0, hpo, 0);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  if (fold > 0) {
    if constexpr (NP == 2) {
      if (fold % TN != 0 || fold > K || 2 * fold < nmir) return hipErrorInvalidValue;
      return right_launch<NP, TM, TN, true>(s, A, C, rows, K, epi, ep, st, fold, nmir);
    }
    return hipErrorInvalidValue;
  }
  return right_launch<NP, TM, TN, false>(s, A, C, rows, K, epi, ep, st, K, 0);
}

// Instantiated tiles: bf16x3 every side in {32, 64, 128}; bf16x6 (three parts
// in LDS) every side in {32, 64}.
#define QN_BF_TILES(FN, NP_, ...)                                          \
  if (NP_ == 2) {                                                          \
    if (tm == 128 && tn == 128) return FN<2, 128, 128>(__VA_ARGS__);       \
    if (tm == 128 && tn == 64) return FN<2, 128, 64>(__VA_ARGS__);         \
    if (tm == 128 && tn == 32) return FN<2, 128, 32>(__VA_ARGS__);         \
    if (tm == 64 && tn == 128) return FN<2, 64, 128>(__VA_ARGS__);         \
    if (tm == 64 && tn == 64) return FN<2, 64, 64>(__VA_ARGS__);           \
    if (tm == 64 && tn == 32) return FN<2, 64, 32>(__VA_ARGS__);           \
    if (tm == 32 && tn == 128) return FN<2, 32, 128>(__VA_ARGS__);         \
    if (tm == 32 && tn == 64) return FN<2, 32, 64>(__VA_ARGS__);           \
    if (tm == 32 && tn == 32) return FN<2, 32, 32>(__VA_ARGS__);           \
  } else {                                                                 \
    if (tm == 64 && tn == 64) return FN<3, 64, 64>(__VA_ARGS__);           \
    if (tm == 64 && tn == 32) return FN<3, 64, 32>(__VA_ARGS__);           \
    if (tm == 32 && tn == 64) return FN<3, 32, 64>(__VA_ARGS__);           \
    if (tm == 32 && tn == 32) return FN<3, 32, 32>(__VA_ARGS__);           \
  }                                                                        \
  return hipErrorInvalidValue;

}  // namespace

int gemm_bf_max_tile(int prec) { return parts_of(prec) == 3 ? 64 : 128; }

hipError_t launch_gemm_left(int prec, const GemmOperands& s, const void* B, void* C, int M,
                            int ncols, int batch, long long bstride, int epi, const EpiArgs& ep,
                            int tm, int tn, hipStream_t st, int fold, int nmir, const BfSplit* sp) {
  QN_BF_TILES(left_tile, parts_of(prec), s, B, C, M, ncols, batch, bstride, epi, ep, st, fold, nmir, sp)
}

hipError_t launch_gemm_right(int prec, const GemmOperands& s, const void* A, void* C, int rows,
                             int K, int epi, const EpiArgs& ep, int tm, int tn, hipStream_t st,
                             int fold, int nmir, const BfSplit* sp) {
  QN_BF_TILES(right_tile, parts_of(prec), s, A, C, rows, K, epi, ep, st, fold, nmir, sp)
}

#undef QN_BF_TILES

}  // namespace qn
