// Residual of the Q^k spectral element discretisation (Section 3.1, eq.
// final-system, and the remark on Gauss-Lobatto integration): after the
// diagonal mass is divided out, A_h U is the sum over axes of the banded
// H = M^-1 S applied along that axis (element order k: 2k + 1 coefficients
// per node), and the nonlinearity acts node by node, so
//   R = A_h U + lin U + cub U^3 + V U - F,  mu = 3 cub U^2 + lin + V,
// with the same partials {sum R^2, min mu, max mu, sum F^2} as the
// finite-difference residual, so the finalize and the loop are shared.
//
// 2D: one thread per node, x fastest (coalesced rows); a workgroup covers 256
// nodes of a row and marches SEM_ROWS rows in y.  The neighbours come from
// global memory through L1/L2.  3D: see k_sem_residual3 below.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>

#include "qn_internal.h"
#include "qn_mfma.h"

namespace qn {

namespace {

constexpr int SX = 256;

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wmin(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline double wmax(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

template <typename TO>
__global__ __launch_bounds__(SX) void k_sem_residual(ResidualArgs a) {
  if (a.stop && *a.stop) return;
  const int k = a.sem_k, w = 2 * k + 1;
  const int x = blockIdx.x * SX + threadIdx.x;
  const int y0 = blockIdx.y * SEM_ROWS, z = blockIdx.z;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const long long plane = (long long)nx * ny;
  double s_r = 0.0, s_f = 0.0, mn = DBL_MAX, mx = -DBL_MAX;
  for (int y = y0; y < min(y0 + SEM_ROWS, a.oy); ++y) {
    const bool in = x < nx && y < ny && z < nz;
    const long long o = (long long)z * a.r_zstride + (long long)y * a.r_ystride + x;
    if (in) {
      const long long i = (long long)z * plane + (long long)y * nx + x;
      double lap = 0.0;
      const double* hx = a.hb[0] + (long long)x * w;
      for (int d = -k; d <= k; ++d)
        if (x + d >= 0 && x + d < nx) lap += hx[d + k] * a.U[i + d];
      const double* hy = a.hb[1] + (long long)y * w;
      for (int d = -k; d <= k; ++d)
        if (y + d >= 0 && y + d < ny) lap += hy[d + k] * a.U[i + (long long)d * nx];
      if (a.dim == 3) {
        const double* hz = a.hb[2] + (long long)z * w;
        for (int d = -k; d <= k; ++d)
          if (z + d >= 0 && z + d < nz) lap += hz[d + k] * a.U[i + (long long)d * plane];
      }
      const double u = a.U[i], f = a.F[i];
      const double m = a.lin + (a.pot ? a.pot[i] : 0.0);
      const double r = lap + a.cub * (u * u * u) + a.quad * (u * u) + m * u - f;
      const double fu = 3.0 * a.cub * (u * u) + 2.0 * a.quad * u + m;
      s_r += r * r;
      s_f += f * f;
      mn = fmin(mn, fu);
      mx = fmax(mx, fu);
      reinterpret_cast<TO*>(a.R)[o] = (TO)r;
    } else if (x < a.ox && y < a.oy && z < a.oz) {
      reinterpret_cast<TO*>(a.R)[o] = (TO)0.0;
    }
  }
  __shared__ double red[SX / 64][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  s_r = wsum(s_r);
  mn = wmin(mn);
  mx = wmax(mx);
  s_f = wsum(s_f);
  if (lane == 0) {
    red[wv][0] = s_r;
    red[wv][1] = mn;
    red[wv][2] = mx;
    red[wv][3] = s_f;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < SX / 64; ++i) {
      s_r += red[i][0];
      mn = fmin(mn, red[i][1]);
      mx = fmax(mx, red[i][2]);
      s_f += red[i][3];
    }
    double* pp = a.partials + 4LL * ((blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x);
    pp[0] = s_r;
    pp[1] = mn;
    pp[2] = mx;
    pp[3] = s_f;
  }
}

dim3 sem_grid(int ox, int oy, int oz) {
  return dim3((ox + SX - 1) / SX, (oy + SEM_ROWS - 1) / SEM_ROWS, oz);
}

// 3D: a 64 x 8 (x, y) tile of threads marches in z over SEM_RZ planes.  Each
// thread keeps the 2K + 1 values U(x, y, z - K .. z + K) of its own column in
// registers (the z band), and every plane is staged in LDS with K-wide x and y
// halo strips (the x and y bands), its own values written from the window, so
// each node of U is fetched from global memory about once plus the halo
// share.  Tiles are dealt to the XCDs in contiguous ranges (x fastest), so the
// halo lines a tile shares with its neighbours meet in one L2.
constexpr int TX = 64, TY = 8;

template <int K, typename TO>
__global__ __launch_bounds__(TX * TY) void k_sem_residual3(ResidualArgs a) {
  constexpr int W = 2 * K + 1;
  constexpr int NH = 2 * K * TY + 2 * K * TX;           // halo cells per plane
  constexpr int NS = (NH + TX * TY - 1) / (TX * TY);    // halo slots per thread
  __shared__ double tile[TY + 2 * K][TX + 2 * K];
  __shared__ double cx[TX][W], cy[TY][W];               // x and y bands of the tile
  __shared__ double red[TX * TY / 64][4];
  if (a.stop && *a.stop) return;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  const int gx = gridDim.x, gy = gridDim.y;
  const int t = xcd_tile((blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x, gx * gy * gridDim.z);
  const int bx = t % gx, by = (t / gx) % gy, bz = t / (gx * gy);
  const int x0 = bx * TX, y0 = by * TY;
  const int x = x0 + tx, y = y0 + ty;
  const int z0 = bz * SEM_RZ, z1 = min(z0 + SEM_RZ, a.oz);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const long long plane = (long long)nx * ny;
  const bool col = x < nx && y < ny;
  const long long c = (long long)y * nx + x;
  auto ld = [&](int z) { return (col && z >= 0 && z < nz) ? a.U[(long long)z * plane + c] : 0.0; };
  double win[W];
#pragma unroll
  for (int d = 0; d < W; ++d) win[d] = ld(z0 - K + d);
  for (int i = tid; i < TX * W; i += TX * TY) {
    const int xx = x0 + i / W;
    cx[i / W][i % W] = xx < nx ? a.hb[0][(long long)xx * W + i % W] : 0.0;
  }
  if (tid < TY * W) {
    const int yy = y0 + tid / W;
    cy[tid / W][tid % W] = yy < ny ? a.hb[1][(long long)yy * W + tid % W] : 0.0;
  }
  // halo strips (left/right K columns x TY rows, bottom/top K rows x TX
  // columns): this thread's cells as (tile slot, plane offset or -1)
  int hs[NS];
  long long ho[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const int h = tid + j * TX * TY;
    hs[j] = -1;
    ho[j] = -1;
    if (h < NH) {
      int r, cc;
      if (h < 2 * K * TY) {
        const int side = h / (K * TY), q = h % (K * TY);
        r = K + q / K;
        cc = side == 0 ? q % K : TX + K + q % K;
      } else {
        const int q = h - 2 * K * TY, side = q / (K * TX), p = q % (K * TX);
        r = side == 0 ? p / TX : TY + K + p / TX;
        cc = K + p % TX;
      }
      const int gxh = x0 + cc - K, gyh = y0 + r - K;
      hs[j] = r * (TX + 2 * K) + cc;
      if (gxh >= 0 && gxh < nx && gyh >= 0 && gyh < ny) ho[j] = (long long)gyh * nx + gxh;
    }
  }
  double s_r = 0.0, s_f = 0.0, mn = DBL_MAX, mx = -DBL_MAX;
  for (int z = z0; z < z1; ++z) {
    const bool zin = z < nz;
    tile[ty + K][tx + K] = win[K];
#pragma unroll
    for (int j = 0; j < NS; ++j)
      if (hs[j] >= 0)
        (&tile[0][0])[hs[j]] = (zin && ho[j] >= 0) ? a.U[(long long)z * plane + ho[j]] : 0.0;
    __syncthreads();
    const long long o = (long long)z * a.r_zstride + (long long)y * a.r_ystride + x;
    if (col && zin) {
      const long long i = (long long)z * plane + c;
      const double* hz = a.hb[2] + (long long)z * W;  // uniform over the workgroup
      double lap = 0.0;
#pragma unroll
      for (int d = 0; d < W; ++d)
        lap += cx[tx][d] * tile[ty + K][tx + d] + cy[ty][d] * tile[ty + d][tx + K] + hz[d] * win[d];
      const double u = win[K], f = a.F[i];
      const double m = a.lin + (a.pot ? a.pot[i] : 0.0);
      const double r = lap + a.cub * (u * u * u) + a.quad * (u * u) + m * u - f;
      const double fu = 3.0 * a.cub * (u * u) + 2.0 * a.quad * u + m;
      s_r += r * r;
      s_f += f * f;
      mn = fmin(mn, fu);
      mx = fmax(mx, fu);
      reinterpret_cast<TO*>(a.R)[o] = (TO)r;
    } else if (x < a.ox && y < a.oy) {
      reinterpret_cast<TO*>(a.R)[o] = (TO)0.0;
    }
    __syncthreads();  // the tile is restaged for the next plane
#pragma unroll
    for (int d = 0; d < W - 1; ++d) win[d] = win[d + 1];
    win[W - 1] = ld(z + 1 + K);
  }
  const int lane = tid & 63, wv = tid >> 6;
  s_r = wsum(s_r);
  mn = wmin(mn);
  mx = wmax(mx);
  s_f = wsum(s_f);
  if (lane == 0) {
    red[wv][0] = s_r;
    red[wv][1] = mn;
    red[wv][2] = mx;
    red[wv][3] = s_f;
  }
  __syncthreads();
  if (tid == 0) {
    for (int i = 1; i < TX * TY / 64; ++i) {
      s_r += red[i][0];
      mn = fmin(mn, red[i][1]);
      mx = fmax(mx, red[i][2]);
      s_f += red[i][3];
    }
    double* pp = a.partials + 4LL * t;
    pp[0] = s_r;
    pp[1] = mn;
    pp[2] = mx;
    pp[3] = s_f;
  }
}

dim3 sem_grid3(int ox, int oy, int oz) {
  return dim3((ox + TX - 1) / TX, (oy + TY - 1) / TY, (oz + SEM_RZ - 1) / SEM_RZ);
}

template <int K>
void launch3(const ResidualArgs& a, dim3 g, hipStream_t st) {
  if (a.out_prec == 0)
    hipLaunchKernelGGL((k_sem_residual3<K, double>), g, dim3(TX, TY), 0, st, a);
  else
    hipLaunchKernelGGL((k_sem_residual3<K, float>), g, dim3(TX, TY), 0, st, a);
}

}  // namespace

int sem_residual_blocks(int dim, int ox, int oy, int oz) {
  const dim3 g = dim == 3 ? sem_grid3(ox, oy, oz) : sem_grid(ox, oy, oz);
  return (int)(g.x * g.y * g.z);
}

hipError_t launch_sem_residual(const ResidualArgs& a, int* nblocks_out, hipStream_t st) {
  if (a.dim == 3) {
    const dim3 g = sem_grid3(a.ox, a.oy, a.oz);
    *nblocks_out = (int)(g.x * g.y * g.z);
    switch (a.sem_k) {
      case 1: launch3<1>(a, g, st); break;
      case 2: launch3<2>(a, g, st); break;
      case 3: launch3<3>(a, g, st); break;
      case 4: launch3<4>(a, g, st); break;
      case 5: launch3<5>(a, g, st); break;
      case 6: launch3<6>(a, g, st); break;
      case 7: launch3<7>(a, g, st); break;
      default: launch3<8>(a, g, st); break;
    }
    return hipGetLastError();
  }
  const dim3 g = sem_grid(a.ox, a.oy, a.oz);
  *nblocks_out = (int)(g.x * g.y * g.z);
  if (a.out_prec == 0)
    hipLaunchKernelGGL(k_sem_residual<double>, g, dim3(SX), 0, st, a);
  else
    hipLaunchKernelGGL(k_sem_residual<float>, g, dim3(SX), 0, st, a);
  return hipGetLastError();
}

}  // namespace qn
