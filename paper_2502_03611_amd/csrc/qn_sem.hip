// Residual of the Q^k spectral element discretisation (Section 3.1, eq.
// final-system, and the remark on Gauss-Lobatto integration): after the
// diagonal mass is divided out, A_h U is the sum over axes of the banded
// H = M^-1 S applied along that axis (element order k: 2k + 1 coefficients
// per node), and the nonlinearity acts node by node, so
//   R = A_h U + lin U + cub U^3 + V U - F,  mu = 3 cub U^2 + lin + V,
// with the same partials {sum R^2, min mu, max mu, sum F^2} as the
// finite-difference residual, so the finalize and the loop are shared.
//
// One thread per node, x fastest (coalesced rows); a workgroup covers 256
// nodes of a row and marches SEM_ROWS rows in y at one z.  The x, y and z
// neighbours come from global memory through L1/L2.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>

#include "qn_internal.h"

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
      const double r = lap + a.cub * (u * u * u) + m * u - f;
      const double fu = 3.0 * a.cub * (u * u) + m;
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

}  // namespace

int sem_residual_blocks(int ox, int oy, int oz) {
  const dim3 g = sem_grid(ox, oy, oz);
  return (int)(g.x * g.y * g.z);
}

hipError_t launch_sem_residual(const ResidualArgs& a, int* nblocks_out, hipStream_t st) {
  const dim3 g = sem_grid(a.ox, a.oy, a.oz);
  *nblocks_out = (int)(g.x * g.y * g.z);
  if (a.out_prec == 0)
    hipLaunchKernelGGL(k_sem_residual<double>, g, dim3(SX), 0, st, a);
  else
    hipLaunchKernelGGL(k_sem_residual<float>, g, dim3(SX), 0, st, a);
  return hipGetLastError();
}

}  // namespace qn
