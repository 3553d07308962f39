// Bandwidth-bound passes of the quasi-Newton iteration:
//  * the residual F^h(U) = A_h vec(U) + N_h(U) (Section 4, eq. F_u) with the
//    pointwise nonlinearity fused into the stencil pass, the squared norms of
//    R and F and the extreme values of the Jacobian-diagonal quantity
//    reduced per workgroup (wave64 shuffles, then LDS across its waves);
//  * a one-workgroup, fixed-order reduction of those partials that also
//    evaluates the shift rule on the device (Section 4 midpoint beta;
//    Section 4.3 eq. eigenvalues for the 2-component system);
//  * the dense -> padded copy feeding a stand-alone solve.
//
// The residual kernel marches along z: each thread owns one (x, y) column of
// a z-slab and keeps U(z-1), U(z), U(z+1) in registers, so each U value is
// fetched once for its z-neighbours; the block's current plane (a tile of
// whole 512-, 256-, 128- or 64-column row segments with a one-point halo) is
// staged in LDS for the x/y neighbours, so U is re-read only along the halo.  2D grids are the nz = 1 case with 1/h_z^2 = 0.  Output points
// outside the interior (padding of the transform workspace) are written as
// zero on every call, so padding never carries stale values.

#include <algorithm>
#include <type_traits>
#include <cfloat>

#include "qn_internal.h"
#include "qn_mfma.h"

namespace qn {

// 3D residual workgroups: residual_threads(nl, bc) threads (1024 or 512) as
// TX x (threads / TX) columns of a z-slab (TX chosen per grid by
// residual_tile_x, the slab depth by residual_slab_depth; both are
// launch-time choices).

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Reduce (s0, mn, mx, s1) over a block of NW wave64s; thread 0 gets the result.
// ALLSUM: the middle two are sums as well.
template <int NW, bool ALLSUM = false>
__device__ inline void block_reduce4(double& s0, double& mn, double& mx, double& s1) {
  __shared__ double red[NW][4];
  const int lane = threadIdx.x + blockDim.x * threadIdx.y;
  const int w = lane >> 6, l = lane & 63;
  s0 = wave_sum(s0);
  mn = ALLSUM ? wave_sum(mn) : wave_min(mn);
  mx = ALLSUM ? wave_sum(mx) : wave_max(mx);
  s1 = wave_sum(s1);
  if (l == 0) {
    red[w][0] = s0;
    red[w][1] = mn;
    red[w][2] = mx;
    red[w][3] = s1;
  }
  __syncthreads();
  if (lane == 0) {
    for (int i = 1; i < NW; ++i) {
      s0 += red[i][0];
      mn = ALLSUM ? mn + red[i][1] : fmin(mn, red[i][1]);
      mx = ALLSUM ? mx + red[i][2] : fmax(mx, red[i][2]);
      s1 += red[i][3];
    }
  }
}

// Output element types: double, float, or the split-bf16 part pair of the
// FP32 value (hi = RNE(x) in the plane at base, lo = RNE(x - hi) in the plane
// `plane` elements further), the storage of the bf16x3 transforms.
struct BfPair {};
template <typename TO>
__device__ inline void put(void* base, long long idx, double v, long long plane) {
  if constexpr (std::is_same<TO, BfPair>::value) {
    const float x = (float)v;
    const __bf16 h = (__bf16)x;
    reinterpret_cast<__bf16*>(base)[idx] = h;
    reinterpret_cast<__bf16*>(base)[plane + idx] = (__bf16)(x - (float)h);
  } else {
    reinterpret_cast<TO*>(base)[idx] = (TO)v;
  }
}

// Trapezoid weight of node i of n along an axis with Neumann data.
__device__ inline double end_weight(int i, int n) { return (i == 0 || i == n - 1) ? 0.5 : 1.0; }

// BC = 1: homogeneous Neumann data by ghost nodes: a neighbour beyond either
// end of an axis is the mirror image of the one on the other side (first and
// last rows h^-2 (2, -2)); BC = 0: zero outside (Dirichlet).  MODE 1 and 2:
// the two passes of the eigenproblem residual (cubic problem only; see
// ResidualArgs), which read no F.
// XF: bf16 part-plane output folded along x (a.xfold, whole-row tiles).
template <int NL, typename TO, int BC, int MODE, int RX, bool XF = false>
__global__ __launch_bounds__(residual_threads(NL, BC), residual_threads(NL, BC) == 1024 ? 8 : 1)
void k_residual(ResidualArgs a) {
  constexpr int NC = (NL == NL_SYS2) ? 2 : 1;
  constexpr int RTHREADS = residual_threads(NL, BC);
  constexpr int RY = RTHREADS / RX;
  static_assert(RY >= 2, "the halo rows below and above need two tile rows");
  // Current z-plane of the block's RX x RY tile plus a one-point x/y halo,
  // double-buffered by plane parity: plane z+1 is written into the other
  // buffer while slower waves may still read plane z, so one barrier per
  // plane suffices (a wave can only overwrite a buffer two planes later,
  // after every wave has passed the barrier that follows its last read).
  __shared__ double s_buf[2][NC][RY + 2][RX + 2];
  // XF: each plane's R (rounded to FP32, as the part planes split it) is kept
  // in LDS, double-buffered by plane parity, and stored as the row's mirror
  // sums and differences after the next plane's barrier
  static_assert(!XF || (std::is_same<TO, BfPair>::value && MODE == 0), "x-folded output: bf16 parts");
  constexpr bool XFC = XF;
  __shared__ float s_x[XFC ? 2 : 1][NC][RY][XFC ? RX : 1];
  const int tx = threadIdx.x, ty = threadIdx.y;
  // Workgroups are dealt to the 8 XCDs round-robin in launch order; remapped,
  // each XCD walks a contiguous range of tiles (x fastest), so the halo lines
  // a tile shares with its x and y neighbours are fetched once into that
  // XCD's L2 instead of once per neighbour.
  const int gx = gridDim.x, gy = gridDim.y;
  const int tile = xcd_tile((blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x, gx * gy * gridDim.z);
  const int bx = tile % gx, by = (tile / gx) % gy, bz = tile / (gx * gy);
  const int x = bx * RX + tx;
  const int y = by * RY + ty;
  const int z0 = bz * a.rz;
  const int z1 = min(z0 + a.rz, a.oz);
  if (a.skip && a.skip[z0]) return;  // batched solver: finished instance (rz = 1)
  if (a.stop && *a.stop) return;      // single problem: the iteration has stopped
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const long long plane = (long long)nx * ny;
  const long long comp = plane * nz;
  const bool in_xy = (x < nx) && (y < ny);
  const bool out_xy = (x < a.ox) && (y < a.oy);
  // 2D problems (and the batched solver, whose z-planes are independent
  // instances) have no z coupling: never read a neighbouring plane.
  const bool zc = a.ihz2 != 0.0;
  // Halo duty of this thread: one x-neighbour column or one y-neighbour row.
  int hx = -1, hy = -1, lx = 0, ly = 0;
  if (tx == 0) { hx = x - 1; hy = y; lx = 0; ly = ty + 1; }
  else if (tx == RX - 1) { hx = x + 1; hy = y; lx = RX + 1; ly = ty + 1; }
  int vx = -1, vy = -1, mx_ = 0, my_ = 0;
  if (ty == 0) { vx = x; vy = y - 1; mx_ = tx + 1; my_ = 0; }
  else if (ty == RY - 1) { vx = x; vy = y + 1; mx_ = tx + 1; my_ = RY + 1; }
  const bool has_h = tx == 0 || tx == RX - 1, has_v = ty == 0 || ty == RY - 1;
  const bool h_ok = hx >= 0 && hx < nx && hy < ny;
  const bool v_ok = vy >= 0 && vy < ny && vx < nx;

  double s_r = 0.0, s_f = 0.0, mn = DBL_MAX, mx = -DBL_MAX;
  if constexpr (MODE == 1) mn = mx = 0.0;  // four sums
  const long long col = (long long)y * nx + x;
  const long long hoff = (long long)hy * nx + hx, voff = (long long)vy * nx + vx;
  // Register pipeline one plane deep: while plane z is computed, the loads of
  // plane z+1 (its U values, F, halo cells and U(z+2)) are already in flight.
  double um[NC], uc[NC], up[NC], f[NC], hc[NC], vc[NC];
  double n_up[NC], n_f[NC], n_hc[NC], n_vc[NC];
  double pv = 0.0, n_pv = 0.0;  // cubic problem: potential V at (x, y, z) and (x, y, z+1)
  auto load_plane = [&](int z, double* u_next, double* fz, double* hz, double* vz, double& pz) {
    const bool zin = z < nz;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double* Uc = a.U + c * comp + (long long)z * plane;
      u_next[c] = (in_xy && z + 1 < nz && (zc || z + 1 < z1)) ? Uc[plane + col] : 0.0;
      fz[c] = (MODE == 0 && in_xy && zin) ? a.F[c * comp + (long long)z * plane + col] : 0.0;
      hz[c] = (has_h && h_ok && zin) ? Uc[hoff] : 0.0;
      vz[c] = (has_v && v_ok && zin) ? Uc[voff] : 0.0;
    }
    if constexpr (NL == NL_CUBIC) pz = (a.pot && in_xy && zin) ? a.pot[(long long)z * plane + col] : 0.0;
  };
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    um[c] = (zc && in_xy && z0 > 0 && z0 - 1 < nz) ? a.U[c * comp + (long long)(z0 - 1) * plane + col] : 0.0;
    uc[c] = (in_xy && z0 < nz) ? a.U[c * comp + (long long)z0 * plane + col] : 0.0;
  }
  constexpr bool xf = XFC;
  // store plane zp of the x-folded output (its R values sit in s_x)
  auto put_folded = [&](int zp) {
    if constexpr (XFC) {
      if (y >= a.oy) return;
      const int hpx = a.xfold;
      const bool dif = tx >= hpx;
      const int j = dif ? tx - hpx : tx, jm = nx - 1 - j;
      const auto& sx = s_x[(zp - z0) & 1];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        float v = 0.0f;
        if (j < (nx + 1) / 2)
          v = jm == j ? (dif ? 0.0f : sx[c][ty][j])
                      : (dif ? sx[c][ty][j] - sx[c][ty][jm] : sx[c][ty][j] + sx[c][ty][jm]);
        const long long o = c * a.r_cstride + (long long)zp * a.r_zstride + (long long)y * a.r_ystride + tx;
        put<TO>(a.R, o, v, a.r_plane);
      }
    }
  };
  if (z0 < z1) load_plane(z0, up, f, hc, vc, pv);
  for (int z = z0; z < z1; ++z) {
    const bool zin = z < nz;
    auto& s_u = s_buf[(z - z0) & 1];
    if (z + 1 < z1) load_plane(z + 1, n_up, n_f, n_hc, n_vc, n_pv);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      s_u[c][ty + 1][tx + 1] = uc[c];
      // Halo cells are always written: zero outside the interior (Dirichlet data).
      if (has_h) s_u[c][ly][lx] = hc[c];
      if (has_v) s_u[c][my_][mx_] = vc[c];
    }
    __syncthreads();
    if (xf && z > z0) put_folded(z - 1);  // its R values were stored before this barrier
    if (in_xy && zin) {
      double r[NC];
      double rw = 1.0;  // mode 2: mass weight of the node in sum W R^2
      if (NL == NL_QUASILIN) {
        const double u = uc[0];
        const double ac = 1.0 + u * u;
        const double n_xm = s_u[0][ty + 1][tx], n_xp = s_u[0][ty + 1][tx + 2];
        const double n_ym = s_u[0][ty][tx + 1], n_yp = s_u[0][ty + 2][tx + 1];
        const double n_zm = zc ? um[0] : 0.0, n_zp = zc ? up[0] : 0.0;
        auto flux = [&](double un) { return 0.5 * (ac + (1.0 + un * un)) * (u - un); };
        const double lx_ = (flux(n_xm) + flux(n_xp)) * a.ihx2;
        const double ly_ = (flux(n_ym) + flux(n_yp)) * a.ihy2;
        const double lz_ = (flux(n_zm) + flux(n_zp)) * a.ihz2;
        r[0] = lx_ + ly_ + lz_ - f[0];
        s_f += f[0] * f[0];
        mn = fmin(mn, ac);
        mx = fmax(mx, ac);
      } else {
        double lap[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const double u = uc[c];
          double n_xm = s_u[c][ty + 1][tx], n_xp = s_u[c][ty + 1][tx + 2];
          double n_ym = s_u[c][ty][tx + 1], n_yp = s_u[c][ty + 2][tx + 1];
          double n_zm = zc ? um[c] : 0.0, n_zp = zc ? up[c] : 0.0;
          if constexpr (BC == 1) {  // n >= 2 per axis: an end has one real neighbour
            if (x == 0) n_xm = n_xp;
            if (x == nx - 1) n_xp = n_xm;
            if (y == 0) n_ym = n_yp;
            if (y == ny - 1) n_yp = n_ym;
            if (z == 0) n_zm = n_zp;
            if (z == nz - 1) n_zp = n_zm;
          }
          lap[c] = (2.0 * u - n_xm - n_xp) * a.ihx2 + (2.0 * u - n_ym - n_yp) * a.ihy2 +
                   (2.0 * u - n_zm - n_zp) * a.ihz2;
          s_f += f[c] * f[c];
        }
        if (NL == NL_CUBIC) {
          const double u = uc[0];
          const double m = a.lin + pv;
          if constexpr (MODE == 0) {
            r[0] = lap[0] + a.cub * (u * u * u) + a.quad * (u * u) + m * u - f[0];
            const double fu = 3.0 * a.cub * (u * u) + 2.0 * a.quad * u + m;
            mn = fmin(mn, fu);
            mx = fmax(mx, fu);
          } else {
            double wt = 1.0;
            if constexpr (BC == 1) wt = end_weight(x, nx) * end_weight(y, ny) * end_weight(z, nz);
            if constexpr (MODE == 1) {
              const double wu = wt * u;
              s_r += wu * lap[0];
              mn += wu * u;
              mx += wu * u * (u * u);
              s_f += wu * (m * u);
            } else {
              const double lam = a.eig[0], sc = a.eig[1];
              const double us = sc * u;
              r[0] = sc * lap[0] + a.cub * (us * us * us) + (m - lam) * us;
              const double fu = 3.0 * a.cub * (us * us) + (m - lam);
              mn = fmin(mn, fu);
              mx = fmax(mx, fu);
              rw = wt;
            }
          }
        } else {
          const double u = uc[0], v = uc[NC - 1];
          r[0] = lap[0] + u * u * u - v - f[0];
          r[NC - 1] = lap[NC - 1] + v * v * v - u - f[NC - 1];
          // 2x2 block [[3u^2, -1], [-1, 3v^2]]: eigenvalues (a+d -+ sqrt((a-d)^2 + 4)) / 2
          const double ea = 3.0 * u * u, ed = 3.0 * v * v;
          const double disc = sqrt((ea - ed) * (ea - ed) + 4.0);
          mn = fmin(mn, 0.5 * (ea + ed - disc));
          mx = fmax(mx, 0.5 * (ea + ed + disc));
        }
      }
      if constexpr (MODE != 1) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          s_r += rw * (r[c] * r[c]);
          const long long o = c * a.r_cstride + (long long)z * a.r_zstride + (long long)y * a.r_ystride + x;
          if constexpr (XFC) {
            if (xf) {
              s_x[(z - z0) & 1][c][ty][tx] = (float)r[c];
              continue;
            }
          }
          put<TO>(a.R, o, r[c], a.r_plane);
        }
      }
    } else if (MODE != 1 && out_xy) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const long long o = c * a.r_cstride + (long long)z * a.r_zstride + (long long)y * a.r_ystride + x;
        if constexpr (XFC) {
          if (xf) {
            s_x[(z - z0) & 1][c][ty][tx] = 0.0f;
            continue;
          }
        }
        put<TO>(a.R, o, 0.0, a.r_plane);
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      um[c] = uc[c];
      uc[c] = up[c];
      up[c] = n_up[c];
      f[c] = n_f[c];
      hc[c] = n_hc[c];
      vc[c] = n_vc[c];
    }
    pv = n_pv;
  }
  if (xf && z1 > z0) {  // the slab's last plane
    __syncthreads();
    put_folded(z1 - 1);
  }

  block_reduce4<RTHREADS / 64, MODE == 1>(s_r, mn, mx, s_f);
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    double* pp = a.partials + 4LL * tile;  // tile = (bz * gy + by) * gx + bx
    pp[0] = s_r;
    pp[1] = mn;
    pp[2] = mx;
    pp[3] = s_f;
  }
}

// Planar residual (2D problems and the batched solver's instances, 1/h_z^2 =
// 0): each wave owns 64 consecutive x and marches a.rz rows in y, keeping
// U(y-1), U(y), U(y+1) of its column in registers; x-neighbours come from the
// adjacent lanes (wave shuffles), the two strip-edge columns from global
// memory.  No LDS staging and no barriers in the march; the loads of row y+1
// are issued before row y is computed.  A workgroup (4 waves, 256 columns)
// stays inside one plane, so its partials belong to one instance.  Many
// planes per launch march 16 rows; a single small plane takes fewer rows per
// workgroup so that it still spreads over about a thousand workgroups.
constexpr int R2X = 256;

template <int NL, typename TO, int BC, int MODE = 0>
__global__ __launch_bounds__(R2X) void k_residual2d(ResidualArgs a) {
  constexpr int NC = (NL == NL_SYS2 || NL == NL_GS) ? 2 : 1;
  const int lane = threadIdx.x & 63;
  const int gx = gridDim.x, gy = gridDim.y;
  const int tile = xcd_tile((blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x, gx * gy * gridDim.z);
  const int bx = tile % gx, by = (tile / gx) % gy, pl = tile / (gx * gy);
  if (a.skip && a.skip[pl]) return;  // batched solver: finished instance
  if (a.stop && *a.stop) return;      // single problem: the iteration has stopped
  const int nx = a.nx, ny = a.ny;
  const int x = bx * R2X + threadIdx.x;
  const int y0 = by * a.rz, y1 = min(y0 + a.rz, a.oy);
  const long long plane = (long long)nx * ny;
  const long long comp = plane * a.nz;
  const bool xin = x < nx, xout = x < a.ox;
  const bool lh = lane == 0 && x >= 1 && x - 1 < nx;  // left strip edge: load U(x-1)
  const bool rh = lane == 63 && x + 1 < nx;           // right strip edge: load U(x+1)
  const double* Up = a.U + (long long)pl * plane;
  const double* Fp = MODE == 0 ? a.F + (long long)pl * plane : nullptr;
  auto ld = [&](const double* p, int c, int y, int xx, bool ok) {
    return (ok && y >= 0 && y < ny) ? p[c * comp + (long long)y * nx + xx] : 0.0;
  };
  // Cubic problem: potential V of the plane (single problems only: pl = 0).
  const bool has_pot = NL == NL_CUBIC && a.pot != nullptr;
  const double* Pp = has_pot ? a.pot + (long long)pl * plane : nullptr;

  double s_r = 0.0, s_f = 0.0, mn = DBL_MAX, mx = -DBL_MAX;
  if constexpr (MODE == 1) mn = mx = 0.0;  // four sums
  double um[NC], uc[NC], up[NC], f[NC], hl[NC], hr[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    um[c] = ld(Up, c, y0 - 1, x, xin);
    uc[c] = ld(Up, c, y0, x, xin);
    up[c] = ld(Up, c, y0 + 1, x, xin);
    f[c] = MODE == 0 ? ld(Fp, c, y0, x, xin) : 0.0;
    hl[c] = ld(Up, c, y0, x - 1, lh);
    hr[c] = ld(Up, c, y0, x + 1, rh);
  }
  double pv = has_pot ? ld(Pp, 0, y0, x, xin) : 0.0;
  for (int y = y0; y < y1; ++y) {
    // row y + 1 in flight while row y is computed
    double nup[NC], nf[NC], nhl[NC], nhr[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      nup[c] = ld(Up, c, y + 2, x, xin);
      nf[c] = MODE == 0 ? ld(Fp, c, y + 1, x, xin) : 0.0;
      nhl[c] = ld(Up, c, y + 1, x - 1, lh);
      nhr[c] = ld(Up, c, y + 1, x + 1, rh);
    }
    const double npv = has_pot ? ld(Pp, 0, y + 1, x, xin) : 0.0;
    double xm[NC], xp[NC], ym[NC], yp[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double l = __shfl_up(uc[c], 1, 64), r = __shfl_down(uc[c], 1, 64);
      xm[c] = lane == 0 ? hl[c] : l;
      xp[c] = lane == 63 ? hr[c] : r;
      ym[c] = um[c];
      yp[c] = up[c];
      if constexpr (BC == 1) {  // mirrored ghost nodes (n >= 2 per axis)
        if (x == 0) xm[c] = xp[c];
        if (x == nx - 1) xp[c] = xm[c];
        if (y == 0) ym[c] = yp[c];
        if (y == ny - 1) yp[c] = ym[c];
      }
    }
    const bool in = xin && y < ny;
    if (in) {
      double r[NC];
      double rw = 1.0;  // mode 2: mass weight of the node in sum W R^2
      if (NL == NL_QUASILIN) {
        const double u = uc[0];
        const double ac = 1.0 + u * u;
        auto flux = [&](double un) { return 0.5 * (ac + (1.0 + un * un)) * (u - un); };
        const double lx_ = (flux(xm[0]) + flux(xp[0])) * a.ihx2;
        const double ly_ = (flux(ym[0]) + flux(yp[0])) * a.ihy2;
        r[0] = lx_ + ly_ - f[0];
        s_f += f[0] * f[0];
        mn = fmin(mn, ac);
        mx = fmax(mx, ac);
      } else {
        double lap[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const double u = uc[c];
          lap[c] = (2.0 * u - xm[c] - xp[c]) * a.ihx2 + (2.0 * u - ym[c] - yp[c]) * a.ihy2;
          s_f += f[c] * f[c];
        }
        if (NL == NL_CUBIC) {
          const double u = uc[0];
          const double m = a.lin + pv;
          if constexpr (MODE == 0) {
            r[0] = lap[0] + a.cub * (u * u * u) + a.quad * (u * u) + m * u - f[0];
            const double fu = 3.0 * a.cub * (u * u) + 2.0 * a.quad * u + m;
            mn = fmin(mn, fu);
            mx = fmax(mx, fu);
          } else {
            double wt = 1.0;
            if constexpr (BC == 1) wt = end_weight(x, nx) * end_weight(y, ny);
            if constexpr (MODE == 1) {
              const double wu = wt * u;
              s_r += wu * lap[0];
              mn += wu * u;
              mx += wu * u * (u * u);
              s_f += wu * (m * u);
            } else {
              const double lam = a.eig[0], sc = a.eig[1];
              const double us = sc * u;
              r[0] = sc * lap[0] + a.cub * (us * us * us) + (m - lam) * us;
              const double fu = 3.0 * a.cub * (us * us) + (m - lam);
              mn = fmin(mn, fu);
              mx = fmax(mx, fu);
              rw = wt;
            }
          }
        } else if (NL == NL_GS) {
          // Gray-Scott: diffusion D_A, D_S on the Laplacians, all reaction
          // terms pointwise; the shift uses the real parts of the eigenvalues
          // of the reaction block [[-2SA + mu + rho, -A^2], [2SA, A^2 + rho]].
          const double A = uc[0], S = uc[NC - 1];
          const double sa = S * A, sa2 = sa * A, a2 = A * A;
          r[0] = a.gs_da * lap[0] - sa2 + (a.gs_mu + a.gs_rho) * A - f[0];
          r[NC - 1] = a.gs_ds * lap[NC - 1] + sa2 + a.gs_rho * S - f[NC - 1];
          const double ea = -2.0 * sa + a.gs_mu + a.gs_rho, eb = -a2, ec = 2.0 * sa,
                       ed = a2 + a.gs_rho;
          const double root = sqrt(fmax((ea - ed) * (ea - ed) + 4.0 * eb * ec, 0.0));
          mn = fmin(mn, 0.5 * (ea + ed - root));
          mx = fmax(mx, 0.5 * (ea + ed + root));
        } else {
          const double u = uc[0], v = uc[NC - 1];
          r[0] = lap[0] + u * u * u - v - f[0];
          r[NC - 1] = lap[NC - 1] + v * v * v - u - f[NC - 1];
          // 2x2 block [[3u^2, -1], [-1, 3v^2]]: eigenvalues (a+d -+ sqrt((a-d)^2 + 4)) / 2
          const double ea = 3.0 * u * u, ed = 3.0 * v * v;
          const double disc = sqrt((ea - ed) * (ea - ed) + 4.0);
          mn = fmin(mn, 0.5 * (ea + ed - disc));
          mx = fmax(mx, 0.5 * (ea + ed + disc));
        }
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if constexpr (MODE != 1) {
          s_r += rw * (r[c] * r[c]);
          const long long o = c * a.r_cstride + (long long)pl * a.r_zstride + (long long)y * a.r_ystride + x;
          put<TO>(a.R, o, r[c], a.r_plane);
        }
      }
    } else if (MODE != 1 && xout) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const long long o = c * a.r_cstride + (long long)pl * a.r_zstride + (long long)y * a.r_ystride + x;
        put<TO>(a.R, o, 0.0, a.r_plane);
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      um[c] = uc[c];
      uc[c] = up[c];
      up[c] = nup[c];
      f[c] = nf[c];
      hl[c] = nhl[c];
      hr[c] = nhr[c];
    }
    pv = npv;
  }

  block_reduce4<R2X / 64, MODE == 1>(s_r, mn, mx, s_f);
  if (threadIdx.x == 0) {
    double* pp = a.partials + 4LL * tile;  // tile = (pl * gy + by) * gx + bx
    pp[0] = s_r;
    pp[1] = mn;
    pp[2] = mx;
    pp[3] = s_f;
  }
}

// Tile width of the 3D residual: rows of 512, 256, 128 or 64 columns (at
// most half the workgroup's threads: a tile has at least two rows, one for
// each y halo), the widest whose lanes past the grid's x extent are at most an
// eighth of the tiles' span, else the one that leaves the fewest idle.  Long
// contiguous row segments per workgroup stream HBM best (511^3: 64-wide tiles
// 0.655 ms, 512-wide 0.611 ms at the same slab depth).
int residual_tile_x(int ox, int threads) {
  int best = 64;
  long long best_pad = -1;
  for (int rx = std::min(512, threads / 2); rx >= 64; rx >>= 1) {
    const long long span = (long long)((ox + rx - 1) / rx) * rx, pad = span - ox;
    if (pad * 8 <= span) return rx;
    if (best_pad < 0 || pad < best_pad) {
      best_pad = pad;
      best = rx;
    }
  }
  return best;
}

// Slab depth of the 3D residual: the fewest z-slabs per column tile that
// fill the last round of resident workgroups (256 CUs x 2048 threads) to at
// least 90 %, else the best fill with at most 64 slabs.  At 511^3 this is two
// slabs of 256 planes, one resident round of 512 workgroups of 1024 threads
// (64-plane slabs: 0.611 ms, 128: 0.601, 256: 0.580).
int residual_slab_depth(int ox, int oy, int oz, int threads) {
  const long long kResident = 256LL * 2048 / threads;
  const int rx = residual_tile_x(ox, threads), ry = threads / rx;
  const long long cols = (long long)((ox + rx - 1) / rx) * ((oy + ry - 1) / ry);
  const int smax = std::max(1, std::min(oz, 64));
  int best = 1;
  double best_fill = 0.0;
  for (int sl = 1; sl <= smax; ++sl) {
    const long long total = cols * sl;
    const double fill = (double)total / (double)(kResident * ((total + kResident - 1) / kResident));
    if (fill >= 0.9) {
      best = sl;
      break;
    }
    if (fill > best_fill) {
      best_fill = fill;
      best = sl;
    }
  }
  return (oz + best - 1) / best;
}

static dim3 residual_grid(int ox, int oy, int oz, int rz, bool planar, int threads) {
  if (planar) return dim3((ox + R2X - 1) / R2X, (oy + rz - 1) / rz, oz);
  const int rx = residual_tile_x(ox, threads), ry = threads / rx;
  return dim3((ox + rx - 1) / rx, (oy + ry - 1) / ry, (oz + rz - 1) / rz);
}

int residual_planar_rows(int ox, int oy) {
  const long long gx = (ox + R2X - 1) / R2X;
  int r = RESIDUAL_PLANAR_ROWS;
  while (r > 1 && gx * ((oy + r - 1) / r) < 1024) r >>= 1;
  return r;
}

int residual_max_blocks(int ox, int oy, int oz, int rz, bool planar, int threads) {
  const dim3 g = residual_grid(ox, oy, oz, rz, planar, threads);
  return (int)(g.x * g.y * g.z);
}

template <int NL, int BC, int MODE, int TX>
static void launch_3d(const ResidualArgs& a, dim3 g, hipStream_t st) {
  const dim3 b(TX, residual_threads(NL, BC) / TX);
  if constexpr (MODE == 0 && BC == 0) {  // the split-bf16 transforms: Dirichlet data only
    if (a.out_prec == 2 && a.xfold > 0) {
      hipLaunchKernelGGL((k_residual<NL, BfPair, BC, MODE, TX, true>), g, b, 0, st, a);
      return;
    }
  }
  if (a.out_prec == 0 || MODE == 1)
    hipLaunchKernelGGL((k_residual<NL, double, BC, MODE, TX>), g, b, 0, st, a);
  else if (a.out_prec == 2 && MODE == 0)
    hipLaunchKernelGGL((k_residual<NL, BfPair, BC, MODE, TX>), g, b, 0, st, a);
  else
    hipLaunchKernelGGL((k_residual<NL, float, BC, MODE, TX>), g, b, 0, st, a);
}

template <int NL, int BC, int MODE = 0>
static void launch_nl_bc(const ResidualArgs& a, dim3 g, bool planar, hipStream_t st) {
  if (planar) {
    if (a.out_prec == 0 || MODE == 1)
      hipLaunchKernelGGL((k_residual2d<NL, double, BC, MODE>), g, dim3(R2X), 0, st, a);
    else if (a.out_prec == 2 && MODE == 0)
      hipLaunchKernelGGL((k_residual2d<NL, BfPair, BC, MODE>), g, dim3(R2X), 0, st, a);
    else
      hipLaunchKernelGGL((k_residual2d<NL, float, BC, MODE>), g, dim3(R2X), 0, st, a);
    return;
  }
  constexpr int RT = residual_threads(NL, BC);
  switch (residual_tile_x(a.ox, RT)) {
    case 512:  // only when RT = 1024 (residual_tile_x keeps two tile rows)
      if constexpr (RT >= 1024) launch_3d<NL, BC, MODE, 512>(a, g, st);
      break;
    case 256: launch_3d<NL, BC, MODE, 256>(a, g, st); break;
    case 128: launch_3d<NL, BC, MODE, 128>(a, g, st); break;
    default: launch_3d<NL, BC, MODE, 64>(a, g, st); break;
  }
}

template <int BC>
static void launch_cubic(const ResidualArgs& a, dim3 g, bool planar, hipStream_t st) {
  if (a.mode == 1)
    launch_nl_bc<NL_CUBIC, BC, 1>(a, g, planar, st);
  else if (a.mode == 2)
    launch_nl_bc<NL_CUBIC, BC, 2>(a, g, planar, st);
  else
    launch_nl_bc<NL_CUBIC, BC, 0>(a, g, planar, st);
}

template <int NL>
static void launch_nl(const ResidualArgs& a, dim3 g, bool planar, hipStream_t st) {
  launch_nl_bc<NL, 0>(a, g, planar, st);
}

hipError_t launch_residual(const ResidualArgs& a, int* nblocks_out, hipStream_t st) {
  // planes without z coupling (2D problems, batched instances): the planar kernel
  const bool planar = a.ihz2 == 0.0;
  const dim3 g = residual_grid(a.ox, a.oy, a.oz, a.rz, planar, residual_threads(a.nl, a.bc));
  *nblocks_out = (int)(g.x * g.y * g.z);
  // the x-folded output pairs points of one row inside a tile: whole-row tiles
  if (a.xfold > 0 && (planar || a.out_prec != 2 || a.mode != 0 || a.ox != 2 * a.xfold ||
                      2 * a.xfold < a.nx || residual_tile_x(a.ox, residual_threads(a.nl, a.bc)) != a.ox))
    return hipErrorInvalidValue;
  switch (a.nl) {
    case NL_CUBIC:  // the only nonlinearity with Neumann data and eigenproblem passes
      if (a.bc == 1)
        launch_cubic<1>(a, g, planar, st);
      else
        launch_cubic<0>(a, g, planar, st);
      break;
    case NL_QUASILIN: launch_nl<NL_QUASILIN>(a, g, planar, st); break;
    case NL_GS:  // 2D only (planar kernel), Dirichlet or Neumann data
      if (!planar) return hipErrorInvalidValue;
      if (a.out_prec == 0) {
        if (a.bc == 1)
          hipLaunchKernelGGL((k_residual2d<NL_GS, double, 1>), g, dim3(R2X), 0, st, a);
        else
          hipLaunchKernelGGL((k_residual2d<NL_GS, double, 0>), g, dim3(R2X), 0, st, a);
      } else {
        if (a.bc == 1)
          hipLaunchKernelGGL((k_residual2d<NL_GS, float, 1>), g, dim3(R2X), 0, st, a);
        else
          hipLaunchKernelGGL((k_residual2d<NL_GS, float, 0>), g, dim3(R2X), 0, st, a);
      }
      break;
    default: launch_nl<NL_SYS2>(a, g, planar, st); break;
  }
  return hipGetLastError();
}

constexpr int FIN_THREADS = 1024;

// beta_k of the shift rules (the midpoint of Section 4 and the alternatives
// the paper's tables compare it with), c_k = 1.
__device__ inline double rule_beta(int rule, double mn, double mx, double beta_fixed) {
  switch (rule) {
    case RULE_MIDPOINT: return 0.5 * (mn + mx);
    case RULE_MAX: return mx;
    case RULE_SUM: return mn + mx;
    case RULE_MIN: return mn;
    default: return beta_fixed;
  }
}

__global__ __launch_bounds__(FIN_THREADS) void k_finalize(const double* __restrict__ partials,
                                                          int nblocks, DevScalars* sc, int rule,
                                                          double beta_fixed, double lam_min_sum,
                                                          double* red_out, double rtol, int iter,
                                                          int max_iter, DevScalars* mirror) {
  double s0 = 0.0, s1 = 0.0, mn = DBL_MAX, mx = -DBL_MAX;
  for (int i = threadIdx.x; i < nblocks; i += FIN_THREADS) {
    s0 += partials[4 * i + 0];
    mn = fmin(mn, partials[4 * i + 1]);
    mx = fmax(mx, partials[4 * i + 2]);
    s1 += partials[4 * i + 3];
  }
  block_reduce4<FIN_THREADS / 64>(s0, mn, mx, s1);
  if (threadIdx.x == 0) {
    DevScalars r{};
    r.scale = 1.0;
    r.beta = rule_beta(rule, mn, mx, beta_fixed);
    if (rule == RULE_COEFF_MID) r.scale = 0.5 * (mn + mx);
    r.sumsqR = s0;
    r.mumin = mn;
    r.mumax = mx;
    r.sumsqF = s1;
    r.relres = sqrt(s0) / sqrt(s1);
    r.flag = (r.scale > 0.0 && r.scale * lam_min_sum + r.beta > 0.0) ? 0.0 : 1.0;
    const double rr = r.relres;
    r.done = iter >= 0 && (!(rr <= 1e30) || rr <= rtol || iter >= max_iter || r.flag != 0.0);
    *sc = r;
    if (mirror) *mirror = r;  // the host's read-back slot (pinned, coherent)
    if (red_out) {
      red_out[0] = s0;
      red_out[1] = mn;
      red_out[2] = mx;
      red_out[3] = s1;
    }
  }
}

hipError_t launch_finalize(const double* partials, int nblocks, DevScalars* sc, int rule,
                           double beta_fixed, double lam_min_sum, double* red_out, double rtol,
                           int iter, int max_iter, hipStream_t st, DevScalars* mirror) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_THREADS), 0, st, partials, nblocks, sc, rule,
                     beta_fixed, lam_min_sum, red_out, rtol, iter, max_iter, mirror);
  return hipGetLastError();
}

// Eigenproblem, phase 1: from the sums over the stored iterate U~ (Section
// 4.4) the normalised iterate is U = s U~ with s = 1 / sqrt(h^d sum W U~^2),
// and, f(u) = cub u^3 + (lin + V) u being a polynomial in s,
//   lam = <A U + f(U), U>_M = (sum W (A U~) U~ + sum W (lin + V) U~^2) / sum W U~^2
//         + cub sum W U~^4 / (h^d (sum W U~^2)^2).
__global__ __launch_bounds__(FIN_THREADS) void k_eig_finalize1(const double* __restrict__ partials,
                                                               int nblocks, DevScalars* sc,
                                                               double cub, double hvol,
                                                               const int* stop) {
  if (stop && *stop) return;
  double au = 0.0, uu = 0.0, u4 = 0.0, vu = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += FIN_THREADS) {
    au += partials[4 * i + 0];
    uu += partials[4 * i + 1];
    u4 += partials[4 * i + 2];
    vu += partials[4 * i + 3];
  }
  block_reduce4<FIN_THREADS / 64, true>(au, uu, u4, vu);
  if (threadIdx.x == 0) {
    sc->uscale = 1.0 / sqrt(hvol * uu);
    sc->eig = (au + vu) / uu + cub * u4 / (hvol * uu * uu);
  }
}

hipError_t launch_eig_finalize1(const double* partials, int nblocks, DevScalars* sc, double cub,
                                double hvol, const int* stop, hipStream_t st) {
  hipLaunchKernelGGL(k_eig_finalize1, dim3(1), dim3(FIN_THREADS), 0, st, partials, nblocks, sc,
                     cub, hvol, stop);
  return hipGetLastError();
}

// Eigenproblem, phase 2: stopping rule ||F^h(U)||_M / |lam| and the shift.
__global__ __launch_bounds__(FIN_THREADS) void k_eig_finalize2(
    const double* __restrict__ partials, int nblocks, DevScalars* sc, int rule, double beta_fixed,
    double lam_min_sum, double hvol, double* red_out, double rtol, int iter, int max_iter,
    const int* stop, DevScalars* mirror) {
  if (stop && *stop) return;
  double s0 = 0.0, s1 = 0.0, mn = DBL_MAX, mx = -DBL_MAX;
  for (int i = threadIdx.x; i < nblocks; i += FIN_THREADS) {
    s0 += partials[4 * i + 0];
    mn = fmin(mn, partials[4 * i + 1]);
    mx = fmax(mx, partials[4 * i + 2]);
    s1 += partials[4 * i + 3];
  }
  block_reduce4<FIN_THREADS / 64>(s0, mn, mx, s1);
  if (threadIdx.x == 0) {
    DevScalars r = *sc;  // keeps lam and s from phase 1
    r.scale = 1.0;
    r.beta = rule_beta(rule, mn, mx, beta_fixed);
    r.sumsqR = hvol * s0;
    r.mumin = mn;
    r.mumax = mx;
    r.sumsqF = r.eig * r.eig;
    r.relres = sqrt(hvol * s0) / fabs(r.eig);
    r.flag = (lam_min_sum + r.beta > 0.0) ? 0.0 : 1.0;
    const double rr = r.relres;
    r.done = iter >= 0 && (!(rr <= 1e30) || rr <= rtol || iter >= max_iter || r.flag != 0.0);
    *sc = r;
    if (mirror) *mirror = r;
    if (red_out) {
      red_out[0] = r.eig;
      red_out[1] = r.uscale;
      red_out[2] = r.sumsqR;
      red_out[3] = mn;
      red_out[4] = mx;
      red_out[5] = rr;
    }
  }
}

hipError_t launch_eig_finalize2(const double* partials, int nblocks, DevScalars* sc, int rule,
                                double beta_fixed, double lam_min_sum, double hvol,
                                double* red_out, double rtol, int iter, int max_iter,
                                const int* stop, hipStream_t st, DevScalars* mirror) {
  hipLaunchKernelGGL(k_eig_finalize2, dim3(1), dim3(FIN_THREADS), 0, st, partials, nblocks, sc,
                     rule, beta_fixed, lam_min_sum, hvol, red_out, rtol, iter, max_iter, stop,
                     mirror);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_scale(double* __restrict__ u, long long n,
                                               const double* s) {
  const double f = *s;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    u[i] *= f;
}

hipError_t launch_scale(double* u, long long n, const double* s, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const long long blocks = std::min<long long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_scale, dim3((unsigned)blocks), dim3(256), 0, st, u, n, s);
  return hipGetLastError();
}

// Batched finalize: block k reduces instance k's partials and applies the
// stopping rule, then the shift rule for the next solve (rule_beta: a fixed
// beta, or the midpoint, max, min + max or min of the Jacobian-diagonal
// eigenvalue range).
__global__ __launch_bounds__(256) void k_bfinalize(const double* __restrict__ partials, int bpi,
                                                   BState* __restrict__ st, int* __restrict__ done,
                                                   int rule, double beta_fixed, double rtol,
                                                   int max_iter, double lam_min) {
  BState& s = st[blockIdx.x];
  if (s.done) return;
  const double* pp = partials + 4LL * bpi * blockIdx.x;
  double s0 = 0.0, s1 = 0.0, mn = DBL_MAX, mx = -DBL_MAX;
  for (int i = threadIdx.x; i < bpi; i += 256) {
    s0 += pp[4 * i + 0];
    mn = fmin(mn, pp[4 * i + 1]);
    mx = fmax(mx, pp[4 * i + 2]);
    s1 += pp[4 * i + 3];
  }
  block_reduce4<4>(s0, mn, mx, s1);
  if (threadIdx.x == 0) {
    const double rel = sqrt(s0) / sqrt(s1);
    if (s.iters == 0) {
      s.relres0 = rel;
      s.sumsqF = s1;
    }
    s.relres = rel;
    if (!(rel <= 1e30)) {  // also catches NaN
      s.done = 1;
      s.status = 4;  // QN_ERR_DIVERGED
    } else if (rel <= rtol) {
      s.done = 1;
      s.status = 0;
    } else if (s.iters >= max_iter) {
      s.done = 1;
      s.status = 3;  // QN_ERR_NOT_CONVERGED
    } else {
      const double b = rule_beta(rule, mn, mx, beta_fixed);
      if (!(lam_min + b > 0.0)) {  // singular or indefinite solve operator
        s.done = 1;
        s.status = 4;  // QN_ERR_DIVERGED
      } else {
        s.scale = 1.0;
        s.beta = b;
        s.iters += 1;
      }
    }
    done[blockIdx.x] = s.done;
  }
}

hipError_t launch_bfinalize(const double* partials, int bpi, int K, BState* st, int* done,
                            int rule, double beta_fixed, double rtol, int max_iter,
                            double lam_min, hipStream_t s) {
  hipLaunchKernelGGL(k_bfinalize, dim3(K), dim3(256), 0, s, partials, bpi, st, done, rule,
                     beta_fixed, rtol, max_iter, lam_min);
  return hipGetLastError();
}

__global__ void k_breset(BState* st, int* done, int K) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= K) return;
  BState z{};
  z.scale = 1.0;
  st[i] = z;
  done[i] = 0;
}

hipError_t launch_breset(BState* st, int* done, int K, hipStream_t s) {
  hipLaunchKernelGGL(k_breset, dim3((K + 255) / 256), dim3(256), 0, s, st, done, K);
  return hipGetLastError();
}

template <typename TO>
__global__ __launch_bounds__(256) void k_pad_copy(const double* __restrict__ src, void* __restrict__ dst,
                                                  int nx, int ny, int nz, int px, int py, int pz,
                                                  long long plane, int xfold) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  const int zc = blockIdx.z;  // c * pz + z
  const int z = zc % pz, c = zc / pz;
  if (x >= px || y >= py) return;
  double v = 0.0;
  const long long row = (((long long)c * nz + z) * ny + y) * nx;  // read only where y, z are interior
  if (xfold > 0) {  // folded along x: mirror sums, then differences
    const bool dif = x >= xfold;
    const int j = dif ? x - xfold : x, jm = nx - 1 - j;
    if (j < (nx + 1) / 2 && y < ny && z < nz)
      v = jm == j ? (dif ? 0.0 : src[row + j])
                  : (dif ? src[row + j] - src[row + jm] : src[row + j] + src[row + jm]);
  } else if (x < nx && y < ny && z < nz) {
    v = src[row + x];
  }
  put<TO>(dst, ((long long)zc * py + y) * px + x, v, plane);
}

hipError_t launch_pad_copy(const double* src, void* dst, int out_prec, int ncomp, int nx, int ny,
                           int nz, int px, int py, int pz, hipStream_t st, int xfold) {
  if (xfold > 0 && (out_prec != 2 || px != 2 * xfold || 2 * xfold < nx)) return hipErrorInvalidValue;
  dim3 g((px + 63) / 64, (py + 3) / 4, ncomp * pz);
  const long long plane = (long long)ncomp * pz * py * px;
  if (out_prec == 0)
    hipLaunchKernelGGL((k_pad_copy<double>), g, dim3(64, 4), 0, st, src, dst, nx, ny, nz, px, py,
                       pz, plane, 0);
  else if (out_prec == 2)
    hipLaunchKernelGGL((k_pad_copy<BfPair>), g, dim3(64, 4), 0, st, src, dst, nx, ny, nz, px, py,
                       pz, plane, xfold);
  else
    hipLaunchKernelGGL((k_pad_copy<float>), g, dim3(64, 4), 0, st, src, dst, nx, ny, nz, px, py,
                       pz, plane, 0);
  return hipGetLastError();
}

__global__ void k_set_coef(double* slot, double scale, double beta) {
  slot[0] = scale;
  slot[1] = beta;
}

hipError_t launch_set_coef(double* slot, double scale, double beta, hipStream_t st) {
  hipLaunchKernelGGL(k_set_coef, dim3(1), dim3(1), 0, st, slot, scale, beta);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_zero(uint4* p, size_t n16) {
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * 256;
  for (; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  // Workspace segments are 256-byte aligned and sized in multiples of 256.
  const size_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  size_t blocks = (n16 + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, (uint4*)p, n16);
  return hipGetLastError();
}

}  // namespace qn
