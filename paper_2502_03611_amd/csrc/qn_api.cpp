// Host side of libqn: the C ABI declared in include/qn.h.
//
// A context holds the grid, the closed-form 1D eigen-data per axis (computed
// on the host at setup, uploaded into the caller-bound workspace), and the
// per-iteration kernel sequence:
//   residual + reductions -> finalize (norms, shift rule on device)
//   -> forward mode products x, y(, z) with the spectral divide fused into the
//   last one -> inverse mode products (z,) y, x with U -= dU fused into the
//   last one (Section 4.1 eq. fin_inverse, Section 4 eq. identity-method).
// All work is enqueued on the context's stream; qn_iterate takes the stopping
// decision on the device and reads the scalars of each iteration back while
// the next one is already queued.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qn.h"
#include "qn_host.h"
#include "qn_internal.h"

using namespace qn;

namespace {

thread_local std::string g_err;

qn_status fail(qn_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

enum KernelId {
  K_RESIDUAL = 0,
  K_FINALIZE,
  K_GEMM_X,         // forward x product
  K_GEMM_YZ,        // forward y / z products (plain store)
  K_GEMM_DIVIDE,    // last forward product with the spectral divide
  K_GEMM_X_UPDATE,  // inverse x product with U -= dU (or X = dU)
  K_PAD_COPY,
  K_GEMM_YZ_INV,    // inverse y / z products
  K_EIG_SUMS,       // eigenproblem: sums over the stored iterate
  K_EIG_FINALIZE,   // eigenproblem: Rayleigh quotient and normalising factor
  K_COUNT
};
const char* const kKernelNames[K_COUNT] = {"residual",    "finalize",      "gemm_x",
                                           "gemm_yz",     "gemm_divide",   "gemm_x_update",
                                           "pad_copy",    "gemm_yz_inv",   "eig_sums",
                                           "eig_finalize"};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Largest tile side (up to cap) dividing a padded extent (a multiple of 32).
int pick_tile(long long extent, int cap) {
  if (cap >= 128 && extent % 128 == 0) return 128;
  if (cap >= 64 && extent % 64 == 0) return 64;
  return 32;
}

struct Pending {
  int kid;
  hipEvent_t a, b;
};

}  // namespace

namespace qn {
// Shared with the network's C ABI (qnn_api.cpp): sets the thread-local message.
qn_status set_error(qn_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}
}  // namespace qn

struct qn_ctx_s {
  int dim = 3, ncomp = 1, nl = 0, prec = 0, beta_mode = 0, timing = 0;
  int n[3] = {1, 1, 1};  // interior x, y, z (z = 1 in 2D)
  int p[3] = {32, 32, 1};
  double beta = 0.0;
  double lam_min_sum = 0.0;
  int bc = QN_BC_DIRICHLET;
  double length = 1.0, lin = 0.0, cub = 1.0, quad = 0.0;
  double hvol = 1.0;  // h^d: the mass of one interior node
  int sem_k = 0;      // spectral elements: element order (0: finite differences)
  std::vector<double> hHb[3];  // spectral elements: banded H per axis
  size_t off_Hb[3] = {0, 0, 0};
  double sem_lmin[3] = {0.0, 0.0, 0.0};
  std::vector<double> hx[3];  // node coordinates per axis, from one end of the side
  const double* pot = nullptr;  // caller-owned potential V, or NULL
  double ih2[3] = {1.0, 1.0, 0.0};  // h^-2 per axis (0 for the missing z of 2D)
  hipStream_t stream = nullptr;
  bool fold = true;       // reflection-folded transforms (FP64/FP32); dense for split-bf16
  FoldAxis ax[3] = {};
  FoldTile tile[6] = {};  // per mode-product launch of the folded solve (after qn_autotune)
  bool tuned = false;
  std::vector<double> hS[3], hlam[3];  // dense S or folded FeT|FoT|Fe|Fo; lam (split if folded)
  // 3D split-bf16 solves with folded forward y and z products: half extents
  // of the folded layouts and the forward operands (bf16 parts) of y and z
  bool fwdfold = false;
  bool xfold = false;  // the x product too, from a residual written folded along x
  int hp[3] = {0, 0, 0};
  std::vector<double> hSf[3];
  size_t off_Sf[3][2] = {};
  // workspace layout (byte offsets)
  size_t off_S[3] = {0, 0, 0}, off_Slo[3] = {0, 0, 0}, off_Slo2[3] = {0, 0, 0}, off_lam[3] = {0, 0, 0};
  size_t off_W1 = 0, off_W2 = 0, off_part = 0, off_scal = 0, off_coef = 0, off_cscale = 0,
         need = 0;
  double step = 1.0;  // qn_iterate: U -= step * dU
  double gs[4] = {0.0, 0.0, 0.0, 0.0};  // Gray-Scott: D_A, D_S, rho, mu
  int max_blocks = 0;
  char* ws = nullptr;
  hipError_t sticky = hipSuccess;
  // timing
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  // qn_iterate: pinned two-slot ring of per-iteration scalars and their events
  DevScalars* hring = nullptr;  // host address
  DevScalars* dring = nullptr;  // the same slots' device address
  hipEvent_t ring_ev[2] = {nullptr, nullptr};
  double tot_ms[K_COUNT] = {};
  long long launches[K_COUNT] = {};

  size_t elem() const { return prec == QN_PREC_FP64 ? 8 : 4; }
  size_t tensor_elems() const { return (size_t)ncomp * p[2] * p[1] * p[0]; }
  template <typename T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  DevScalars* scal() const { return at<DevScalars>(off_scal); }
};

namespace {

qn_status check_ctx(qn_ctx c, bool need_ws) {
  if (!c) return fail(QN_ERR_INVALID, "null context");
  if (c->sticky != hipSuccess)
    return fail(QN_ERR_HIP, "context has a sticky HIP error: %s", hipGetErrorString(c->sticky));
  if (need_ws && !c->ws) return fail(QN_ERR_WORKSPACE, "workspace not bound");
  return QN_OK;
}

qn_status hip_fail(qn_ctx c, hipError_t e, const char* what) {
  c->sticky = e;
  return fail(QN_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned8(const void* p) { return ((uintptr_t)p & 7u) == 0; }

hipEvent_t take_event(qn_ctx c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch `fn` bracketed by timing events when the context asks for them.
template <typename Fn>
hipError_t timed(qn_ctx c, int kid, Fn fn) {
  hipEvent_t a = nullptr, b = nullptr;
  if (c->timing) {
    a = take_event(c);
    b = take_event(c);
    if (a) (void)hipEventRecord(a, c->stream);
  }
  hipError_t e = fn();
  if (c->timing && a && b) {
    (void)hipEventRecord(b, c->stream);
    c->pending.push_back({kid, a, b});
  }
  return e;
}

void fold_timing(qn_ctx c) {
  if (c->pending.empty()) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto& p : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->tot_ms[p.kid] += ms;
      c->launches[p.kid] += 1;
    }
    c->pool.push_back(p.a);
    c->pool.push_back(p.b);
  }
  c->pending.clear();
}

int rule_of(qn_ctx c) {
  if (c->nl == QN_NL_QUASILIN) return RULE_COEFF_MID;
  switch (c->beta_mode) {
    case QN_BETA_MIDPOINT: return RULE_MIDPOINT;
    case QN_BETA_MAX: return RULE_MAX;
    case QN_BETA_SUM: return RULE_SUM;
    case QN_BETA_MIN: return RULE_MIN;
    default: return RULE_FIXED;
  }
}

FoldOperands fold_ops(qn_ctx c, int axis) {
  const size_t bb = (size_t)c->ax[axis].bk * c->ax[axis].bk * c->elem();
  char* base = c->ws + c->off_S[axis];
  FoldOperands f{};
  f.FeT = base;
  f.FoT = base + bb;
  f.Fe = base + 2 * bb;
  f.Fo = base + 3 * bb;
  return f;
}

// Tile of a fold launch: the first instantiated shape (in order of preference)
// that divides the launch's extents and gives at least two workgroups per CU;
// when none does (small 2D grids), the admissible shape with the most
// workgroups.
FoldTile pick_fold_tile(int kind, int bk, int ncols, int batch, int rows) {
  const FoldTile* list;
  const int nc = fold_tiles(kind, &list);
  const long long want = 2LL * 256;
  FoldTile best{32, 32, 0, 0};
  long long best_blocks = -1;
  for (int i = 0; i < nc; ++i) {
    if (!fold_tile_fits(kind, list[i], bk, ncols, rows)) continue;
    const long long blocks = fold_blocks(kind, list[i], bk, ncols, batch, rows);
    if (blocks >= want) return list[i];
    if (blocks > best_blocks) {
      best_blocks = blocks;
      best = list[i];
    }
  }
  return best;
}

// One mode-product launch of the folded solve.
struct FoldStep {
  int kind, axis, kid;
  const void* in;
  void* out;
  int ncols, batch;     // form L: columns of a slab, slab count
  long long bstride;    // form L: slab stride
  int rows;             // form R: row count
  int epi;
  EpiArgs ep;
  int m, k;             // dense split-bf16 steps: contraction length (P of the axis)
  int nmir = 0;         // bf16x3 inverse steps: folded form over an axis of nmir points
  BfSplit sp{};         // 3D bf16x3 folded forward steps (mode 0: none)
  int sop = 0;          // operands: 0 S, 1 the folded forward Sf
};

// Dense split-bf16 step kinds (the folded ones are FK_*).
enum DenseKind { DK_RIGHT = 10, DK_LEFT = 11 };

GemmOperands operands(qn_ctx c, int axis, int sop = 0) {
  GemmOperands g{};
  g.Shi = c->ws + (sop == 1 ? c->off_Sf[axis][0] : c->off_S[axis]);
  g.Slo = c->ws + (sop == 1 ? c->off_Sf[axis][1] : c->off_Slo[axis]);
  g.Slo2 = c->ws + c->off_Slo2[axis];
  return g;
}

// Residual arguments for U (and F) with the output R either the padded
// transform workspace W1 in the context's precision (into_ws) or a caller
// array of the interior layout in FP64.
ResidualArgs residual_args(qn_ctx c, const double* U, const double* F, double* R_caller) {
  ResidualArgs a{};
  a.U = U;
  a.F = F;
  const int* ext = R_caller ? c->n : c->p;
  a.R = R_caller ? (void*)R_caller : (void*)(c->ws + c->off_W1);
  // split-bf16 two-part transforms keep their tensors as bf16 part planes
  a.out_prec = (R_caller || c->prec == QN_PREC_FP64) ? 0 : c->prec == QN_PREC_BF16X3 ? 2 : 1;
  a.r_cstride = (long long)ext[2] * ext[1] * ext[0];
  a.r_zstride = ext[1] * ext[0];
  a.r_ystride = ext[0];
  a.r_plane = (long long)c->ncomp * a.r_cstride;
  a.ox = ext[0];
  a.oy = ext[1];
  a.oz = ext[2];
  a.nx = c->n[0];
  a.ny = c->n[1];
  a.nz = c->n[2];
  a.dim = c->dim;
  a.nl = c->nl;
  a.ihx2 = c->ih2[0];
  a.ihy2 = c->ih2[1];
  a.ihz2 = c->ih2[2];
  a.lin = c->lin;
  a.cub = c->cub;
  a.quad = c->quad;
  a.pot = c->pot;
  a.bc = c->bc;
  a.partials = c->at<double>(c->off_part);
  a.xfold = (!R_caller && c->xfold) ? c->hp[0] : 0;  // the x product reads it folded
  a.rz = c->dim == 3 ? residual_slab_depth(a.ox, a.oy, a.oz, residual_threads(c->nl, c->bc))
                      : residual_planar_rows(a.ox, a.oy);
  a.sem_k = c->sem_k;
  for (int i = 0; i < c->dim && c->sem_k > 0; ++i) a.hb[i] = c->at<double>(c->off_Hb[i]);
  a.gs_da = c->gs[0];
  a.gs_ds = c->gs[1];
  a.gs_rho = c->gs[2];
  a.gs_mu = c->gs[3];
  return a;
}

// The residual launch of the context's discretization.
hipError_t launch_any_residual(const ResidualArgs& a, int* nb, hipStream_t st) {
  return a.sem_k > 0 ? launch_sem_residual(a, nb, st) : launch_residual(a, nb, st);
}

// Residual of U into the padded transform workspace W1 (+ partials), then
// the on-device finalize with the context's shift rule.
hipError_t residual_into_ws(qn_ctx c, const double* U, const double* F, double* red_out,
                            double rtol = 0.0, int iter = -1, int max_iter = 0,
                            const int* stop = nullptr, DevScalars* mirror = nullptr) {
  ResidualArgs a = residual_args(c, U, F, nullptr);
  a.stop = stop;
  int nb = 0;
  hipError_t e = timed(c, K_RESIDUAL, [&] { return launch_any_residual(a, &nb, c->stream); });
  if (e != hipSuccess) return e;
  return timed(c, K_FINALIZE, [&] {
    return launch_finalize(a.partials, nb, c->scal(), rule_of(c), c->beta, c->lam_min_sum, red_out,
                           rtol, iter, max_iter, c->stream, mirror);
  });
}

// Eigenproblem residual (Section 4.4) of the stored iterate U~: the sums
// pass and its finalize (lam, s into the device scalars), then R at U = s U~
// into W1 (R_caller == NULL) or the caller's array, and the stopping / shift
// finalize.  U~ itself is not modified.
hipError_t eigen_residual(qn_ctx c, const double* U, double* R_caller, double* red_out,
                          double rtol, int iter, int max_iter, const int* stop,
                          DevScalars* mirror) {
  ResidualArgs a = residual_args(c, U, nullptr, R_caller);
  a.stop = stop;
  a.mode = 1;
  int nb = 0;
  hipError_t e = timed(c, K_EIG_SUMS, [&] { return launch_residual(a, &nb, c->stream); });
  if (e == hipSuccess)
    e = timed(c, K_EIG_FINALIZE, [&] {
      return launch_eig_finalize1(a.partials, nb, c->scal(), c->cub, c->hvol, stop, c->stream);
    });
  a.mode = 2;
  a.eig = &c->scal()->eig;
  if (e == hipSuccess) e = timed(c, K_RESIDUAL, [&] { return launch_residual(a, &nb, c->stream); });
  if (e == hipSuccess)
    e = timed(c, K_FINALIZE, [&] {
      return launch_eig_finalize2(a.partials, nb, c->scal(), rule_of(c), c->beta, c->lam_min_sum,
                                  c->hvol, red_out, rtol, iter, max_iter, stop, c->stream, mirror);
    });
  return e;
}

// The folded solve as a list of launches (3D: x, y forward; z forward with
// the divide; z, y inverse; x inverse with the dense epilogue.  2D: x
// forward; y forward with the divide; y inverse; x inverse).  The transform
// ping-pongs between W1 and W2; `ep` carries coefficients and the dense
// target.  Returns the number of launches.
int fold_plan(qn_ctx c, const EpiArgs& ep, int epi_last, FoldStep* st) {
  void* W1 = c->ws + c->off_W1;
  void* W2 = c->ws + c->off_W2;
  const int px = c->p[0], py = c->p[1], pz = c->p[2];
  const int rows = c->ncomp * pz * py;
  const long long yslab = (long long)py * px, zslab = (long long)pz * py * px;
  int ns = 0;
  auto add = [&](int kind, int axis, int kid, const void* in, void* out, int ncols, int batch,
                 long long bstride, int epi, const EpiArgs& e) {
    FoldStep f{};
    f.kind = kind;
    f.axis = axis;
    f.kid = kid;
    f.in = in;
    f.out = out;
    f.ncols = ncols;
    f.batch = batch;
    f.bstride = bstride;
    f.rows = rows;
    f.epi = epi;
    f.ep = e;
    st[ns++] = f;
  };
  add(FK_RFWD, 0, K_GEMM_X, W1, W2, 0, 0, 0, EPI_STORE, ep);
  if (c->dim == 2) {
    EpiArgs ed = ep;
    ed.lamM = c->at<double>(c->off_lam[1]);
    ed.lamY = nullptr;
    add(FK_LFWD, 1, K_GEMM_DIVIDE, W2, W1, px, c->ncomp, yslab, EPI_DIVIDE, ed);
    add(FK_LINV, 1, K_GEMM_YZ_INV, W1, W2, px, c->ncomp, yslab, EPI_STORE, ep);
  } else {
    add(FK_LFWD, 1, K_GEMM_YZ, W2, W1, px, c->ncomp * pz, yslab, EPI_STORE, ep);
    EpiArgs ed = ep;
    ed.lamM = c->at<double>(c->off_lam[2]);
    ed.lamY = c->at<double>(c->off_lam[1]);
    add(FK_LFWD, 2, K_GEMM_DIVIDE, W1, W2, (int)yslab, c->ncomp, zslab, EPI_DIVIDE, ed);
    add(FK_LINV, 2, K_GEMM_YZ_INV, W2, W1, (int)yslab, c->ncomp, zslab, EPI_STORE, ep);
    add(FK_LINV, 1, K_GEMM_YZ_INV, W1, W2, px, c->ncomp * pz, yslab, EPI_STORE, ep);
  }
  // x inverse: the dense epilogue writes ep.dense; with EPI_STORE it writes W1
  add(FK_RINV, 0, K_GEMM_X_UPDATE, W2, W1, 0, 0, 0, epi_last, ep);
  return ns;
}

// The dense split-bf16 solve as a list of launches (same order and timing
// keys as the folded one; 3D y/z products are form L over slabs, the x
// products form R over rows).
int dense_plan(qn_ctx c, const EpiArgs& ep, int epi_last, FoldStep* st) {
  void* W1 = c->ws + c->off_W1;
  void* W2 = c->ws + c->off_W2;
  const int px = c->p[0], py = c->p[1], pz = c->p[2];
  const int rows = c->ncomp * pz * py;
  const long long yslab = (long long)py * px, zslab = (long long)pz * py * px;
  int ns = 0;
  // bf16x3: the inverse products in the reflection-folded form (half the
  // output tiles, each from the even- and odd-mode sums); bf16x6 dense
  const bool fold_inv = c->prec == QN_PREC_BF16X3;
  auto add = [&](int kind, int axis, int kid, const void* in, void* out, int m, int ncols, int batch,
                 long long bstride, int epi, const EpiArgs& e) {
    FoldStep f{};
    f.kind = kind;
    f.axis = axis;
    f.kid = kid;
    f.in = in;
    f.out = out;
    f.m = m;
    f.k = px;
    if (fold_inv && (kid == K_GEMM_YZ_INV || kid == K_GEMM_X_UPDATE)) f.nmir = c->n[axis];
    f.ncols = ncols;
    f.batch = batch;
    f.bstride = bstride;
    f.rows = rows;
    f.epi = epi;
    f.ep = e;
    st[ns++] = f;
  };
  if (c->fwdfold) {
    // folded forward y and z products: the x product writes its output folded
    // along z, the z product reads it and writes its output folded along y,
    // the y product reads that and divides; the inverse products are the
    // folded ones below
    const int hy = c->hp[1], hz = c->hp[2];
    add(DK_RIGHT, 0, K_GEMM_X, W1, W2, 0, 0, 0, 0, EPI_STORE, ep);
    st[ns - 1].sp = BfSplit{3, c->xfold ? c->hp[0] : 0, hz};  // from the x-folded residual
    st[ns - 1].sop = c->xfold ? 1 : 0;
    add(DK_LEFT, 2, K_GEMM_YZ, W2, W1, pz, (int)yslab, c->ncomp, zslab, EPI_STORE, ep);
    st[ns - 1].sp = BfSplit{2, hz, hy};
    st[ns - 1].sop = 1;
    EpiArgs ed = ep;
    ed.lamM = c->at<double>(c->off_lam[1]);
    ed.lamY = nullptr;
    ed.lamB = c->at<double>(c->off_lam[2]);
    add(DK_LEFT, 1, K_GEMM_DIVIDE, W1, W2, py, px, c->ncomp * pz, yslab, EPI_DIVIDE, ed);
    st[ns - 1].sp = BfSplit{1, hy, 0};
    st[ns - 1].sop = 1;
    add(DK_LEFT, 2, K_GEMM_YZ_INV, W2, W1, pz, (int)yslab, c->ncomp, zslab, EPI_STORE, ep);
    add(DK_LEFT, 1, K_GEMM_YZ_INV, W1, W2, py, px, c->ncomp * pz, yslab, EPI_STORE, ep);
    add(DK_RIGHT, 0, K_GEMM_X_UPDATE, W2, W1, 0, 0, 0, 0, epi_last, ep);
    return ns;
  }
  add(DK_RIGHT, 0, K_GEMM_X, W1, W2, 0, 0, 0, 0, EPI_STORE, ep);
  if (c->dim == 2) {
    EpiArgs ed = ep;
    ed.lamM = c->at<double>(c->off_lam[1]);
    ed.lamY = nullptr;
    add(DK_LEFT, 1, K_GEMM_DIVIDE, W2, W1, py, px, c->ncomp, yslab, EPI_DIVIDE, ed);
    add(DK_LEFT, 1, K_GEMM_YZ_INV, W1, W2, py, px, c->ncomp, yslab, EPI_STORE, ep);
  } else {
    add(DK_LEFT, 1, K_GEMM_YZ, W2, W1, py, px, c->ncomp * pz, yslab, EPI_STORE, ep);
    EpiArgs ed = ep;
    ed.lamM = c->at<double>(c->off_lam[2]);
    ed.lamY = c->at<double>(c->off_lam[1]);
    add(DK_LEFT, 2, K_GEMM_DIVIDE, W1, W2, pz, (int)yslab, c->ncomp, zslab, EPI_DIVIDE, ed);
    add(DK_LEFT, 2, K_GEMM_YZ_INV, W2, W1, pz, (int)yslab, c->ncomp, zslab, EPI_STORE, ep);
    add(DK_LEFT, 1, K_GEMM_YZ_INV, W1, W2, py, px, c->ncomp * pz, yslab, EPI_STORE, ep);
  }
  add(DK_RIGHT, 0, K_GEMM_X_UPDATE, W2, W1, 0, 0, 0, 0, epi_last, ep);
  return ns;
}

int solve_plan(qn_ctx c, const EpiArgs& ep, int epi_last, FoldStep* st) {
  return c->fold ? fold_plan(c, ep, epi_last, st) : dense_plan(c, ep, epi_last, st);
}

hipError_t run_step(qn_ctx c, const FoldStep& f, const FoldTile& t) {
  // folded split-bf16 inverse: output rows / columns [0, ceil(n / 2)) rounded up to the tile
  auto fold = [&](int side) { return f.nmir ? ((f.nmir + 1) / 2 + side - 1) / side * side : 0; };
  const BfSplit* sp = f.sp.mode ? &f.sp : nullptr;
  if (f.kind == DK_RIGHT)
    return launch_gemm_right(c->prec, operands(c, f.axis, f.sop), f.in, f.out, f.rows, f.k, f.epi,
                             f.ep, t.tm, t.tn, c->stream, fold(t.tn), f.nmir, sp);
  if (f.kind == DK_LEFT)
    return launch_gemm_left(c->prec, operands(c, f.axis, f.sop), f.in, f.out, f.m, f.ncols, f.batch,
                            f.bstride, f.epi, f.ep, t.tm, t.tn, c->stream, fold(t.tm), f.nmir, sp);
  return launch_fold(f.kind, c->prec, fold_ops(c, f.axis), f.in, f.out, c->ax[f.axis], f.ncols,
                     f.batch, f.bstride, f.rows, f.epi, f.ep, t, c->stream);
}

// Extents a dense tile must divide.
void dense_extents(const FoldStep& f, long long* mext, long long* next) {
  *mext = f.kind == DK_RIGHT ? f.rows : f.m;
  *next = f.kind == DK_RIGHT ? f.k : f.ncols;
  if (f.sp.mode == 3) *mext = 2LL * f.ep.py;  // half tiles of TM / 2 rows per plane
  if (f.sp.mode == 3 && f.sp.K > 0) *next = f.sp.K;  // tiles in one half of the x-folded rows
  if (f.sp.mode == 2 || (f.sp.mode == 1 && !f.nmir)) *mext = f.sp.K;  // tiles in one half
  if (f.sp.mode == 2) *next = 2LL * f.ep.px;  // half tiles of TN / 2 x values per row
}

// Smallest tile sides of a dense launch: the folded-output forms pair the
// halves of each wave's fragment blocks.
bool dense_tile_ok(const FoldStep& f, int tm, int tn) {
  return !(f.sp.mode == 3 && tm < 64) && !(f.sp.mode == 2 && tn < 64);
}

// Every instantiated tile that fits launch f (at most 16).
int step_candidates(qn_ctx c, const FoldStep& f, FoldTile* out) {
  int n = 0;
  long long mext, next;
  if (!c->fold) {
    dense_extents(f, &mext, &next);
    const int cap = gemm_bf_max_tile(c->prec);
    for (int tm = 32; tm <= cap; tm *= 2)
      for (int tn = 32; tn <= cap; tn *= 2)
        if (mext % tm == 0 && next % tn == 0 && dense_tile_ok(f, tm, tn)) out[n++] = FoldTile{tm, tn, 0, 0};
    return n;
  }
  const FoldTile* list;
  const int nc = fold_tiles(f.kind, &list);
  for (int i = 0; i < nc && n < 16; ++i)
    if (fold_tile_fits(f.kind, list[i], c->ax[f.axis].bk, f.ncols, f.rows)) out[n++] = list[i];
  return n;
}

// Tile of launch i of the plan: the autotuned one, else the default rule.
FoldTile step_tile(qn_ctx c, const FoldStep& f, int i) {
  if (c->tuned) return c->tile[i];
  if (!c->fold) {
    long long mext, next;
    dense_extents(f, &mext, &next);
    const int cap = gemm_bf_max_tile(c->prec);
    return FoldTile{pick_tile(mext, cap), pick_tile(next, cap), 0, 0};
  }
  return pick_fold_tile(f.kind, c->ax[f.axis].bk, f.ncols, f.batch, f.rows);
}

EpiArgs epi_args(qn_ctx c, const double* coef, double* dense) {
  EpiArgs ep{};
  ep.inst_mod = 1;
  ep.coef = coef;
  ep.dense = dense;
  ep.px = c->p[0];
  ep.py = c->p[1];
  ep.pz = c->p[2];
  ep.nx = c->n[0];
  ep.ny = c->n[1];
  ep.nz = c->n[2];
  ep.lamX = c->at<double>(c->off_lam[0]);
  ep.step = c->step;
  if (c->nl == QN_NL_GRAYSCOTT) {  // 2D: the divide's slab index is the component
    ep.cscale = c->at<double>(c->off_cscale);
    ep.comp_div = 1;
  }
  return ep;
}

// skip (device int, may be NULL): when set, every launch of the solve exits
// at once (the quasi-Newton loop has stopped).
hipError_t solve_ws(qn_ctx c, const double* coef, double* dense, int epi_last,
                    const int* skip = nullptr, const double* uscale = nullptr) {
  EpiArgs ep = epi_args(c, coef, dense);
  ep.skip = skip;
  ep.uscale = uscale;
  FoldStep st[6];
  const int ns = solve_plan(c, ep, epi_last, st);
  for (int i = 0; i < ns; ++i) {
    const FoldStep& f = st[i];
    const FoldTile t = step_tile(c, f, i);
    const hipError_t e = timed(c, f.kid, [&] { return run_step(c, f, t); });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

// ---------------------------------------------------------------------------
// Allocation-free residual.  The workgroup partials of the residual launch
// and the finalize kernel's scalars live in `scratch`, a fixed array of this
// library's code object (each device holds its own copy from the first call
// on it until the process ends), instead of the bound workspace.  Host code
// never uses the array's name as a device address: the address comes from
// hipGetSymbolAddress, taken once per device with that device current.
namespace {
constexpr size_t kNoAllocSlots = QN_NOALLOC_MAX_BLOCKS;  // workgroups of one residual launch
constexpr size_t kNoAllocPartialBytes = kNoAllocSlots * 4 * sizeof(double);
constexpr size_t kNoAllocBytes = kNoAllocPartialBytes + ((sizeof(DevScalars) + 255) / 256) * 256;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) char scratch[kNoAllocBytes];

namespace {
// Device address of `scratch` on the current device (resolved once per device).
hipError_t noalloc_scratch(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

extern "C" {

qn_status qn_setup(const qn_grid* grid, double beta, int32_t nonlinearity, const qn_options* opt,
                   qn_ctx* out) {
  if (!grid || !out) return fail(QN_ERR_INVALID, "null grid or output pointer");
  if (grid->dim != 2 && grid->dim != 3) return fail(QN_ERR_INVALID, "dim must be 2 or 3");
  for (int a = 0; a < grid->dim; ++a)
    if (grid->n[a] < 1 || grid->n[a] > 4096)
      return fail(QN_ERR_INVALID, "n[%d] = %d out of range [1, 4096]", a, grid->n[a]);
  if (nonlinearity < 0 || nonlinearity > 3) return fail(QN_ERR_INVALID, "unknown nonlinearity");
  const int want_comp =
      (nonlinearity == QN_NL_SYS2_CUBIC || nonlinearity == QN_NL_GRAYSCOTT) ? 2 : 1;
  if (grid->ncomp != want_comp)
    return fail(QN_ERR_INVALID, "ncomp = %d but the nonlinearity needs %d", grid->ncomp,
                want_comp);
  qn_options o{};
  if (opt) o = *opt;
  if (o.precision < 0 || o.precision > 3) return fail(QN_ERR_INVALID, "unknown precision");
  if (o.beta_mode < 0 || o.beta_mode > 4) return fail(QN_ERR_INVALID, "unknown beta_mode");
  if (nonlinearity == QN_NL_QUASILIN && o.beta_mode != QN_BETA_FIXED)
    return fail(QN_ERR_INVALID, "the quasi-linear problem uses the coefficient midpoint rule "
                                "and a fixed beta; only QN_BETA_FIXED is accepted");
  if (!std::isfinite(beta)) return fail(QN_ERR_INVALID, "beta is not finite");
  if (o.boundary != QN_BC_DIRICHLET && o.boundary != QN_BC_NEUMANN)
    return fail(QN_ERR_INVALID, "unknown boundary condition");
  const double length = o.length == 0.0 ? 1.0 : o.length;
  if (!(length > 0.0) || !std::isfinite(length))
    return fail(QN_ERR_INVALID, "length must be positive and finite");
  if (!std::isfinite(o.lin)) return fail(QN_ERR_INVALID, "lin is not finite");
  if (o.lin != 0.0 && nonlinearity != QN_NL_CUBIC)
    return fail(QN_ERR_INVALID, "a linear coefficient is supported for QN_NL_CUBIC only");
  if (!std::isfinite(o.cub)) return fail(QN_ERR_INVALID, "cub is not finite");
  // 0 selects the default coefficient 1; a magnitude below 1e-200 selects 0
  const double cub = o.cub == 0.0 ? 1.0 : (std::fabs(o.cub) < 1e-200 ? 0.0 : o.cub);
  if (!std::isfinite(o.quad)) return fail(QN_ERR_INVALID, "quad is not finite");
  if ((cub != 1.0 || o.quad != 0.0 || o.potential) && nonlinearity != QN_NL_CUBIC)
    return fail(QN_ERR_INVALID, "cubic / quadratic coefficients and a potential are supported "
                                "for QN_NL_CUBIC only");
  const double step = o.step == 0.0 ? 1.0 : o.step;
  if (!(step > 0.0) || !std::isfinite(step))
    return fail(QN_ERR_INVALID, "step must be positive and finite");
  double gs[4] = {o.gs_da, o.gs_ds, o.gs_rho, o.gs_mu};
  if (nonlinearity == QN_NL_GRAYSCOTT) {
    const double paper[4] = {2.5e-4, 5e-4, 0.04, 0.065};  // Section 6.2
    for (int i = 0; i < 4; ++i) {
      if (gs[i] == 0.0) gs[i] = paper[i];
      if (!(gs[i] > 0.0) || !std::isfinite(gs[i]))
        return fail(QN_ERR_INVALID, "Gray-Scott parameters must be positive and finite");
    }
    if (grid->dim != 2)
      return fail(QN_ERR_UNSUPPORTED, "the Gray-Scott system is built for 2D grids");
    if (o.boundary != QN_BC_NEUMANN)
      return fail(QN_ERR_UNSUPPORTED, "the Gray-Scott system is built with Neumann data");
  } else if (gs[0] != 0.0 || gs[1] != 0.0 || gs[2] != 0.0 || gs[3] != 0.0) {
    return fail(QN_ERR_INVALID, "Gray-Scott parameters given for another nonlinearity");
  }
  if (o.boundary == QN_BC_NEUMANN) {
    if (nonlinearity != QN_NL_CUBIC && nonlinearity != QN_NL_GRAYSCOTT)
      return fail(QN_ERR_UNSUPPORTED,
                  "Neumann data is supported for QN_NL_CUBIC and QN_NL_GRAYSCOTT only");
    if (o.precision != QN_PREC_FP64 && o.precision != QN_PREC_FP32)
      return fail(QN_ERR_UNSUPPORTED, "Neumann data is supported with FP64 and FP32 transforms");
    for (int a = 0; a < grid->dim; ++a)
      if (grid->n[a] < 2) return fail(QN_ERR_INVALID, "Neumann data needs n >= 2 per axis");
  }
  if (o.discretization != QN_DISC_FD && o.discretization != QN_DISC_SEM)
    return fail(QN_ERR_INVALID, "unknown discretization");
  if (o.discretization == QN_DISC_SEM) {
    if (nonlinearity != QN_NL_CUBIC)
      return fail(QN_ERR_UNSUPPORTED, "spectral elements are supported for QN_NL_CUBIC only");
    if (o.precision != QN_PREC_FP64 && o.precision != QN_PREC_FP32)
      return fail(QN_ERR_UNSUPPORTED, "spectral elements need FP64 or FP32 transforms");
    const int k = o.sem_order;
    if (k < 1 || k > 8) return fail(QN_ERR_INVALID, "sem_order = %d out of range [1, 8]", k);
    for (int a = 0; a < grid->dim; ++a) {
      const int n = grid->n[a];
      const bool neu = o.boundary == QN_BC_NEUMANN;
      const int rem = neu ? (n - 1) % k : (n + 1) % k;
      const int elements = neu ? (n - 1) / k : (n + 1) / k;
      if (rem != 0 || elements < 1 || n < 1 || n > 1025)
        return fail(QN_ERR_INVALID,
                    "n[%d] = %d is not E k %s 1 nodes with E >= 1 elements of order %d "
                    "(and at most 1025)", a, n, neu ? "+" : "-", k);
    }
  }

  qn_ctx c = new qn_ctx_s();
  c->dim = grid->dim;
  c->ncomp = grid->ncomp;
  c->nl = nonlinearity;
  c->prec = o.precision;
  c->beta_mode = o.beta_mode;
  c->timing = o.timing;
  c->beta = beta;
  c->stream = (hipStream_t)o.stream;
  c->n[0] = grid->n[0];
  c->n[1] = grid->n[1];
  c->n[2] = grid->dim == 3 ? grid->n[2] : 1;
  c->fold = c->prec == QN_PREC_FP64 || c->prec == QN_PREC_FP32;
  c->bc = o.boundary;
  c->length = length;
  c->lin = o.lin;
  c->cub = cub;
  c->quad = o.quad;
  c->pot = o.potential;
  c->sem_k = o.discretization == QN_DISC_SEM ? o.sem_order : 0;
  c->step = step;
  for (int i = 0; i < 4; ++i) c->gs[i] = gs[i];
  c->lam_min_sum = 0.0;
  for (int a = 0; a < 3; ++a) {
    if (a >= c->dim) {
      c->p[a] = 1;
      continue;
    }
    const int n = c->n[a];
    // 1 / h: n interior nodes (Dirichlet, h = L/(n+1)) or n nodes with both
    // ends (Neumann, h = L/(n-1)); exact integers on the unit interval
    const double ih = (c->bc == QN_BC_NEUMANN ? n - 1 : n + 1) / length;
    c->ih2[a] = ih * ih;
    c->hvol /= ih;
    if (c->sem_k > 0) {  // spectral elements: Jacobi on the even and odd halves
      const int k = c->sem_k, bk = fold_block(n);
      const int elements = c->bc == QN_BC_NEUMANN ? (n - 1) / k : (n + 1) / k;
      c->ax[a] = FoldAxis{n, n / 2, n & 1, bk};
      c->p[a] = 2 * bk;
      int same = -1;  // an earlier axis of the same length has the same data
      for (int b = 0; b < a; ++b)
        if (c->n[b] == n) same = b;
      if (same >= 0) {
        c->hx[a] = c->hx[same];
        c->hS[a] = c->hS[same];
        c->hlam[a] = c->hlam[same];
        c->hHb[a] = c->hHb[same];
        c->lam_min_sum += c->sem_lmin[same];
        c->sem_lmin[a] = c->sem_lmin[same];
        continue;
      }
      std::vector<double> m, S;
      sem_axis(elements, k, length, c->bc == QN_BC_NEUMANN, m, S, &c->hx[a]);
      c->sem_lmin[a] = fold_sem(n, m, S, bk, c->hS[a], c->hlam[a]);
      c->lam_min_sum += c->sem_lmin[a];
      sem_band(n, k, m, S, c->hHb[a]);
      continue;
    }
    c->hx[a].resize((size_t)n);
    for (int i = 0; i < n; ++i) c->hx[a][i] = (c->bc == QN_BC_NEUMANN ? i : i + 1) / ih;
    if (c->fold) {
      const int bk = fold_block(n);
      c->ax[a] = FoldAxis{n, n / 2, n & 1, bk};
      c->p[a] = 2 * bk;
      if (c->bc == QN_BC_NEUMANN)
        fold_cosine(n, c->ih2[a], bk, c->hS[a], c->hlam[a]);
      else
        fold_eigen(n, bk, c->hS[a], c->hlam[a]);
    } else {
      c->p[a] = ((n + 31) / 32) * 32;
      dense_eigen(n, c->p[a], c->hS[a], c->hlam[a]);
    }
    // the sine eigenvalues are for the unit interval: h = 1 / (n + 1)
    if (c->bc == QN_BC_DIRICHLET && length != 1.0)
      for (double& l : c->hlam[a]) l /= length * length;
    c->lam_min_sum += c->hlam[a][0];  // lam_1 (Dirichlet) or 0 (Neumann) leads both orderings
  }
  // 3D bf16x3: the forward y and z products run folded when both axes fit it
  c->fwdfold = c->prec == QN_PREC_BF16X3 && c->dim == 3 && c->sem_k == 0 && c->bc == QN_BC_DIRICHLET;
  for (int a = 1; a < 3 && c->fwdfold; ++a)
    c->fwdfold = 2 * fold_half(c->n[a]) == c->p[a];
  // x as well when the residual's tiles cover whole rows (the mirror pairs
  // meet in one workgroup) and its folded variant keeps its registers
  // (quasi-linear and 2-component problems; the cubic one would spill)
  c->xfold = c->fwdfold && (c->nl == QN_NL_QUASILIN || c->nl == QN_NL_SYS2_CUBIC) &&
             2 * fold_half(c->n[0]) == c->p[0] &&
             residual_tile_x(c->p[0], residual_threads(c->nl, c->bc)) == c->p[0];
  for (int a = c->xfold ? 0 : 1; a < 3 && c->fwdfold; ++a) {
    c->hp[a] = fold_half(c->n[a]);
    fold_forward(c->n[a], c->p[a], c->hS[a], c->hSf[a]);
  }
  // Gray-Scott: component c solves with D_c A_h, so the smallest eigenvalue
  // of the solve operator's linear part is min(D_A, D_S) lam_min(A_h).
  if (c->nl == QN_NL_GRAYSCOTT) c->lam_min_sum *= std::min(c->gs[0], c->gs[1]);
  // The fixed beta must give a positive definite solve operator (Section 5:
  // beta > -lam_min(A_h)).  The midpoint rules produce beta >= 0 here.
  if (o.beta_mode == QN_BETA_FIXED && c->lam_min_sum + beta <= 0.0) {
    const double lmin = c->lam_min_sum;
    delete c;
    return fail(QN_ERR_INVALID, "beta = %g makes A_h + beta I singular or indefinite "
                                "(lam_min(A_h) = %g)", beta, lmin);
  }

  size_t off = 0;
  for (int a = 0; a < c->dim; ++a) {
    const size_t pp = c->hS[a].size();  // p*p dense, or 4 bk^2 = p*p folded
    const size_t eb = c->prec == QN_PREC_FP64 ? 8 : (c->prec == QN_PREC_FP32 ? 4 : 2);
    c->off_S[a] = off;
    off += align256(pp * eb);
    if (!c->fold) {  // further bf16 parts
      c->off_Slo[a] = off;
      off += align256(pp * 2);
      if (c->prec == QN_PREC_BF16X6) {
        c->off_Slo2[a] = off;
        off += align256(pp * 2);
      }
    }
    c->off_lam[a] = off;
    off += align256((size_t)c->p[a] * 8);
    if (c->sem_k > 0) {
      c->off_Hb[a] = off;
      off += align256(c->hHb[a].size() * 8);
    }
  }
  for (int a = c->xfold ? 0 : 1; a < 3 && c->fwdfold; ++a)
    for (int q = 0; q < 2; ++q) {
      c->off_Sf[a][q] = off;
      off += align256(c->hSf[a].size() * 2);
    }
  if (c->dim == 2) {  // unused z axis aliases y (never read)
    c->off_S[2] = c->off_S[1];
    c->off_Slo[2] = c->off_Slo[1];
    c->off_Slo2[2] = c->off_Slo2[1];
    c->off_lam[2] = c->off_lam[1];
    c->ax[2] = c->ax[1];
  }
  c->off_W1 = off;
  off += align256(c->tensor_elems() * c->elem());
  c->off_W2 = off;
  off += align256(c->tensor_elems() * c->elem());
  // partial slots for both residual launches: padded (the iteration) and
  // interior (qn_residual) extents
  const int rt = residual_threads(c->nl, c->bc);
  if (c->dim == 3)
    c->max_blocks = std::max(  // padded extents (transform workspace) and a caller's R
        residual_max_blocks(c->p[0], c->p[1], c->p[2],
                            residual_slab_depth(c->p[0], c->p[1], c->p[2], rt), false, rt),
        residual_max_blocks(c->n[0], c->n[1], c->n[2],
                            residual_slab_depth(c->n[0], c->n[1], c->n[2], rt), false, rt));
  else
    c->max_blocks = std::max(
        residual_max_blocks(c->p[0], c->p[1], 1, residual_planar_rows(c->p[0], c->p[1]), true),
        residual_max_blocks(c->n[0], c->n[1], 1, residual_planar_rows(c->n[0], c->n[1]), true));
  if (c->sem_k > 0)
    c->max_blocks =
        std::max({c->max_blocks, sem_residual_blocks(c->dim, c->p[0], c->p[1], c->p[2]),
                  sem_residual_blocks(c->dim, c->n[0], c->n[1], c->n[2])});
  c->off_part = off;
  off += align256((size_t)c->max_blocks * 4 * sizeof(double));
  c->off_scal = off;
  off += align256(sizeof(DevScalars));
  c->off_coef = off;
  off += align256(2 * sizeof(double));
  c->off_cscale = off;  // Gray-Scott: per-component diffusion {D_A, D_S}
  off += align256(2 * sizeof(double));
  c->need = off;
  *out = c;
  return QN_OK;
}

qn_status qn_workspace_bytes(qn_ctx ctx, size_t* bytes) {
  if (!ctx || !bytes) return fail(QN_ERR_INVALID, "null argument");
  *bytes = ctx->need;
  return QN_OK;
}

qn_status qn_bind_workspace(qn_ctx c, void* d_ws, size_t bytes) {
  qn_status s = check_ctx(c, false);
  if (s != QN_OK) return s;
  if (!d_ws) return fail(QN_ERR_WORKSPACE, "null workspace");
  if (((uintptr_t)d_ws & 255u) != 0) return fail(QN_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (bytes < c->need)
    return fail(QN_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", bytes, c->need);
  c->ws = (char*)d_ws;
  hipError_t e = hipSuccess;
  if (!c->hring) {
    // coherent: the finalize kernel writes the slots directly, the host reads
    // them once the slot's event has completed
    e = hipHostMalloc((void**)&c->hring, 2 * sizeof(DevScalars), hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&c->dring, c->hring, 0);
  }
  for (int i = 0; i < 2 && e == hipSuccess; ++i)
    if (!c->ring_ev[i]) e = hipEventCreateWithFlags(&c->ring_ev[i], hipEventDisableTiming);
  if (e != hipSuccess) return hip_fail(c, e, "iteration read-back buffers");
  e = launch_zero(c->ws, c->need, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "zero workspace");
  for (int a = 0; a < c->dim; ++a) {
    const size_t pp = c->hS[a].size();
    if (c->prec == QN_PREC_FP64) {
      e = hipMemcpyAsync(c->ws + c->off_S[a], c->hS[a].data(), pp * 8, hipMemcpyHostToDevice,
                         c->stream);
    } else if (c->prec == QN_PREC_FP32) {
      std::vector<float> s32(pp);
      for (size_t i = 0; i < pp; ++i) s32[i] = (float)c->hS[a][i];
      e = hipMemcpyAsync(c->ws + c->off_S[a], s32.data(), pp * 4, hipMemcpyHostToDevice, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // s32 is a host temporary
    } else {
      // S = s0 + s1 (+ s2), each part the RNE bf16 of what the previous ones leave
      const int np = c->prec == QN_PREC_BF16X6 ? 3 : 2;
      std::vector<uint16_t> parts[3];
      for (int q = 0; q < np; ++q) parts[q].resize(pp);
      for (size_t i = 0; i < pp; ++i) {
        float r = (float)c->hS[a][i];
        for (int q = 0; q < np; ++q) {
          parts[q][i] = bf16_rne(r);
          r -= bf16_value(parts[q][i]);
        }
      }
      const size_t offs[3] = {c->off_S[a], c->off_Slo[a], c->off_Slo2[a]};
      for (int q = 0; q < np && e == hipSuccess; ++q)
        e = hipMemcpyAsync(c->ws + offs[q], parts[q].data(), pp * 2, hipMemcpyHostToDevice,
                           c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // host temporaries
      if (!c->hSf[a].empty() && e == hipSuccess) {  // folded forward operand: bf16 parts
        const std::vector<double>& v = c->hSf[a];
        std::vector<uint16_t> sp[2];
        sp[0].resize(v.size());
        sp[1].resize(v.size());
        for (size_t i = 0; i < v.size(); ++i) {
          const float r = (float)v[i];
          sp[0][i] = bf16_rne(r);
          sp[1][i] = bf16_rne(r - bf16_value(sp[0][i]));
        }
        for (int q = 0; q < 2 && e == hipSuccess; ++q)
          e = hipMemcpyAsync(c->ws + c->off_Sf[a][q], sp[q].data(), v.size() * 2,
                             hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // host temporaries
      }
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->ws + c->off_lam[a], c->hlam[a].data(), (size_t)c->p[a] * 8,
                         hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && c->sem_k > 0)
      e = hipMemcpyAsync(c->ws + c->off_Hb[a], c->hHb[a].data(), c->hHb[a].size() * 8,
                         hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "upload eigen-data");
  }
  if (c->nl == QN_NL_GRAYSCOTT) {
    e = hipMemcpyAsync(c->ws + c->off_cscale, c->gs, 2 * sizeof(double), hipMemcpyHostToDevice,
                       c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "upload diffusion coefficients");
  }
  // hS/hlam/gs stay alive in the context, so the async uploads above are safe.
  return QN_OK;
}

qn_status qn_set_stream(qn_ctx c, void* stream) {
  if (!c) return fail(QN_ERR_INVALID, "null context");
  c->stream = (hipStream_t)stream;
  return QN_OK;
}

qn_status qn_residual(qn_ctx c, const double* d_U, const double* d_F, double* d_R, double* d_red) {
  qn_status s = check_ctx(c, true);
  if (s != QN_OK) return s;
  if (!d_U || !d_F || !d_R) return fail(QN_ERR_INVALID, "null U, F or R");
  if (!aligned8(d_U) || !aligned8(d_F) || !aligned8(d_R) || (d_red && !aligned8(d_red)))
    return fail(QN_ERR_INVALID, "pointers must be 8-byte aligned");
  if (d_R == d_U) return fail(QN_ERR_INVALID, "R may not alias U");
  ResidualArgs a = residual_args(c, d_U, d_F, d_R);
  int nb = 0;
  hipError_t e = timed(c, K_RESIDUAL, [&] { return launch_any_residual(a, &nb, c->stream); });
  if (e == hipSuccess)
    e = timed(c, K_FINALIZE, [&] {
      return launch_finalize(a.partials, nb, c->scal(), rule_of(c), c->beta, c->lam_min_sum, d_red,
                             0.0, -1, 0, c->stream);
    });
  if (e != hipSuccess) return hip_fail(c, e, "residual launch");
  return QN_OK;
}

qn_status qn_residual_noalloc(qn_ctx c, const double* d_U, const double* d_F, double* d_R,
                              double* d_red) {
  qn_status s = check_ctx(c, false);
  if (s != QN_OK) return s;
  if (c->sem_k > 0)
    return fail(QN_ERR_UNSUPPORTED,
                "qn_residual_noalloc: spectral elements keep their operator bands in the workspace");
  // The capacity check comes before the pointer checks, so that a grid the
  // fixed array cannot hold is refused whatever the pointers are.  The
  // launch's workgroup count, as residual_args and launch_residual form it
  // for a caller's R (unpadded extents).
  const bool planar = c->dim != 3;
  const int rt = residual_threads(c->nl, c->bc);
  const int blocks = residual_max_blocks(
      c->n[0], c->n[1], c->n[2],
      planar ? residual_planar_rows(c->n[0], c->n[1])
             : residual_slab_depth(c->n[0], c->n[1], c->n[2], rt),
      planar, rt);
  if (blocks < 0 || (size_t)blocks > kNoAllocSlots)
    return fail(QN_ERR_WORKSPACE,
                "qn_residual_noalloc: the grid needs %d workgroup partials, the static scratch "
                "holds %zu (use qn_residual with a bound workspace)",
                blocks, kNoAllocSlots);
  if (!d_U || !d_F || !d_R) return fail(QN_ERR_INVALID, "null U, F or R");
  if (!aligned8(d_U) || !aligned8(d_F) || !aligned8(d_R) || (d_red && !aligned8(d_red)))
    return fail(QN_ERR_INVALID, "pointers must be 8-byte aligned");
  if (d_R == d_U) return fail(QN_ERR_INVALID, "R may not alias U");
  ResidualArgs a = residual_args(c, d_U, d_F, d_R);
  // the launch's own grid, which the partials slots must cover
  const int launch_blocks = residual_max_blocks(a.ox, a.oy, a.oz, a.rz, a.ihz2 == 0.0, rt);
  if (launch_blocks < 0 || (size_t)launch_blocks > kNoAllocSlots)
    return fail(QN_ERR_WORKSPACE, "qn_residual_noalloc: the grid needs %d workgroup partials",
                launch_blocks);
  char* base = nullptr;
  hipError_t e = noalloc_scratch(&base);
  if (e != hipSuccess) return hip_fail(c, e, "qn_residual_noalloc: scratch address");
  a.partials = reinterpret_cast<double*>(base);
  DevScalars* sc = reinterpret_cast<DevScalars*>(base + kNoAllocPartialBytes);
  // launched without the timing events of qn_residual (they would be created on demand)
  int nb = 0;
  e = launch_any_residual(a, &nb, c->stream);
  if (e == hipSuccess)
    e = launch_finalize(a.partials, nb, sc, rule_of(c), c->beta, c->lam_min_sum, d_red, 0.0, -1, 0,
                        c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "qn_residual_noalloc launch");
  return QN_OK;
}

qn_status qn_fdm_solve(qn_ctx c, const double* d_R, double scale, double shift, double* d_X) {
  qn_status s = check_ctx(c, true);
  if (s != QN_OK) return s;
  if (!d_R || !d_X) return fail(QN_ERR_INVALID, "null R or X");
  if (!aligned8(d_R) || !aligned8(d_X)) return fail(QN_ERR_INVALID, "pointers must be 8-byte aligned");
  if (!(scale > 0.0) || !std::isfinite(scale) || !std::isfinite(shift))
    return fail(QN_ERR_INVALID, "scale must be positive and finite, shift finite");
  if (scale * c->lam_min_sum + shift <= 0.0)
    return fail(QN_ERR_INVALID, "scale*lam_min(A_h) + shift = %g <= 0: singular or indefinite",
                scale * c->lam_min_sum + shift);
  double* coef = c->at<double>(c->off_coef);
  hipError_t e = launch_set_coef(coef, scale, shift, c->stream);
  if (e == hipSuccess)
    e = timed(c, K_PAD_COPY, [&] {
      return launch_pad_copy(d_R, c->ws + c->off_W1, transform_storage(c->prec), c->ncomp,
                             c->n[0], c->n[1], c->n[2], c->p[0], c->p[1], c->p[2], c->stream,
                             c->xfold ? c->hp[0] : 0);
    });
  if (e == hipSuccess) e = solve_ws(c, coef, d_X, EPI_STORE_DENSE);
  if (e != hipSuccess) return hip_fail(c, e, "fdm solve launch");
  return QN_OK;
}

qn_status qn_iterate(qn_ctx c, double* d_U, const double* d_F, double rtol, int32_t max_iter,
                     qn_stats* stats) {
  qn_stats st{};
  st.status = QN_ERR_INVALID;
  auto finish = [&](qn_status s) {
    st.status = s;
    if (stats) *stats = st;
    return s;
  };
  qn_status s = check_ctx(c, true);
  if (s != QN_OK) return finish(s);
  if (!d_U || !d_F) return finish(fail(QN_ERR_INVALID, "null U or F"));
  if (!aligned8(d_U) || !aligned8(d_F)) return finish(fail(QN_ERR_INVALID, "pointers must be 8-byte aligned"));
  if (!(rtol >= 0.0) || max_iter < 0) return finish(fail(QN_ERR_INVALID, "rtol < 0 or max_iter < 0"));
  const auto t0 = std::chrono::steady_clock::now();
  auto elapsed = [&] {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  // Iteration k = residual + reductions + loop decision (finalize, on the
  // device), then the solve of step k.  The host runs one iteration ahead: it
  // enqueues iteration k + 1 (whose solve and residual skip themselves on the
  // device once iteration k decided to stop) before it reads iteration k's
  // scalars, so the GPU does not idle during the read-back.  Nothing is
  // enqueued past max_iter.  (The finalize after a skipped residual recomputes
  // the previous iteration's scalars from its partials, and nothing reads them.)
  const int* done = &c->scal()->done;
  auto enqueue = [&](int k) {
    hipError_t e = hipSuccess;
    if (k > 0) e = solve_ws(c, &c->scal()->scale, d_U, EPI_SUB_DENSE, done);
    // the finalize kernel also writes the scalars into host slot k & 1
    if (e == hipSuccess)
      e = residual_into_ws(c, d_U, d_F, nullptr, rtol, k, max_iter, k > 0 ? done : nullptr,
                           c->dring + (k & 1));
    if (e == hipSuccess) e = hipEventRecord(c->ring_ev[k & 1], c->stream);
    return e;
  };
  auto drain = [&](qn_status r) {
    const hipError_t e = hipStreamSynchronize(c->stream);
    st.seconds = elapsed();
    if (e != hipSuccess) return finish(hip_fail(c, e, "iteration"));
    return finish(r);
  };
  hipError_t e = enqueue(0);
  for (int k = 0; e == hipSuccess; ++k) {
    if (k < max_iter) e = enqueue(k + 1);
    if (e == hipSuccess) e = hipEventSynchronize(c->ring_ev[k & 1]);
    if (e != hipSuccess) break;
    const DevScalars h = c->hring[k & 1];
    if (k == 0) {
      if (h.sumsqF == 0.0)
        return drain(fail(QN_ERR_INVALID, "||F|| = 0: the relative stopping rule is undefined"));
      st.relres0 = h.relres;
    }
    st.relres = h.relres;
    st.iters = k;
    if (!std::isfinite(h.relres) || h.relres > 1e30)
      return drain(fail(QN_ERR_DIVERGED, "residual became non-finite or exploded at iteration %d", k));
    if (h.relres <= rtol) {
      g_err.clear();
      return drain(QN_OK);
    }
    if (k >= max_iter)
      return drain(fail(QN_ERR_NOT_CONVERGED, "no convergence in %d solves (relres %.3e)", k,
                        h.relres));
    if (h.flag != 0.0)
      return drain(fail(QN_ERR_DIVERGED, "shift rule produced a singular operator at iteration %d", k));
    st.beta_last = h.beta;
    st.scale_last = h.scale;
  }
  st.seconds = elapsed();
  return finish(hip_fail(c, e, "iteration"));
}

qn_status qn_nodes(qn_ctx c, int32_t axis, double* x) {
  if (!c || !x) return fail(QN_ERR_INVALID, "null argument");
  if (axis < 0 || axis >= c->dim) return fail(QN_ERR_INVALID, "axis %d out of range", axis);
  std::memcpy(x, c->hx[axis].data(), c->hx[axis].size() * sizeof(double));
  return QN_OK;
}

static qn_status eigen_check(qn_ctx c) {
  qn_status s = check_ctx(c, true);
  if (s != QN_OK) return s;
  if (c->nl != QN_NL_CUBIC || !c->fold || c->sem_k > 0 || c->quad != 0.0)
    return fail(QN_ERR_UNSUPPORTED, "the eigenproblem needs QN_NL_CUBIC without a quadratic "
                                    "term, finite differences and FP64 or FP32 transforms");
  return QN_OK;
}

qn_status qn_eigen_residual(qn_ctx c, const double* d_U, double* d_R, double* d_out) {
  qn_status s = eigen_check(c);
  if (s != QN_OK) return s;
  if (!d_U || !d_R) return fail(QN_ERR_INVALID, "null U or R");
  if (!aligned8(d_U) || !aligned8(d_R) || (d_out && !aligned8(d_out)))
    return fail(QN_ERR_INVALID, "pointers must be 8-byte aligned");
  if (d_R == d_U) return fail(QN_ERR_INVALID, "R may not alias U");
  const hipError_t e = eigen_residual(c, d_U, d_R, d_out, 0.0, -1, 0, nullptr, nullptr);
  if (e != hipSuccess) return hip_fail(c, e, "eigen residual launch");
  return QN_OK;
}

qn_status qn_eigen_iterate(qn_ctx c, double* d_U, double rtol, int32_t max_iter, qn_stats* stats,
                           double* lam_out) {
  qn_stats st{};
  st.status = QN_ERR_INVALID;
  double lam = std::nan("");
  auto finish = [&](qn_status s) {
    st.status = s;
    if (stats) *stats = st;
    if (lam_out) *lam_out = lam;
    return s;
  };
  qn_status s = eigen_check(c);
  if (s != QN_OK) return finish(s);
  if (!d_U) return finish(fail(QN_ERR_INVALID, "null U"));
  if (!aligned8(d_U)) return finish(fail(QN_ERR_INVALID, "pointers must be 8-byte aligned"));
  if (!(rtol >= 0.0) || max_iter < 0) return finish(fail(QN_ERR_INVALID, "rtol < 0 or max_iter < 0"));
  const auto t0 = std::chrono::steady_clock::now();
  // Same pipelining as qn_iterate.  Iteration k: the solve of step k - 1,
  // whose update epilogue forms U~_k = s_{k-1} U~_{k-1} - dU (the stored
  // iterate stays unnormalised), then the two residual passes at
  // U_k = s_k U~_k and the loop decision.  On return the stored iterate is
  // scaled once by the last s, so d_U holds the normalised U_k.
  const int* done = &c->scal()->done;
  auto enqueue = [&](int k) {
    hipError_t e = hipSuccess;
    if (k > 0)
      e = solve_ws(c, &c->scal()->scale, d_U, EPI_SUB_DENSE, done, &c->scal()->uscale);
    if (e == hipSuccess)
      e = eigen_residual(c, d_U, nullptr, nullptr, rtol, k, max_iter, k > 0 ? done : nullptr,
                         c->dring + (k & 1));
    if (e == hipSuccess) e = hipEventRecord(c->ring_ev[k & 1], c->stream);
    return e;
  };
  auto drain = [&](qn_status r) {
    const long long n = (long long)c->ncomp * c->n[2] * c->n[1] * c->n[0];
    hipError_t e = launch_scale(d_U, n, &c->scal()->uscale, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (e != hipSuccess) return finish(hip_fail(c, e, "eigen iteration"));
    return finish(r);
  };
  hipError_t e = enqueue(0);
  for (int k = 0; e == hipSuccess; ++k) {
    if (k < max_iter) e = enqueue(k + 1);
    if (e == hipSuccess) e = hipEventSynchronize(c->ring_ev[k & 1]);
    if (e != hipSuccess) break;
    const DevScalars h = c->hring[k & 1];
    if (k == 0) st.relres0 = h.relres;
    st.relres = h.relres;
    st.iters = k;
    lam = h.eig;
    if (!std::isfinite(h.relres) || h.relres > 1e30)
      return drain(fail(QN_ERR_DIVERGED, "eigen residual became non-finite at iteration %d", k));
    if (h.relres <= rtol) {
      g_err.clear();
      return drain(QN_OK);
    }
    if (k >= max_iter)
      return drain(fail(QN_ERR_NOT_CONVERGED, "no convergence in %d solves (relres %.3e)", k,
                        h.relres));
    if (h.flag != 0.0)
      return drain(fail(QN_ERR_DIVERGED,
                        "shift %.6g with lam_min(A_h) = %.6g is singular or indefinite at "
                        "iteration %d", h.beta, c->lam_min_sum, k));
    st.beta_last = h.beta;
    st.scale_last = h.scale;
  }
  st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return finish(hip_fail(c, e, "eigen iteration"));
}

qn_status qn_autotune(qn_ctx c) {
  qn_status s = check_ctx(c, true);
  if (s != QN_OK) return s;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipError_t e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  // finite transform contents; the coefficient slot holds {scale, shift} = {1, 1}
  const size_t tbytes = c->tensor_elems() * c->elem();
  if (e == hipSuccess) e = launch_zero(c->ws + c->off_W1, tbytes, c->stream);
  if (e == hipSuccess) e = launch_zero(c->ws + c->off_W2, tbytes, c->stream);
  double* coef = c->at<double>(c->off_coef);
  if (e == hipSuccess) e = launch_set_coef(coef, 1.0, 1.0, c->stream);
  FoldStep st[6];
  const int ns = solve_plan(c, epi_args(c, coef, nullptr), EPI_STORE, st);
  const bool was_tuned = c->tuned;
  c->tuned = false;  // step_tile gives the default rule below
  FoldTile best[6] = {};
  for (int i = 0; i < ns && e == hipSuccess; ++i) {
    const FoldStep& f = st[i];
    best[i] = step_tile(c, f, i);
    FoldTile cand[16];
    const int nc = step_candidates(c, f, cand);
    float best_ms = 1e30f;
    for (int k = 0; k < nc && e == hipSuccess; ++k) {
      const FoldTile t = cand[k];
      e = run_step(c, f, t);  // warm-up
      if (e == hipSuccess) e = hipEventRecord(t0, c->stream);
      for (int r = 0; r < 3 && e == hipSuccess; ++r) e = run_step(c, f, t);
      if (e == hipSuccess) e = hipEventRecord(t1, c->stream);
      if (e == hipSuccess) e = hipEventSynchronize(t1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
      if (e == hipSuccess && ms < best_ms) {
        best_ms = ms;
        best[i] = t;
      }
    }
  }
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  if (e != hipSuccess) {
    c->tuned = was_tuned;
    return hip_fail(c, e, "autotune");
  }
  for (int i = 0; i < 6; ++i) c->tile[i] = best[i];
  c->tuned = true;
  return QN_OK;
}

qn_status qn_tile_info(qn_ctx c, int32_t i, int32_t* info4) {
  qn_status s = check_ctx(c, true);
  if (s != QN_OK) return s;
  if (!info4) return fail(QN_ERR_INVALID, "null argument");
  FoldStep st[6];
  const int ns = solve_plan(c, epi_args(c, nullptr, nullptr), EPI_STORE, st);
  if (i < 0 || i >= ns) return fail(QN_ERR_INVALID, "launch index %d out of range [0, %d)", i, ns);
  const FoldTile t = step_tile(c, st[i], i);
  const int kid = st[i].kid;
  const int kind = kid == K_GEMM_X ? 0 : kid == K_GEMM_X_UPDATE ? 3 : kid == K_GEMM_YZ_INV ? 2 : 1;
  info4[0] = kind + (t.paired ? 4 : 0) + t.tk;
  info4[1] = st[i].axis;
  info4[2] = t.tm;
  info4[3] = t.tn;
  return QN_OK;
}

qn_status qn_set_tile(qn_ctx c, int32_t i, const int32_t* info4) {
  qn_status s = check_ctx(c, true);
  if (s != QN_OK) return s;
  if (!info4) return fail(QN_ERR_INVALID, "null argument");
  FoldStep st[6];
  const int ns = solve_plan(c, epi_args(c, nullptr, nullptr), EPI_STORE, st);
  if (i < 0 || i >= ns) return fail(QN_ERR_INVALID, "launch index %d out of range [0, %d)", i, ns);
  const int kid = st[i].kid;
  const int kind = kid == K_GEMM_X ? 0 : kid == K_GEMM_X_UPDATE ? 3 : kid == K_GEMM_YZ_INV ? 2 : 1;
  if ((info4[0] & 3) != kind || info4[1] != st[i].axis)
    return fail(QN_ERR_INVALID, "launch %d is kind %d on axis %d", i, kind, st[i].axis);
  FoldTile cand[16];
  const int nc = step_candidates(c, st[i], cand);
  for (int k = 0; k < nc; ++k) {
    const FoldTile& t = cand[k];
    const int flags = kind + (t.paired ? 4 : 0) + t.tk;
    if (flags == info4[0] && t.tm == info4[2] && t.tn == info4[3]) {
      if (!c->tuned)
        for (int j = 0; j < ns; ++j) c->tile[j] = step_tile(c, st[j], j);
      c->tile[i] = t;
      c->tuned = true;
      return QN_OK;
    }
  }
  return fail(QN_ERR_INVALID, "tile {%d, %d, %d, %d} is not an admissible shape of launch %d",
              info4[0], info4[1], info4[2], info4[3], i);
}

int32_t qn_timing_count(void) { return K_COUNT; }

qn_status qn_timing_read(qn_ctx c, int32_t i, const char** name, int64_t* launches,
                         double* total_ms) {
  if (!c) return fail(QN_ERR_INVALID, "null context");
  if (i < 0 || i >= K_COUNT) return fail(QN_ERR_INVALID, "timing index out of range");
  fold_timing(c);
  if (name) *name = kKernelNames[i];
  if (launches) *launches = c->launches[i];
  if (total_ms) *total_ms = c->tot_ms[i];
  return QN_OK;
}

qn_status qn_timing_reset(qn_ctx c) {
  if (!c) return fail(QN_ERR_INVALID, "null context");
  fold_timing(c);
  for (int i = 0; i < K_COUNT; ++i) {
    c->tot_ms[i] = 0.0;
    c->launches[i] = 0;
  }
  return QN_OK;
}

void qn_destroy(qn_ctx c) {
  if (!c) return;
  if (!c->pending.empty()) (void)hipStreamSynchronize(c->stream);
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  for (auto e : c->ring_ev)
    if (e) (void)hipEventDestroy(e);
  if (c->hring) (void)hipHostFree(c->hring);
  delete c;
}

const char* qn_last_error(void) { return g_err.c_str(); }

}  // extern "C"
