// Host side of the batched solver (include/qn_batched.h).
//
// Instances with equal (n, ncomp) form a class whose fields are stored as one
// (ncomp, K, n, n) block, and whose transform workspace is (ncomp, K, P, P)
// with P = n rounded up to 32.  With that layout the single-problem kernels
// cover a whole class per launch: the residual treats the K instances as
// z-planes (1/h_z^2 = 0, one plane per workgroup), the y products batch over
// the ncomp*K slabs, and the x products run over ncomp*K*P rows; per-instance
// skip flags and shift coefficients are looked up as slab or row index % K.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "../../include/qn_batched.h"
#include "qn_host.h"
#include "qn_internal.h"

namespace qn {
qn_status set_error(qn_status s, const char* fmt, ...);
}
using namespace qn;

namespace {

size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

int largest_tile(long long extent) {
  if (extent % 128 == 0) return 128;
  if (extent % 64 == 0) return 64;
  return 32;
}

struct Cls {
  int n = 0, p = 0, ncomp = 1, K = 0;
  std::vector<int> members;
  long long off_field = 0;  // element offset of the (ncomp, K, n, n) block
  size_t off_S = 0, off_Slo = 0, off_lam = 0, off_W1 = 0, off_W2 = 0, off_part = 0, off_state = 0,
         off_done = 0;
  int bpi = 0;                // residual workgroups per instance
  int tmL = 32, tnL = 32;     // y-product tile (forward)
  int tmR = 32, tnR = 32;     // x-product tile (forward)
  // folded transforms: tiles of the x forward, y forward (+ divide), y
  // inverse and x inverse (+ update) launches
  FoldTile fR{32, 32, 0}, fL{32, 32, 0}, fLi{32, 32, 0}, fRi{32, 32, 0};
  FoldAxis ax{};
  double ih2 = 0.0;           // 1 / h^2 of both axes
  double lam_min = 0.0;       // smallest eigenvalue of the solve operator without the shift
  hipStream_t s = nullptr;    // per-class stream (default priority)
  hipEvent_t ev = nullptr;
  std::vector<double> hS, hlam;
};

}  // namespace

struct qnb_ctx_s {
  int count = 0, prec = 0, beta_mode = 0;
  bool fold = true;  // reflection-folded transforms (FP64/FP32); dense for split-bf16
  double beta = 0.0;
  int bc = QN_BC_DIRICHLET;
  double length = 1.0, lin = 0.0;
  int system = 0;                        // 2-component problem: 0 cubic system, 1 Gray-Scott
  double step = 1.0;                     // U -= step dU
  double gs[4] = {0.0, 0.0, 0.0, 0.0};  // Gray-Scott: D_A, D_S, rho, mu
  size_t off_cscale = 0;                 // device {D_A, D_S}
  size_t off_coef = 0;                   // device {scale, shift} of qnb_fdm_solve
  std::vector<int> n, ncomp, inst_cls, inst_pos;
  std::vector<Cls> cls;
  long long field_elems = 0;
  size_t need = 0;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  // parameters the captured graph was built with
  double* g_U = nullptr;
  const double* g_F = nullptr;
  double g_rtol = -1.0;
  int g_max = -1, g_iters = 0;
  hipStream_t g_stream = nullptr;
  int* h_done = nullptr;      // pinned host copies of every class's done flags
  BState* h_state = nullptr;  // and per-instance states (count entries each)
  hipError_t sticky = hipSuccess;
  size_t elem() const { return prec == QN_PREC_FP64 ? 8 : 4; }
};

namespace {

qn_status bad(qn_status s, const char* m) { return set_error(s, "%s", m); }
qn_status hip_bad(qnb_ctx c, hipError_t e, const char* what) {
  c->sticky = e;
  return set_error(QN_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

FoldOperands fops(qnb_ctx c, const Cls& k) {
  const size_t bb = (size_t)k.ax.bk * k.ax.bk * c->elem();
  char* base = c->ws + k.off_S;
  FoldOperands f{};
  f.FeT = base;
  f.FoT = base + bb;
  f.Fe = base + 2 * bb;
  f.Fo = base + 3 * bb;
  return f;
}

// bf16 parts of S for the dense split-bf16 transforms.
GemmOperands ops(qnb_ctx c, const Cls& k) {
  GemmOperands g{};
  g.Shi = c->ws + k.off_S;
  g.Slo = c->ws + k.off_Slo;
  return g;
}

EpiArgs epi_for(qnb_ctx c, const Cls& k, double* dense_base) {
  EpiArgs ep{};
  ep.lamM = (const double*)(c->ws + k.off_lam);
  ep.lamX = ep.lamM;
  ep.lamY = nullptr;
  BState* st = (BState*)(c->ws + k.off_state);
  ep.coef = &st[0].scale;
  ep.coef_stride = (int)(sizeof(BState) / sizeof(double));
  ep.dense = dense_base ? dense_base + k.off_field : nullptr;
  ep.px = ep.py = k.p;
  ep.pz = 1;
  ep.nx = ep.ny = k.n;
  ep.nz = 1;
  ep.skip = (const int*)(c->ws + k.off_done);
  ep.inst_mod = k.K;
  ep.step = c->step;
  if (c->system == 1 && k.ncomp == 2) {  // slab index = c * K + instance
    ep.cscale = (const double*)(c->ws + c->off_cscale);
    ep.comp_div = k.K;
  }
  return ep;
}

// Shift rule of the finalize kernel for a qn_beta_mode.
int batch_rule(int beta_mode) {
  switch (beta_mode) {
    case QN_BETA_MIDPOINT: return RULE_MIDPOINT;
    case QN_BETA_MAX: return RULE_MAX;
    case QN_BETA_SUM: return RULE_SUM;
    case QN_BETA_MIN: return RULE_MIN;
    default: return RULE_FIXED;
  }
}

// One quasi-Newton iteration of class k on stream s.
hipError_t class_iteration(qnb_ctx c, Cls& k, double* U, const double* F, double rtol, int max_iter,
                           hipStream_t s) {
  ResidualArgs a{};
  a.U = U + k.off_field;
  a.F = F + k.off_field;
  a.R = c->ws + k.off_W1;
  a.out_prec = transform_storage(c->prec);
  a.r_cstride = (long long)k.K * k.p * k.p;
  a.r_zstride = k.p * k.p;
  a.r_ystride = k.p;
  a.ox = a.oy = k.p;
  a.oz = k.K;
  a.nx = a.ny = k.n;
  a.nz = k.K;
  a.dim = 2;
  a.nl = k.ncomp == 2 ? (c->system == 1 ? NL_GS : NL_SYS2) : NL_CUBIC;
  a.gs_da = c->gs[0];
  a.gs_ds = c->gs[1];
  a.gs_rho = c->gs[2];
  a.gs_mu = c->gs[3];
  a.bc = c->bc;
  a.lin = c->lin;
  a.ihx2 = a.ihy2 = k.ih2;
  a.ihz2 = 0.0;
  a.partials = (double*)(c->ws + k.off_part);
  a.rz = RESIDUAL_PLANAR_ROWS;
  a.skip = (const int*)(c->ws + k.off_done);
  int nb = 0;
  hipError_t e = launch_residual(a, &nb, s);
  if (e != hipSuccess) return e;
  BState* st = (BState*)(c->ws + k.off_state);
  int* done = (int*)(c->ws + k.off_done);
  e = launch_bfinalize(a.partials, k.bpi, k.K, st, done, batch_rule(c->beta_mode), c->beta, rtol,
                       max_iter, k.lam_min, s);
  if (e != hipSuccess) return e;
  void* W1 = c->ws + k.off_W1;
  void* W2 = c->ws + k.off_W2;
  const GemmOperands S = ops(c, k);
  EpiArgs ep = epi_for(c, k, U);
  const int rows = k.ncomp * k.K * k.p;
  const int slabs = k.ncomp * k.K;
  const long long sl = (long long)k.p * k.p;
  if (c->fold) {
    const FoldOperands F = fops(c, k);
    e = launch_fold(FK_RFWD, c->prec, F, W1, W2, k.ax, 0, 0, 0, rows, EPI_STORE, ep, k.fR, s);
    if (e == hipSuccess)
      e = launch_fold(FK_LFWD, c->prec, F, W2, W1, k.ax, k.p, slabs, sl, rows, EPI_DIVIDE, ep, k.fL,
                      s);
    if (e == hipSuccess)
      e = launch_fold(FK_LINV, c->prec, F, W1, W2, k.ax, k.p, slabs, sl, rows, EPI_STORE, ep, k.fLi,
                      s);
    if (e == hipSuccess)
      e = launch_fold(FK_RINV, c->prec, F, W2, nullptr, k.ax, 0, 0, 0, rows, EPI_SUB_DENSE, ep,
                      k.fRi, s);
    return e;
  }
  e = launch_gemm_right(c->prec, S, W1, W2, rows, k.p, EPI_STORE, ep, k.tmR, k.tnR, s);
  if (e == hipSuccess)
    e = launch_gemm_left(c->prec, S, W2, W1, k.p, k.p, slabs, sl, EPI_DIVIDE, ep, k.tmL, k.tnL, s);
  if (e == hipSuccess)
    e = launch_gemm_left(c->prec, S, W1, W2, k.p, k.p, slabs, sl, EPI_STORE, ep, k.tmL, k.tnL, s);
  if (e == hipSuccess)
    e = launch_gemm_right(c->prec, S, W2, nullptr, rows, k.p, EPI_SUB_DENSE, ep, k.tmR, k.tnR, s);
  return e;
}

// Enqueue `iters` iterations of every class: fork onto the class streams,
// join back onto the context stream.
hipError_t enqueue(qnb_ctx c, double* U, const double* F, double rtol, int max_iter, int iters) {
  hipError_t e = hipEventRecord(c->fork, c->stream);
  for (auto& k : c->cls) {
    if (e == hipSuccess) e = hipStreamWaitEvent(k.s, c->fork, 0);
    for (int it = 0; it < iters && e == hipSuccess; ++it)
      e = class_iteration(c, k, U, F, rtol, max_iter, k.s);
    if (e == hipSuccess) e = hipEventRecord(k.ev, k.s);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, k.ev, 0);
  }
  return e;
}

void drop_graph(qnb_ctx c) {
  if (c->exec) hipGraphExecDestroy(c->exec);
  if (c->graph) hipGraphDestroy(c->graph);
  c->exec = nullptr;
  c->graph = nullptr;
}

}  // namespace

extern "C" {

qn_status qnb_setup(int32_t count, const int32_t* n, const int32_t* ncomp, int32_t precision,
                    int32_t beta_mode, double beta, qnb_ctx* out) {
  return qnb_setup_ex(count, n, ncomp, precision, beta_mode, beta, nullptr, out);
}

qn_status qnb_setup_ex(int32_t count, const int32_t* n, const int32_t* ncomp, int32_t precision,
                       int32_t beta_mode, double beta, const qnb_options* opt, qnb_ctx* out) {
  if (!out || !n || !ncomp) return bad(QN_ERR_INVALID, "null argument");
  if (count < 1 || count > 65536) return bad(QN_ERR_INVALID, "count must be in [1, 65536]");
  if (precision < 0 || precision > 2) return bad(QN_ERR_INVALID, "unknown precision");
  if (beta_mode < QN_BETA_FIXED || beta_mode > QN_BETA_MIN)
    return bad(QN_ERR_INVALID, "unknown beta_mode");
  if (!std::isfinite(beta)) return bad(QN_ERR_INVALID, "beta not finite");
  qnb_options o{};
  o.boundary = QN_BC_DIRICHLET;
  o.length = 1.0;
  if (opt) o = *opt;
  if (o.system != 0 && o.system != 1) return bad(QN_ERR_INVALID, "unknown system");
  const double step = o.step == 0.0 ? 1.0 : o.step;
  if (!(step > 0.0) || !std::isfinite(step))
    return bad(QN_ERR_INVALID, "step must be positive and finite");
  double gs[4] = {o.gs_da, o.gs_ds, o.gs_rho, o.gs_mu};
  if (o.system == 1) {
    const double paper[4] = {2.5e-4, 5e-4, 0.04, 0.065};  // Section 6.2
    for (int i = 0; i < 4; ++i) {
      if (gs[i] == 0.0) gs[i] = paper[i];
      if (!(gs[i] > 0.0) || !std::isfinite(gs[i]))
        return bad(QN_ERR_INVALID, "Gray-Scott parameters must be positive and finite");
    }
    if (o.boundary != QN_BC_NEUMANN)
      return bad(QN_ERR_UNSUPPORTED, "the Gray-Scott system is built with Neumann data");
    if (precision == QN_PREC_BF16X3)
      return bad(QN_ERR_UNSUPPORTED, "the Gray-Scott system needs FP64 or FP32 transforms");
    for (int i = 0; i < count; ++i)
      if (ncomp[i] != 2)
        return set_error(QN_ERR_UNSUPPORTED, "instance %d: the Gray-Scott batch is 2-component", i);
  } else if (gs[0] != 0.0 || gs[1] != 0.0 || gs[2] != 0.0 || gs[3] != 0.0) {
    return bad(QN_ERR_INVALID, "Gray-Scott parameters given for the cubic system");
  }
  if (o.boundary != QN_BC_DIRICHLET && o.boundary != QN_BC_NEUMANN)
    return bad(QN_ERR_INVALID, "unknown boundary");
  if (!std::isfinite(o.length) || o.length < 0.0)
    return bad(QN_ERR_INVALID, "length must be finite and >= 0 (0 means 1)");
  if (o.length == 0.0) o.length = 1.0;
  if (!std::isfinite(o.lin)) return bad(QN_ERR_INVALID, "lin not finite");
  const bool neu = o.boundary == QN_BC_NEUMANN;
  if (neu && precision == QN_PREC_BF16X3)
    return bad(QN_ERR_INVALID, "Neumann data needs FP64 or FP32 transforms");
  // The Neumann operator has the eigenvalue 0 (constant mode): the shift must
  // stay positive.  Every rule on the range of 3 u^2 + lin is at least lin.
  if (neu && beta_mode == QN_BETA_FIXED && !(beta > 0.0))
    return bad(QN_ERR_INVALID, "Neumann data needs a fixed beta > 0");
  if (neu && beta_mode != QN_BETA_FIXED && o.system == 0 && !(o.lin > 0.0))
    return bad(QN_ERR_INVALID, "Neumann data with a shift rule needs lin > 0");
  std::map<std::pair<int, int>, int> key;
  for (int i = 0; i < count; ++i) {
    if (ncomp[i] == 2 && o.system == 0 && (neu || o.lin != 0.0))
      return set_error(QN_ERR_INVALID, "instance %d: the 2-component system takes neither "
                                       "Neumann data nor lin", i);
    if (neu && n[i] < 2)
      return set_error(QN_ERR_INVALID, "instance %d: Neumann data needs n >= 2", i);
  }
  qnb_ctx c = new qnb_ctx_s();
  c->count = count;
  c->prec = precision;
  c->beta_mode = beta_mode;
  c->beta = beta;
  c->bc = o.boundary;
  c->length = o.length;
  c->lin = o.lin;
  c->system = o.system;
  c->step = step;
  for (int i = 0; i < 4; ++i) c->gs[i] = gs[i];
  c->n.assign(n, n + count);
  c->ncomp.assign(ncomp, ncomp + count);
  c->inst_cls.resize(count);
  c->inst_pos.resize(count);
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || n[i] > 4096 || (ncomp[i] != 1 && ncomp[i] != 2)) {
      delete c;
      return set_error(QN_ERR_INVALID, "instance %d: n = %d, ncomp = %d out of range", i, n[i], ncomp[i]);
    }
    auto kk = std::make_pair(n[i], ncomp[i]);
    auto it = key.find(kk);
    int ci;
    if (it == key.end()) {
      ci = (int)c->cls.size();
      key[kk] = ci;
      Cls k;
      k.n = n[i];
      k.ncomp = ncomp[i];
      if (precision != QN_PREC_BF16X3) {
        const int bk = fold_block(n[i]);
        k.ax = FoldAxis{n[i], n[i] / 2, n[i] & 1, bk};
        k.p = 2 * bk;
      } else {
        k.p = ((n[i] + 31) / 32) * 32;
      }
      c->cls.push_back(k);
    } else {
      ci = it->second;
    }
    c->inst_cls[i] = ci;
    c->inst_pos[i] = c->cls[ci].K++;
    c->cls[ci].members.push_back(i);
  }
  double lam_min = 1e300, lam_min1 = 1e300;  // all classes; scalar classes
  long long fe = 0;
  size_t off = 0;
  c->fold = precision != QN_PREC_BF16X3;
  for (auto& k : c->cls) {
    const double ih = (c->bc == QN_BC_NEUMANN ? k.n - 1 : k.n + 1) / c->length;
    k.ih2 = ih * ih;
    if (c->bc == QN_BC_NEUMANN) {
      fold_cosine(k.n, k.ih2, k.ax.bk, k.hS, k.hlam);
    } else {
      if (c->fold)
        fold_eigen(k.n, k.ax.bk, k.hS, k.hlam);
      else
        dense_eigen(k.n, k.p, k.hS, k.hlam);
      // the sine eigenvalues are for the unit interval
      if (c->length != 1.0)
        for (double& l : k.hlam) l /= c->length * c->length;
    }
    lam_min = std::min(lam_min, 2.0 * k.hlam[0]);
    if (k.ncomp == 1) lam_min1 = std::min(lam_min1, 2.0 * k.hlam[0]);
    // component c solves with D_c A_h for the Gray-Scott system
    k.lam_min = 2.0 * k.hlam[0] * (c->system == 1 ? std::min(c->gs[0], c->gs[1]) : 1.0);
    // The min rule on a 2-component system can give beta down to -1 (the
    // smallest eigenvalue of the 2x2 block at u = v = 0); every other rule
    // gives beta >= 0 on these problems.
    if (beta_mode == QN_BETA_MIN && k.ncomp == 2 && c->system == 0 && 2.0 * k.hlam[0] <= 1.0) {
      const int nn = k.n;
      delete c;
      return set_error(QN_ERR_INVALID, "n = %d: the min rule on a system can make the solve "
                                       "singular (lam_min(A_h) <= 1)", nn);
    }
    k.off_field = fe;
    fe += (long long)k.ncomp * k.K * k.n * k.n;
    const size_t pp = k.hS.size();
    const size_t eb = precision == QN_PREC_FP64 ? 8 : (precision == QN_PREC_FP32 ? 4 : 2);
    k.off_S = off;
    off += a256(pp * eb);
    if (precision == QN_PREC_BF16X3) {
      k.off_Slo = off;
      off += a256(pp * 2);
    }
    k.off_lam = off;
    off += a256((size_t)k.p * 8);
    const size_t te = (size_t)k.ncomp * k.K * pp * c->elem();
    k.off_W1 = off;
    off += a256(te);
    k.off_W2 = off;
    off += a256(te);
    k.bpi = residual_max_blocks(k.p, k.p, 1, RESIDUAL_PLANAR_ROWS, true);
    k.off_part = off;
    off += a256((size_t)k.bpi * k.K * 4 * sizeof(double));
    k.off_state = off;
    off += a256((size_t)k.K * sizeof(BState));
    k.off_done = off;
    off += a256((size_t)k.K * sizeof(int));
    // An x-product row tile must not straddle two instances (skip flags are
    // per tile), so its height divides P; folded tiles stay inside one half.
    if (c->fold) {
      // first listed tile that fits (x-product row tiles divide P)
      auto first = [&](int kind, FoldTile& t) {
        const FoldTile* list;
        const int nc = fold_tiles(kind, &list);
        for (int q = 0; q < nc; ++q)
          if (fold_tile_fits(kind, list[q], k.ax.bk, k.p, k.p)) {
            t = list[q];
            return;
          }
      };
      first(FK_RFWD, k.fR);
      first(FK_LFWD, k.fL);
      first(FK_LINV, k.fLi);
      first(FK_RINV, k.fRi);
    } else {
      k.tmL = largest_tile(k.p);
      k.tnL = largest_tile(k.p);
      k.tmR = largest_tile(k.p);
      k.tnR = largest_tile(k.p);
    }
  }
  if (beta_mode == QN_BETA_FIXED && lam_min + beta <= 0.0) {
    delete c;
    return bad(QN_ERR_INVALID, "fixed beta makes some instance's operator singular or indefinite");
  }
  // Scalar instances under a shift rule: 3 u^2 + lin >= lin, so beta >= lin
  // (>= 2 lin for min + max when lin < 0).
  const double beta_low = o.lin >= 0.0 ? o.lin : (beta_mode == QN_BETA_SUM ? 2.0 : 1.0) * o.lin;
  if (beta_mode != QN_BETA_FIXED && lam_min1 < 1e300 && lam_min1 + beta_low <= 0.0) {
    delete c;
    return bad(QN_ERR_INVALID, "lin makes the shift rule's solve singular or indefinite for some "
                               "instance (lin <= -lam_min(A_h))");
  }
  c->off_cscale = off;
  off += a256(2 * sizeof(double));
  c->off_coef = off;
  off += a256(2 * sizeof(double));
  c->field_elems = fe;
  c->need = off;
  *out = c;
  return QN_OK;
}

qn_status qnb_field_elems(qnb_ctx c, int64_t* elems) {
  if (!c || !elems) return bad(QN_ERR_INVALID, "null argument");
  *elems = c->field_elems;
  return QN_OK;
}

qn_status qnb_instance_layout(qnb_ctx c, int32_t i, int64_t* offset, int64_t* comp_stride) {
  if (!c || !offset || !comp_stride) return bad(QN_ERR_INVALID, "null argument");
  if (i < 0 || i >= c->count) return bad(QN_ERR_INVALID, "instance index out of range");
  const Cls& k = c->cls[c->inst_cls[i]];
  const long long nn = (long long)k.n * k.n;
  *offset = k.off_field + (long long)c->inst_pos[i] * nn;
  *comp_stride = (long long)k.K * nn;
  return QN_OK;
}

qn_status qnb_workspace_bytes(qnb_ctx c, size_t* bytes) {
  if (!c || !bytes) return bad(QN_ERR_INVALID, "null argument");
  *bytes = c->need;
  return QN_OK;
}

qn_status qnb_set_stream(qnb_ctx c, void* stream) {
  if (!c) return bad(QN_ERR_INVALID, "null context");
  c->stream = (hipStream_t)stream;
  return QN_OK;
}

qn_status qnb_bind_workspace(qnb_ctx c, void* d_ws, size_t bytes) {
  if (!c) return bad(QN_ERR_INVALID, "null context");
  if (c->sticky != hipSuccess) return set_error(QN_ERR_HIP, "sticky HIP error");
  if (!d_ws || ((uintptr_t)d_ws & 255u)) return bad(QN_ERR_WORKSPACE, "workspace null or misaligned");
  if (bytes < c->need) return set_error(QN_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", bytes, c->need);
  drop_graph(c);
  c->ws = (char*)d_ws;
  hipError_t e = hipSuccess;
  if (!c->fork) e = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
  for (auto& k : c->cls) {
    if (e == hipSuccess && !k.s) e = hipStreamCreateWithFlags(&k.s, hipStreamNonBlocking);
    if (e == hipSuccess && !k.ev) e = hipEventCreateWithFlags(&k.ev, hipEventDisableTiming);
  }
  if (e == hipSuccess) e = launch_zero(c->ws, c->need, c->stream);
  for (auto& k : c->cls) {
    const size_t pp = k.hS.size();
    if (e != hipSuccess) break;
    if (c->prec == QN_PREC_FP64) {
      e = hipMemcpyAsync(c->ws + k.off_S, k.hS.data(), pp * 8, hipMemcpyHostToDevice, c->stream);
    } else if (c->prec == QN_PREC_FP32) {
      std::vector<float> s32(pp);
      for (size_t i = 0; i < pp; ++i) s32[i] = (float)k.hS[i];
      e = hipMemcpyAsync(c->ws + k.off_S, s32.data(), pp * 4, hipMemcpyHostToDevice, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    } else {
      std::vector<uint16_t> hi(pp), lo(pp);
      for (size_t i = 0; i < pp; ++i) {
        hi[i] = bf16_rne((float)k.hS[i]);
        lo[i] = bf16_rne((float)(k.hS[i] - (double)bf16_value(hi[i])));
      }
      e = hipMemcpyAsync(c->ws + k.off_S, hi.data(), pp * 2, hipMemcpyHostToDevice, c->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(c->ws + k.off_Slo, lo.data(), pp * 2, hipMemcpyHostToDevice, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->ws + k.off_lam, k.hlam.data(), (size_t)k.p * 8, hipMemcpyHostToDevice,
                         c->stream);
  }
  if (e == hipSuccess && c->system == 1)
    e = hipMemcpyAsync(c->ws + c->off_cscale, c->gs, 2 * sizeof(double), hipMemcpyHostToDevice,
                       c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_bad(c, e, "bind workspace");
  return QN_OK;
}

qn_status qnb_autotune(qnb_ctx c) {
  if (!c || !c->ws) return bad(QN_ERR_WORKSPACE, "workspace not bound");
  if (c->sticky != hipSuccess) return set_error(QN_ERR_HIP, "sticky HIP error");
  drop_graph(c);
  hipEvent_t t0, t1;
  hipError_t e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  if (e != hipSuccess) return hip_bad(c, e, "autotune events");
  const int cand[3] = {32, 64, 128};
  for (auto& k : c->cls) {
    EpiArgs ep = epi_for(c, k, nullptr);
    ep.skip = nullptr;  // time every tile
    const GemmOperands S = ops(c, k);
    void* W1 = c->ws + k.off_W1;
    void* W2 = c->ws + k.off_W2;
    const int rows = k.ncomp * k.K * k.p, slabs = k.ncomp * k.K;
    const long long sl = (long long)k.p * k.p;
    const FoldOperands F = c->fold ? fops(c, k) : FoldOperands{};
    auto time_run = [&](auto run, float& ms) {
      hipError_t r = run();  // warm-up
      if (r == hipSuccess) r = hipEventRecord(t0, c->stream);
      for (int q = 0; q < 3 && r == hipSuccess; ++q) r = run();
      if (r == hipSuccess) r = hipEventRecord(t1, c->stream);
      if (r == hipSuccess) r = hipEventSynchronize(t1);
      if (r == hipSuccess) r = hipEventElapsedTime(&ms, t0, t1);
      return r;
    };
    if (c->fold) {
      const int kinds[4] = {FK_LFWD, FK_RFWD, FK_LINV, FK_RINV};
      FoldTile* dst[4] = {&k.fL, &k.fR, &k.fLi, &k.fRi};
      for (int fi = 0; fi < 4 && e == hipSuccess; ++fi) {
        const int kind = kinds[fi];
        const FoldTile* list;
        const int nc = fold_tiles(kind, &list);
        // x-product row tiles divide P, so they never straddle two instances
        float best = 1e30f;
        for (int q = 0; q < nc && e == hipSuccess; ++q) {
          const FoldTile t = list[q];
          if (!fold_tile_fits(kind, t, k.ax.bk, k.p, k.p)) continue;
          float ms = 0.f;
          e = time_run([&] {
            return launch_fold(kind, c->prec, F, W1, W2, k.ax, k.p, slabs, sl, rows, EPI_STORE, ep, t,
                               c->stream);
          }, ms);
          if (e == hipSuccess && ms < best) {
            best = ms;
            *dst[fi] = t;
          }
        }
      }
      continue;
    }
    for (int form = 0; form < 2 && e == hipSuccess; ++form) {
      float best = 1e30f;
      int bm = 32, bn = 32;
      for (int tm : cand)
        for (int tn : cand) {
          if (k.p % tm || k.p % tn) continue;  // tiles never straddle instances
          float ms = 0.f;
          e = time_run([&] {
            return form == 0 ? launch_gemm_left(c->prec, S, W1, W2, k.p, k.p, slabs, sl, EPI_STORE,
                                                ep, tm, tn, c->stream)
                             : launch_gemm_right(c->prec, S, W1, W2, rows, k.p, EPI_STORE, ep, tm,
                                                 tn, c->stream);
          }, ms);
          if (e != hipSuccess) break;
          if (ms < best) {
            best = ms;
            bm = tm;
            bn = tn;
          }
        }
      if (form == 0) {
        k.tmL = bm;
        k.tnL = bn;
      } else {
        k.tmR = bm;
        k.tnR = bn;
      }
    }
  }
  hipEventDestroy(t0);
  hipEventDestroy(t1);
  if (e != hipSuccess) return hip_bad(c, e, "autotune");
  return QN_OK;
}

qn_status qnb_class_count(qnb_ctx c, int32_t* classes) {
  if (!c || !classes) return bad(QN_ERR_INVALID, "null argument");
  *classes = (int32_t)c->cls.size();
  return QN_OK;
}

qn_status qnb_fdm_solve(qnb_ctx c, const double* d_R, double scale, double shift, double* d_X) {
  if (!c || !c->ws) return bad(QN_ERR_WORKSPACE, "workspace not bound");
  if (c->sticky != hipSuccess) return set_error(QN_ERR_HIP, "sticky HIP error");
  if (!d_R || !d_X || ((uintptr_t)d_R & 7u) || ((uintptr_t)d_X & 7u))
    return bad(QN_ERR_INVALID, "null or misaligned R or X");
  if (!(scale > 0.0) || !std::isfinite(scale) || !std::isfinite(shift))
    return bad(QN_ERR_INVALID, "scale must be positive and finite, shift finite");
  for (const auto& k : c->cls)
    if (!(scale * k.lam_min + shift > 0.0))
      return set_error(QN_ERR_INVALID, "n = %d: scale lam_min(A_h) + shift <= 0 (singular or "
                                       "indefinite)", k.n);
  double* coef = (double*)(c->ws + c->off_coef);
  hipError_t e = launch_set_coef(coef, scale, shift, c->stream);
  for (auto& k : c->cls) {
    if (e != hipSuccess) break;
    void* W1 = c->ws + k.off_W1;
    void* W2 = c->ws + k.off_W2;
    // the class block (ncomp, K, n, n) -> (ncomp, K, P, P), zero padding
    e = launch_pad_copy(d_R + k.off_field, W1, transform_storage(c->prec), k.ncomp, k.n, k.n,
                        k.K, k.p, k.p, k.K, c->stream);
    if (e != hipSuccess) break;
    EpiArgs ep = epi_for(c, k, d_X);
    ep.skip = nullptr;  // every instance
    ep.coef = coef;
    ep.coef_stride = 0;
    const int rows = k.ncomp * k.K * k.p;
    const int slabs = k.ncomp * k.K;
    const long long sl = (long long)k.p * k.p;
    if (c->fold) {
      const FoldOperands F = fops(c, k);
      e = launch_fold(FK_RFWD, c->prec, F, W1, W2, k.ax, 0, 0, 0, rows, EPI_STORE, ep, k.fR,
                      c->stream);
      if (e == hipSuccess)
        e = launch_fold(FK_LFWD, c->prec, F, W2, W1, k.ax, k.p, slabs, sl, rows, EPI_DIVIDE, ep,
                        k.fL, c->stream);
      if (e == hipSuccess)
        e = launch_fold(FK_LINV, c->prec, F, W1, W2, k.ax, k.p, slabs, sl, rows, EPI_STORE, ep,
                        k.fLi, c->stream);
      if (e == hipSuccess)
        e = launch_fold(FK_RINV, c->prec, F, W2, nullptr, k.ax, 0, 0, 0, rows, EPI_STORE_DENSE, ep,
                        k.fRi, c->stream);
    } else {
      const GemmOperands S = ops(c, k);
      e = launch_gemm_right(c->prec, S, W1, W2, rows, k.p, EPI_STORE, ep, k.tmR, k.tnR, c->stream);
      if (e == hipSuccess)
        e = launch_gemm_left(c->prec, S, W2, W1, k.p, k.p, slabs, sl, EPI_DIVIDE, ep, k.tmL, k.tnL,
                             c->stream);
      if (e == hipSuccess)
        e = launch_gemm_left(c->prec, S, W1, W2, k.p, k.p, slabs, sl, EPI_STORE, ep, k.tmL, k.tnL,
                             c->stream);
      if (e == hipSuccess)
        e = launch_gemm_right(c->prec, S, W2, nullptr, rows, k.p, EPI_STORE_DENSE, ep, k.tmR,
                              k.tnR, c->stream);
    }
  }
  if (e != hipSuccess) return hip_bad(c, e, "batched solve");
  return QN_OK;
}

qn_status qnb_class_info(qnb_ctx c, int32_t i, int32_t* info) {
  if (!c || !info) return bad(QN_ERR_INVALID, "null argument");
  if (i < 0 || i >= (int)c->cls.size()) return bad(QN_ERR_INVALID, "class index out of range");
  const Cls& k = c->cls[i];
  const int32_t v[8] = {k.n,
                        k.ncomp,
                        k.K,
                        c->fold ? k.fL.tm : k.tmL,
                        c->fold ? k.fL.tn : k.tnL,
                        c->fold ? k.fR.tm : k.tmR,
                        c->fold ? k.fR.tn : k.tnR,
                        k.p};
  std::memcpy(info, v, sizeof v);
  return QN_OK;
}

qn_status qnb_iterate(qnb_ctx c, double* d_U, const double* d_F, double rtol, int32_t max_iter,
                      int32_t graph_iters, qnb_result* results) {
  if (!c) return bad(QN_ERR_INVALID, "null context");
  if (c->sticky != hipSuccess) return set_error(QN_ERR_HIP, "sticky HIP error");
  if (!c->ws) return bad(QN_ERR_WORKSPACE, "workspace not bound");
  if (!d_U || !d_F || ((uintptr_t)d_U & 7u) || ((uintptr_t)d_F & 7u))
    return bad(QN_ERR_INVALID, "U and F must be non-null and 8-byte aligned");
  if (!(rtol >= 0.0) || max_iter < 0 || graph_iters < 1 || graph_iters > 64)
    return bad(QN_ERR_INVALID, "rtol >= 0, max_iter >= 0, 1 <= graph_iters <= 64 required");
  hipError_t e = hipSuccess;
  for (auto& k : c->cls) {
    if (e == hipSuccess)
      e = launch_breset((BState*)(c->ws + k.off_state), (int*)(c->ws + k.off_done), k.K, c->stream);
  }
  if (e != hipSuccess) return hip_bad(c, e, "reset");
  if (!c->exec || c->g_U != d_U || c->g_F != d_F || c->g_rtol != rtol || c->g_max != max_iter ||
      c->g_iters != graph_iters || c->g_stream != c->stream) {
    drop_graph(c);
    // Capture on a private stream so the caller's stream is never in capture mode.
    hipStream_t cap;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_bad(c, e, "capture stream");
    hipStream_t saved = c->stream;
    c->stream = cap;
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t e2 = enqueue(c, d_U, d_F, rtol, max_iter, graph_iters);
      e = hipStreamEndCapture(cap, &c->graph);
      if (e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0);
    c->stream = saved;
    hipStreamDestroy(cap);
    if (e != hipSuccess) {
      drop_graph(c);
      return hip_bad(c, e, "graph capture");
    }
    c->g_U = d_U;
    c->g_F = d_F;
    c->g_rtol = rtol;
    c->g_max = max_iter;
    c->g_iters = graph_iters;
    c->g_stream = c->stream;
  }
  // Replay until every instance is done (at most max_iter + 1 residual
  // evaluations each).  After each replay the done flags of all classes are
  // copied into one pinned host array and read after a single synchronisation.
  if (e == hipSuccess && !c->h_done) e = hipHostMalloc((void**)&c->h_done, c->count * sizeof(int));
  const int max_replays = (max_iter + 1 + graph_iters - 1) / graph_iters + 1;
  bool all_done = false;
  for (int r = 0; r < max_replays && !all_done && e == hipSuccess; ++r) {
    e = hipGraphLaunch(c->exec, c->stream);
    int pos = 0;
    for (auto& k : c->cls) {
      if (e == hipSuccess)
        e = hipMemcpyAsync(c->h_done + pos, c->ws + k.off_done, k.K * sizeof(int),
                           hipMemcpyDeviceToHost, c->stream);
      pos += k.K;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    all_done = e == hipSuccess;
    for (int j = 0; j < pos && all_done; ++j) all_done = c->h_done[j] != 0;
  }
  if (e != hipSuccess) return hip_bad(c, e, "graph replay");
  qn_status worst = QN_OK;
  if (!c->h_state) e = hipHostMalloc((void**)&c->h_state, c->count * sizeof(BState));
  int pos = 0;
  for (auto& k : c->cls) {
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->h_state + pos, c->ws + k.off_state, k.K * sizeof(BState),
                         hipMemcpyDeviceToHost, c->stream);
    pos += k.K;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_bad(c, e, "read results");
  pos = 0;
  for (auto& k : c->cls) {
    const BState* hs = c->h_state + pos;
    pos += k.K;
    for (int j = 0; j < k.K; ++j) {
      const BState& s = hs[j];
      const qn_status st = !s.done ? QN_ERR_NOT_CONVERGED : (qn_status)s.status;
      if (st == QN_ERR_DIVERGED) worst = QN_ERR_DIVERGED;
      else if (st != QN_OK && worst == QN_OK) worst = st;
      if (results) {
        qnb_result& o = results[k.members[j]];
        o.iters = s.iters;
        o.status = st;
        o.relres = s.relres;
        o.relres0 = s.relres0;
      }
    }
  }
  if (worst != QN_OK) set_error(worst, "some instances did not converge");
  return worst;
}

void qnb_destroy(qnb_ctx c) {
  if (!c) return;
  drop_graph(c);
  if (c->h_done) (void)hipHostFree(c->h_done);
  if (c->h_state) (void)hipHostFree(c->h_state);
  for (auto& k : c->cls) {
    if (k.s) hipStreamDestroy(k.s);
    if (k.ev) hipEventDestroy(k.ev);
  }
  if (c->fork) hipEventDestroy(c->fork);
  delete c;
}

}  // extern "C"
