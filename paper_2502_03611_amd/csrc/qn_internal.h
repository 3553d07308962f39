// Internal declarations shared by the HIP kernels and the host API of libqn.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstddef>
#include <cstdint>

#include "qn.h"

namespace qn {

// Device-resident scalars of one context.  The residual reduction writes the
// norms and extreme values; the shift rule writes scale/beta, which the
// spectral-divide epilogue reads, so no host round trip is needed between
// the residual and the solve.
struct DevScalars {
  double sumsqR;   // sum of squared residual entries
  double mumin;    // min of the Jacobian-diagonal quantity (see shift rule)
  double mumax;    // max of it
  double sumsqF;   // sum of squared source entries
  double relres;   // sqrt(sumsqR / sumsqF)
  double scale;    // c_k of the current solve
  double beta;     // beta_k of the current solve
  double flag;     // 1 if the solve operator is singular / indefinite
  int done;        // quasi-Newton loop: stop here (the next solve skips itself)
  int pad;
  // Eigenproblem: the Rayleigh quotient lam_n and the normalising factor
  // s_n = 1 / ||U~_n||_M of the stored iterate (adjacent: read as {lam, s}).
  double eig;
  double uscale;
};

// Shift rules executed on device after the residual reduction.
enum ShiftRule : int {
  RULE_FIXED = 0,      // c = 1, beta fixed
  RULE_MIDPOINT = 1,   // c = 1, beta = (mumin + mumax)/2
  RULE_COEFF_MID = 2,  // c = (mumin + mumax)/2, beta fixed (quasi-linear)
  RULE_MAX = 3,        // c = 1, beta = mumax
  RULE_SUM = 4,        // c = 1, beta = mumin + mumax
  RULE_MIN = 5,        // c = 1, beta = mumin
};

// NL_GS: the steady Gray-Scott system (2D), R = (D_A A A - S A^2 + (mu + rho) A - F_A,
// D_S A S + S A^2 + rho S - F_S) with A the discrete -Lap; its shift rule uses the
// real parts of the 2 x 2 reaction-block eigenvalues.
enum Nonlin : int { NL_CUBIC = 0, NL_QUASILIN = 1, NL_SYS2 = 2, NL_GS = 3 };

// Threads per workgroup of the 3D residual: 1024 (two workgroups per CU) for
// the variants that fit in 64 VGPRs, 512 where the kernel needs more registers
// (two components, or Neumann data), which would otherwise leave a single
// 1024-thread workgroup per CU.  bc: 0 Dirichlet, 1 Neumann.
constexpr int residual_threads(int nl, int bc) {
  return (nl == NL_QUASILIN || (nl == NL_CUBIC && bc == 0)) ? 1024 : 512;
}

// Epilogues of the mode-product GEMMs.
enum Epi : int {
  EPI_STORE = 0,        // padded store
  EPI_DIVIDE = 1,       // padded store of acc / (scale * (lamM + lamX + lamY) + beta)
  EPI_SUB_DENSE = 2,    // dense[..] -= acc (interior only)
  EPI_STORE_DENSE = 3,  // dense[..] = acc (interior only)
};

struct EpiArgs {
  const double* lamM;   // eigenvalues along the product's own axis (row index m)
  const double* lamX;   // eigenvalues along x (column index n % px)
  const double* lamY;   // eigenvalues along y (column index n / px), NULL in 2D
  const double* coef;   // device {scale, beta} (points into DevScalars or solve slot)
  double* dense;        // caller array (ncomp, nz, ny, nx) for the dense epilogues
  int px, py, pz;       // padded extents
  int nx, ny, nz;       // interior extents
  // Batched solver: slabs / row blocks belong to instance (index % inst_mod);
  // an instance whose skip flag is set is left untouched, and its {scale, beta}
  // sit at coef + instance * coef_stride.  A single problem uses skip = NULL,
  // inst_mod = 1, coef_stride = 0.
  const int* skip;
  int inst_mod;
  int coef_stride;
  // EPI_SUB_DENSE of the folded kernels: the old values are multiplied by
  // *uscale before the subtraction (the eigenproblem's normalisation), NULL: 1.
  const double* uscale;
  // Per-component multiplier of the eigenvalue sum in EPI_DIVIDE (component
  // = slab index / comp_div), NULL: 1 (the Gray-Scott system's diffusion
  // coefficients: (D_c A + beta I)^-1 per component).
  const double* cscale;
  int comp_div;
  // EPI_SUB_DENSE of the folded kernels: dense = old - step * acc (the damped
  // step of the Gray-Scott system; 1 otherwise).
  double step;
  // EPI_DIVIDE of the split-bf16 form L: eigenvalue added per slab (index
  // b % pz: the z mode of a y product batched over z), NULL: none.
  const double* lamB;
};

// Dense split-bf16 mode products (qn_gemm_bf16.hip), FP32 tensors.  All
// launchers take an explicit stream and return the launch status.
// Form L: C[b][m][n] = sum_k S[m][k] B[b][k][n]  (S symmetric, P x P, ld = P)
// Form R: C[r][n]    = sum_k A[r][k] S[k][n]     (A rows of length K = P)
// prec: QN_PREC_BF16X3 (S as bf16 parts Shi, Slo) or QN_PREC_BF16X6 (Shi,
// Slo, Slo2).
struct GemmOperands {
  const void* Shi;
  const void* Slo;
  const void* Slo2;  // bf16x6 only
};
// Largest tile side instantiated for the precision.
int gemm_bf_max_tile(int prec);

// fold > 0 (bf16x3 inverse products only): the reflection-folded form, which
// computes output rows (form L) or columns (form R) m < fold and their mirrors
// nmir - 1 - m from the even- and odd-mode sums (the eigenvectors are
// symmetric or antisymmetric about the centre by mode parity); fold is
// ceil(nmir / 2) rounded up to the tile side.  The rows or columns from
// nmir up to the padded extent are left unwritten.
//
// sp (bf16x3, 3D): the folded forward products, which pass tensors folded
// along an axis (rows [0, hp) of the axis the mirror sums, [hp, 2 hp) the
// differences, 2 hp = P):
//   form L, mode 1: forward from a folded input, K = hp, M = 2 hp, S the
//                   even modes' rows of S then the odd modes', hp columns;
//                   output rows in mode order
//   form L, mode 2: the same with the output folded along y (the z product;
//                   hpo: half extent of the folded y layout)
//   form R, mode 3: dense x product, output folded along z (hpo: half extent
//                   of the folded z layout)
struct BfSplit {
  int mode;
  int K;    // form L: contraction length, the leading dimension of S
  int hpo;  // modes 2 and 3
};
hipError_t launch_gemm_left(int prec, const GemmOperands& s, const void* B, void* C, int M,
                            int ncols, int batch, long long bstride, int epi, const EpiArgs& ep,
                            int tm, int tn, hipStream_t st, int fold = 0, int nmir = 0,
                            const BfSplit* sp = nullptr);
hipError_t launch_gemm_right(int prec, const GemmOperands& s, const void* A, void* C, int rows,
                             int K, int epi, const EpiArgs& ep, int tm, int tn, hipStream_t st,
                             int fold = 0, int nmir = 0, const BfSplit* sp = nullptr);

// Reflection-folded mode products (qn_gemm_fold.hip).  Along a folded axis of
// n interior points, h = n / 2, odd = n % 2, and the spectral index is stored
// split: even modes in [0, bk), odd modes in [bk, 2 bk); the padded extent is
// 2 bk.
struct FoldAxis {
  int n, h, odd, bk;
};
struct FoldOperands {
  const void* FeT;  // [k][i] = S[k][2i]    (bk x bk, forward)
  const void* FoT;  // [k][i] = S[k][2i+1]
  const void* Fe;   // [i][k] = S[k][2i]    (inverse)
  const void* Fo;   // [i][k] = S[k][2i+1]
};
// Folded mode-product kinds and their instantiated tile shapes, in order of
// preference.  FK_LFWD tiles with paired = 1 compute the even and odd
// spectral rows of a tile together (tm = fold rows per tile).  tk: rows of
// the contraction per LDS stage, 0 for the kernel's own depth, else a deep
// stage for short contractions (valid when it divides bk).  The stage depth
// changes neither the order nor the grouping of the accumulation.
enum FoldKind : int { FK_RFWD = 0, FK_LFWD = 1, FK_LINV = 2, FK_RINV = 3 };
struct FoldTile {
  int tm, tn, paired, tk;
};
int fold_tiles(int kind, const FoldTile** list);
// Extents a tile must divide: (mext, next) = (rows, bk) for the x products,
// (bk, ncols) for the y/z products; workgroups of one launch with tile t.
void fold_extents(int kind, int bk, int ncols, int rows, long long* mext, long long* next);
bool fold_tile_fits(int kind, const FoldTile& t, int bk, int ncols, int rows);
long long fold_blocks(int kind, const FoldTile& t, int bk, int ncols, int batch, int rows);
// One folded mode product: form L (y/z) uses ncols, batch, bstride; form R
// (x) uses rows; epi applies to FK_LFWD (STORE / DIVIDE) and FK_RINV (STORE /
// SUB_DENSE / STORE_DENSE).
hipError_t launch_fold(int kind, int prec, const FoldOperands& f, const void* in, void* out,
                       const FoldAxis& ax, int ncols, int batch, long long bstride, int rows,
                       int epi, const EpiArgs& ep, const FoldTile& t, hipStream_t st);

// Residual of the nonlinear problem, written (with zero padding) into the
// transform workspace or into a dense caller array.  out_prec: 0 fp64, 1 fp32.
struct ResidualArgs {
  const double* U;
  const double* F;
  void* R;                 // output base
  int out_prec;            // 0: double, 1: float, 2: bf16 part pair (hi plane at R, lo plane
                           //    r_plane elements further; the split-bf16 transforms' storage)
  long long r_plane = 0;   // out_prec 2: elements of one plane
  long long r_cstride;     // output stride between components
  int r_zstride, r_ystride;// output strides of z and y (x stride 1)
  int ox, oy, oz;          // output extents to cover (padded or interior)
  int nx, ny, nz;          // interior extents (nz = 1 in 2D)
  int dim, nl;
  double ihx2, ihy2, ihz2; // 1/h^2 per axis
  double* partials;        // per-block {sumR2, mumin, mumax, sumF2}
  int rz;                  // 3D: z-planes per workgroup; planar: y-rows per workgroup
  const int* skip;         // batched solver: per-z-plane (instance) skip flags, else NULL
  const int* stop;         // single problem: the whole launch returns when *stop != 0, or NULL
  // Cubic problem: F^h = A U + lin U + cub U^3 + V U - F, V = pot (one
  // component, interior layout of U) or 0 when pot is NULL.
  double lin;
  int bc;                  // 0 Dirichlet (zero outside), 1 Neumann (mirrored neighbours)
  double cub = 1.0;
  double quad = 0.0;  // cubic problem: coefficient of U^2
  const double* pot = nullptr;
  // Eigenproblem passes (cubic problem only; F is not read):
  // mode 1: no output; per-block sums {W (A U) U, W U^2, W U^4, W (lin + V) U^2}
  //   over the stored iterate U, W = trapezoid end weights for Neumann data
  //   (1 for Dirichlet);
  // mode 2: with {lam, s} = eig[0..1], R = A (sU) + cub (sU)^3 + (lin + V - lam) sU,
  //   partials {sum W R^2, min mu, max mu, 0}, mu = 3 cub (sU)^2 + lin + V - lam.
  int mode = 0;
  const double* eig = nullptr;
  // Spectral elements (sem_k > 0: element order): banded H = M^-1 S per axis,
  // hb[a][j * (2k + 1) + d + k] = H[j][j + d]; the cubic problem only.
  int sem_k = 0;
  const double* hb[3] = {nullptr, nullptr, nullptr};
  // Gray-Scott system (NL_GS): diffusion coefficients and reaction rates.
  double gs_da = 0.0, gs_ds = 0.0, gs_rho = 0.0, gs_mu = 0.0;
  // 3D, out_prec 2, whole-row tiles (tile width = ox = 2 xfold): the output
  // folded along x, position j < xfold of a row the mirror sum R[j] +
  // R[nx-1-j], position xfold + j the difference (the middle point of odd nx
  // once, its difference zero; positions from ceil(nx / 2) on zero); 0: plain.
  int xfold = 0;
};
hipError_t launch_residual(const ResidualArgs& a, int* nblocks_out, hipStream_t st);
// Spectral element residual (qn_sem.hip): same outputs and partials as
// launch_residual for the cubic problem; SEM_ROWS rows of 256 nodes per workgroup.
constexpr int SEM_ROWS = 8;
constexpr int SEM_RZ = 64;  // 3D: z-planes per workgroup
hipError_t launch_sem_residual(const ResidualArgs& a, int* nblocks_out, hipStream_t st);
int sem_residual_blocks(int dim, int ox, int oy, int oz);  // workgroups = partial slots
// Eigenproblem finalizes (one workgroup each; return at once when *stop != 0).
// Phase 1 reduces the mode-1 sums into sc->eig = lam and sc->uscale = s
// (hvol = h^d, the mass of one interior node).  Phase 2 reduces the mode-2
// partials: relres = sqrt(hvol sum W R^2) / |lam|, the shift rule (the midpoint
// of mu, or beta_fixed), the singularity flag and the stop decision, written
// to *sc and *mirror; red_out (may be NULL) receives
// {lam, s, hvol sum W R^2, min mu, max mu, relres}.
hipError_t launch_eig_finalize1(const double* partials, int nblocks, DevScalars* sc, double cub,
                                double hvol, const int* stop, hipStream_t st);
hipError_t launch_eig_finalize2(const double* partials, int nblocks, DevScalars* sc, int rule,
                                double beta_fixed, double lam_min_sum, double hvol,
                                double* red_out, double rtol, int iter, int max_iter,
                                const int* stop, hipStream_t st, DevScalars* mirror = nullptr);
// u[i] *= *s for i < n.
hipError_t launch_scale(double* u, long long n, const double* s, hipStream_t st);
// Workgroups (= partial slots) of a residual launch; planar: no z coupling
// (1/h_z^2 = 0: 2D problems and the batched solver), which uses the planar
// kernel with oz planes.
int residual_max_blocks(int ox, int oy, int oz, int rz, bool planar, int threads = 1024);
// 3D residual geometry (launch and partial-slot sizing use the same rule):
// tile width in x of the workgroups and z-slab depth for an ox x oy x oz grid
// and `threads` (residual_threads) per workgroup.
int residual_tile_x(int ox, int threads);
int residual_slab_depth(int ox, int oy, int oz, int threads);
constexpr int RESIDUAL_PLANAR_ROWS = 16;  // rows per workgroup, many planes per launch
// Rows per workgroup of the planar residual over one ox x oy plane: 16,
// halved until the plane gives at least 1024 workgroups (or 1 row).
int residual_planar_rows(int ox, int oy);

// Per-instance state of the batched solver.  scale and beta are adjacent so
// the divide epilogue can read them as {scale, beta}.
struct BState {
  double relres, relres0, sumsqF, scale, beta;
  int iters, done, status, pad;
};
static_assert(sizeof(BState) % sizeof(double) == 0, "BState must be a whole number of doubles");
// Batched finalize: workgroup k reduces partials [k*bpi, (k+1)*bpi) of one
// class and updates st[k] (stopping rule, shift rule `rule` of ShiftRule
// other than RULE_COEFF_MID, iteration count).  done[k] mirrors st[k].done as
// a plain int array (the GEMM/residual skip flags).  An instance whose shift
// leaves lam_min + beta <= 0 (lam_min: the smallest eigenvalue of the class's
// solve operator without the shift) stops as diverged instead of solving.
hipError_t launch_bfinalize(const double* partials, int bpi, int K, BState* st, int* done,
                            int rule, double beta_fixed, double rtol, int max_iter,
                            double lam_min, hipStream_t s);
hipError_t launch_breset(BState* st, int* done, int K, hipStream_t s);

// Fixed-order reduction of the residual partials + shift rule.
// Final fixed-order reduction of the residual partials, the shift rule and,
// for iter >= 0, the loop decision: done = the relative residual is <= rtol,
// non-finite or above 1e30, iter >= max_iter, or the shift rule gives a
// singular operator.
// mirror (nullable): a second copy of the scalars, e.g. the device address of
// a pinned host slot that the host reads after an event.
hipError_t launch_finalize(const double* partials, int nblocks, DevScalars* sc, int rule,
                           double beta_fixed, double lam_min_sum, double* red_out, double rtol,
                           int iter, int max_iter, hipStream_t st, DevScalars* mirror = nullptr);

// Dense (ncomp, nz, ny, nx) fp64 -> padded (ncomp, pz, py, px) fp64/fp32, zero pads.
// Element storage of the transform workspace tensors for a qn_precision:
// 0 FP64, 1 FP32, 2 bf16 part planes (bf16x3; out_prec of ResidualArgs).
inline int transform_storage(int prec) {
  return prec == QN_PREC_FP64 ? 0 : prec == QN_PREC_BF16X3 ? 2 : 1;
}
// xfold > 0 (out_prec 2, px = 2 xfold): the copy folded along x as the
// residual's xfold output.
hipError_t launch_pad_copy(const double* src, void* dst, int out_prec, int ncomp, int nx, int ny,
                           int nz, int px, int py, int pz, hipStream_t st, int xfold = 0);
// Write {scale, beta} into a device slot.
hipError_t launch_set_coef(double* slot, double scale, double beta, hipStream_t st);
// Fill n bytes with zero (a kernel, not a memset node).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);

}  // namespace qn
