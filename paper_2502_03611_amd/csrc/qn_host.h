// Host-side eigen-data shared by the single-problem and batched contexts.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace qn {

// Closed-form eigenpairs of h^-2 tridiag(-1, 2, -1) of order n (Section 3.2
// eq. Sy; Section 4.2 with M = I): S[j][k] = sqrt(2/(n+1)) sin((j+1)(k+1) pi/(n+1)),
// lam_k = 4 (n+1)^2 sin^2((k+1) pi / (2(n+1))) (0-based).  The sine argument
// is reduced as an integer first, so S is exactly symmetric.
inline void sine_eigen(int n, std::vector<double>& S, std::vector<double>& lam) {
  const long long m = n + 1;
  const double pi = 3.14159265358979323846;
  S.assign((size_t)n * n, 0.0);
  lam.assign((size_t)n, 0.0);
  const double nrm = std::sqrt(2.0 / (double)m);
  for (int j = 1; j <= n; ++j)
    for (int k = 1; k <= n; ++k) {
      const long long red = ((long long)j * k) % (2 * m);
      S[(size_t)(j - 1) * n + (k - 1)] = nrm * std::sin(pi * (double)red / (double)m);
    }
  for (int k = 1; k <= n; ++k) {
    const double s = std::sin(pi * k / (2.0 * m));
    lam[k - 1] = 4.0 * (double)(m * m) * s * s;
  }
}

inline int fold_block(int n) { return (((n + 1) / 2 + 31) / 32) * 32; }

// Dense padded form: S (p x p, zero outside n x n) and lam (p, padded with lam_max).
inline void dense_eigen(int n, int p, std::vector<double>& Sp, std::vector<double>& lp) {
  std::vector<double> S, lam;
  sine_eigen(n, S, lam);
  Sp.assign((size_t)p * p, 0.0);
  lp.assign((size_t)p, lam[n - 1]);
  for (int j = 0; j < n; ++j) {
    for (int k = 0; k < n; ++k) Sp[(size_t)j * p + k] = S[(size_t)j * n + k];
    lp[j] = lam[j];
  }
}

// Folded forward products of the 3D split-bf16 path: along an axis of n
// points the input is folded about the centre (rows j < hp the mirror sums
// U[j] + U[n-1-j], rows hp + j the differences; the middle row of odd n once),
// hp = ceil(n / 2) rounded up to 32; usable when 2 hp equals the padded
// extent.  Forward operand Sf (2 hp x hp): row t < hp holds even mode 2 t,
// row hp + t odd mode 2 t + 1, each at j < ceil(n / 2) (zero rows for modes
// from n on), from the dense padded S (p x p, S[j][k] = entry j of mode k).
inline int fold_half(int n) { return (((n + 1) / 2 + 31) / 32) * 32; }
inline void fold_forward(int n, int p, const std::vector<double>& Sp, std::vector<double>& Sf) {
  const int hp = fold_half(n), h = (n + 1) / 2;
  Sf.assign((size_t)2 * hp * hp, 0.0);
  for (int pos = 0; pos < 2 * hp; ++pos) {
    const int m = pos < hp ? 2 * pos : 2 * (pos - hp) + 1;
    if (m >= n) continue;
    for (int j = 0; j < h; ++j) Sf[(size_t)pos * hp + j] = Sp[(size_t)j * p + m];
  }
}

// Folded form (block bk): FeT, FoT, Fe, Fo (bk x bk each, concatenated in that
// order) and lam in split order (2 bk, padded with lam_max).
inline void fold_eigen(int n, int bk, std::vector<double>& F4, std::vector<double>& ls) {
  std::vector<double> S, lam;
  sine_eigen(n, S, lam);
  const int h = n / 2, ne = h + (n & 1), no = h;
  const size_t bb = (size_t)bk * bk;
  F4.assign(4 * bb, 0.0);
  double* FeT = F4.data();
  double* FoT = FeT + bb;
  double* Fe = FoT + bb;
  double* Fo = Fe + bb;
  for (int k = 0; k < ne; ++k)
    for (int i = 0; i < ne; ++i) {
      const double v = S[(size_t)k * n + 2 * i];
      FeT[(size_t)k * bk + i] = v;
      Fe[(size_t)i * bk + k] = v;
    }
  for (int k = 0; k < h; ++k)
    for (int i = 0; i < no; ++i) {
      const double v = S[(size_t)k * n + 2 * i + 1];
      FoT[(size_t)k * bk + i] = v;
      Fo[(size_t)i * bk + k] = v;
    }
  ls.assign((size_t)2 * bk, lam[n - 1]);
  for (int i = 0; i < ne; ++i) ls[i] = lam[2 * i];
  for (int i = 0; i < no; ++i) ls[bk + i] = lam[2 * i + 1];
}

// Homogeneous Neumann data (ghost nodes, Section 3.2): the 1D stiffness
// matrix S = h^-2 [2 -2; -1 2 -1; ...; -2 2] of order n is W^-1 K with K
// symmetric and W = diag(1/2, 1, .., 1, 1/2) (Section 4.2 with a diagonal
// mass); its eigenvectors T[j][k] = cos(j k pi / (n - 1)) (integer-reduced
// argument), eigenvalues lam_k = 4 h^-2 sin^2(k pi / (2 (n - 1))) (ih2 = h^-2), and
// T^-1 = diag(1 / c_k) T^T W with c_k = (n - 1) / 2, or n - 1 for k = 0 and
// k = n - 1.  Folded like fold_eigen, with the forward blocks taken from T^-1
// (FeT[j][i] = T^-1[2i][j]) and the inverse blocks from T (Fe[i][j] =
// T[j][2i]): both have the reflection parity of the sine case, because W is
// symmetric about the centre.
inline void fold_cosine(int n, double ih2, int bk, std::vector<double>& F4,
                        std::vector<double>& ls) {
  const long long m = n - 1;
  const double pi = 3.14159265358979323846;
  auto T = [&](int j, int k) {
    const long long red = ((long long)j * k) % (2 * m);
    return std::cos(pi * (double)red / (double)m);
  };
  auto w = [&](int j) { return (j == 0 || j == n - 1) ? 0.5 : 1.0; };
  auto c = [&](int k) { return (k == 0 || k == n - 1) ? (double)m : 0.5 * (double)m; };
  auto Tinv = [&](int k, int j) { return T(j, k) * w(j) / c(k); };
  const int h = n / 2, ne = h + (n & 1), no = h;
  const size_t bb = (size_t)bk * bk;
  F4.assign(4 * bb, 0.0);
  double* FeT = F4.data();
  double* FoT = FeT + bb;
  double* Fe = FoT + bb;
  double* Fo = Fe + bb;
  for (int j = 0; j < ne; ++j)
    for (int i = 0; i < ne; ++i) {
      FeT[(size_t)j * bk + i] = Tinv(2 * i, j);
      Fe[(size_t)i * bk + j] = T(j, 2 * i);
    }
  for (int j = 0; j < h; ++j)
    for (int i = 0; i < no; ++i) {
      FoT[(size_t)j * bk + i] = Tinv(2 * i + 1, j);
      Fo[(size_t)i * bk + j] = T(j, 2 * i + 1);
    }
  std::vector<double> lam((size_t)n);
  for (int k = 0; k < n; ++k) {
    const double s = std::sin(pi * (double)k / (2.0 * (double)m));
    lam[k] = 4.0 * ih2 * s * s;
  }
  ls.assign((size_t)2 * bk, lam[n - 1]);
  for (int i = 0; i < ne; ++i) ls[i] = lam[2 * i];
  for (int i = 0; i < no; ++i) ls[bk + i] = lam[2 * i + 1];
}

// ---------------------------------------------------------------- spectral elements
// Q^k spectral elements with Gauss-Lobatto nodes (Section 3.1 and the remark on
// Gauss-Lobatto integration; Section 4.2 for the diagonalisation).

// Gauss-Lobatto nodes (ascending) and weights of order k >= 1 on [-1, 1]: the
// two ends and the k - 1 roots of P_k', found by Newton's method on P_k' (P_k''
// from Legendre's equation) from the Chebyshev-Lobatto points; weights
// 2 / (k (k + 1) P_k(x)^2).
inline void gl_nodes(int k, std::vector<double>& x, std::vector<double>& w) {
  const double pi = 3.14159265358979323846;
  auto legendre = [k](double t, double& pk, double& dpk) {
    double p0 = 1.0, p1 = t;
    if (k == 0) { pk = 1.0; dpk = 0.0; return; }
    for (int j = 1; j < k; ++j) {
      const double p2 = ((2.0 * j + 1.0) * t * p1 - j * p0) / (j + 1.0);
      p0 = p1;
      p1 = p2;
    }
    pk = p1;
    dpk = k * (t * p1 - p0) / (t * t - 1.0);  // interior points only
  };
  x.assign((size_t)k + 1, 0.0);
  w.assign((size_t)k + 1, 0.0);
  x[0] = -1.0;
  x[k] = 1.0;
  for (int j = 1; j < k; ++j) {
    double t = -std::cos(pi * j / k);
    for (int it = 0; it < 100; ++it) {
      double pk, dpk;
      legendre(t, pk, dpk);
      const double d2 = (2.0 * t * dpk - k * (k + 1.0) * pk) / (1.0 - t * t);
      const double step = dpk / d2;
      t -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    x[j] = t;
  }
  for (int j = 0; j <= k; ++j) {
    double p0 = 1.0, p1 = x[j];
    for (int i = 1; i < k; ++i) {
      const double p2 = ((2.0 * i + 1.0) * x[j] * p1 - i * p0) / (i + 1.0);
      p0 = p1;
      p1 = p2;
    }
    const double pk = k == 0 ? 1.0 : p1;
    w[j] = 2.0 / (k * (k + 1.0) * pk * pk);
  }
}

// One axis: E elements of order k on [0, L]; lumped mass m and dense
// stiffness S of the unknown nodes (Dirichlet: the E k - 1 interior nodes;
// Neumann: all E k + 1).
inline void sem_axis(int elements, int k, double length, bool neumann, std::vector<double>& m,
                     std::vector<double>& S, std::vector<double>* nodes = nullptr) {
  std::vector<double> xi, w;
  gl_nodes(k, xi, w);
  const int nq = k + 1;
  std::vector<double> D((size_t)nq * nq);  // D[q][p] = psi_p'(xi_q)
  for (int q = 0; q < nq; ++q)
    for (int p = 0; p < nq; ++p) {
      if (p == q) {
        double v = 0.0;
        for (int r = 0; r < nq; ++r)
          if (r != p) v += 1.0 / (xi[p] - xi[r]);
        D[(size_t)q * nq + p] = v;
      } else {
        double num = 1.0, den = 1.0;
        for (int r = 0; r < nq; ++r) {
          if (r != p && r != q) num *= xi[q] - xi[r];
          if (r != p) den *= xi[p] - xi[r];
        }
        D[(size_t)q * nq + p] = num / den;
      }
    }
  const double jac = 0.5 * length / elements;
  const int ntot = elements * k + 1;
  std::vector<double> mt((size_t)ntot, 0.0), st((size_t)ntot * ntot, 0.0);
  for (int e = 0; e < elements; ++e)
    for (int p = 0; p < nq; ++p) {
      const int gp = e * k + p;
      mt[gp] += w[p] * jac;
      for (int r = 0; r < nq; ++r) {
        double v = 0.0;
        for (int q = 0; q < nq; ++q) v += w[q] * D[(size_t)q * nq + p] * D[(size_t)q * nq + r];
        st[(size_t)gp * ntot + e * k + r] += v / jac;
      }
    }
  const int lo = neumann ? 0 : 1, n = neumann ? ntot : ntot - 2;
  if (nodes) {
    nodes->assign((size_t)n, 0.0);
    for (int i = 0; i < n; ++i) {
      const int g = lo + i, e = std::min(g / k, elements - 1), q = g - e * k;
      (*nodes)[i] = (2.0 * e + 1.0 + xi[q]) * jac;
    }
  }
  m.assign((size_t)n, 0.0);
  S.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    m[i] = mt[lo + i];
    for (int j = 0; j < n; ++j) S[(size_t)i * n + j] = st[(size_t)(lo + i) * ntot + lo + j];
  }
}

// Symmetric eigen-decomposition A = Q diag(d) Q^T by cyclic Jacobi rotations
// (A: n x n row-major, destroyed); columns of Q are the eigenvectors, sorted
// by ascending eigenvalue.
inline void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& Q,
                         std::vector<double>& d) {
  Q.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  double scale = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) scale += a(i, j) * a(i, j);
  scale = std::sqrt(scale);
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += a(i, j) * a(i, j);
    if (std::sqrt(off) <= 1e-17 * scale) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        if (std::fabs(apq) <= 1e-300 * scale) continue;
        // rotation angle that zeroes a(p, q): tan from the smaller root
        const double theta = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int r = 0; r < n; ++r) {  // columns p, q
          const double arp = a(r, p), arq = a(r, q);
          a(r, p) = c * arp - sn * arq;
          a(r, q) = sn * arp + c * arq;
        }
        for (int r = 0; r < n; ++r) {  // rows p, q
          const double apr = a(p, r), aqr = a(q, r);
          a(p, r) = c * apr - sn * aqr;
          a(q, r) = sn * apr + c * aqr;
        }
        a(p, q) = a(q, p) = 0.0;
        for (int r = 0; r < n; ++r) {
          const double vp = Q[(size_t)r * n + p], vq = Q[(size_t)r * n + q];
          Q[(size_t)r * n + p] = c * vp - sn * vq;
          Q[(size_t)r * n + q] = sn * vp + c * vq;
        }
      }
  }
  std::vector<int> order((size_t)n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int x, int y) { return a(x, x) < a(y, y); });
  std::vector<double> Qs((size_t)n * n);
  d.assign((size_t)n, 0.0);
  for (int c = 0; c < n; ++c) {
    d[c] = a(order[c], order[c]);
    for (int r = 0; r < n; ++r) Qs[(size_t)r * n + c] = Q[(size_t)r * n + order[c]];
  }
  Q.swap(Qs);
}

// Folded eigen-data of H = M^-1 S for a reflection-symmetric axis (uniform
// elements): B = M^-1/2 S M^-1/2 is split into its even block (basis
// (e_j + e_{n-1-j}) / sqrt 2, j < n/2, and the centre e_{n/2} for odd n) and its
// odd block ((e_j - e_{n-1-j}) / sqrt 2), each diagonalised by Jacobi; with
// T = M^-1/2 T~ and T^-1 = T~^T M^1/2 (Section 4.2) the blocks are laid out as
// the folded kernels read them: FeT[j][i] = T^-1[i][j], Fe[i][j] = T[j][i] for
// even modes i and folded nodes j (FoT, Fo likewise for odd modes); lam in
// split spectral order, padded with lam_max.  Returns lam_min.
inline double fold_sem(int n, const std::vector<double>& m, const std::vector<double>& S, int bk,
                       std::vector<double>& F4, std::vector<double>& ls) {
  const int h = n / 2, ne = h + (n & 1), no = h;
  const double r2 = std::sqrt(0.5);
  auto B = [&](int i, int j) { return S[(size_t)i * n + j] / std::sqrt(m[i] * m[j]); };
  std::vector<double> Be((size_t)ne * ne), Bo((size_t)no * no);
  for (int a = 0; a < ne; ++a)
    for (int b = 0; b < ne; ++b) {
      double v;
      if (a < h && b < h)
        v = 0.5 * (B(a, b) + B(a, n - 1 - b) + B(n - 1 - a, b) + B(n - 1 - a, n - 1 - b));
      else if (a < h)  // b is the centre
        v = r2 * (B(a, b) + B(n - 1 - a, b));
      else if (b < h)
        v = r2 * (B(a, b) + B(a, n - 1 - b));
      else
        v = B(a, b);
      Be[(size_t)a * ne + b] = v;
    }
  for (int a = 0; a < no; ++a)
    for (int b = 0; b < no; ++b)
      Bo[(size_t)a * no + b] =
          0.5 * (B(a, b) - B(a, n - 1 - b) - B(n - 1 - a, b) + B(n - 1 - a, n - 1 - b));
  std::vector<double> Qe, de, Qo, dd;
  jacobi_eigen(ne, Be, Qe, de);
  jacobi_eigen(no, Bo, Qo, dd);
  const size_t bb = (size_t)bk * bk;
  F4.assign(4 * bb, 0.0);
  double* FeT = F4.data();
  double* FoT = FeT + bb;
  double* Fe = FoT + bb;
  double* Fo = Fe + bb;
  for (int i = 0; i < ne; ++i)
    for (int j = 0; j < ne; ++j) {
      const double t = (j < h ? r2 : 1.0) * Qe[(size_t)j * ne + i];  // T~ entry at node j
      FeT[(size_t)j * bk + i] = t * std::sqrt(m[j]);
      Fe[(size_t)i * bk + j] = t / std::sqrt(m[j]);
    }
  for (int i = 0; i < no; ++i)
    for (int j = 0; j < no; ++j) {
      const double t = r2 * Qo[(size_t)j * no + i];
      FoT[(size_t)j * bk + i] = t * std::sqrt(m[j]);
      Fo[(size_t)i * bk + j] = t / std::sqrt(m[j]);
    }
  double lmax = de.empty() ? 0.0 : de.back(), lmin = de.empty() ? 0.0 : de.front();
  if (!dd.empty()) {
    lmax = std::max(lmax, dd.back());
    lmin = std::min(lmin, dd.front());
  }
  ls.assign((size_t)2 * bk, lmax);
  for (int i = 0; i < ne; ++i) ls[i] = de[i];
  for (int i = 0; i < no; ++i) ls[bk + i] = dd[i];
  return lmin;
}

// Banded H = M^-1 S of one axis: Hb[j][d + k] = H[j][j + d], |d| <= k (0 off the grid).
inline void sem_band(int n, int k, const std::vector<double>& m, const std::vector<double>& S,
                     std::vector<double>& Hb) {
  const int w = 2 * k + 1;
  Hb.assign((size_t)n * w, 0.0);
  for (int j = 0; j < n; ++j)
    for (int d = -k; d <= k; ++d)
      if (j + d >= 0 && j + d < n) Hb[(size_t)j * w + d + k] = S[(size_t)j * n + j + d] / m[j];
}

inline uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

inline float bf16_value(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

}  // namespace qn
