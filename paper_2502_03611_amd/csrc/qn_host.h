// Host-side eigen-data shared by the single-problem and batched contexts.
#pragma once

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
