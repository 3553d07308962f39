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
