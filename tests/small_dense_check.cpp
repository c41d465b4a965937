// Checks the host routines of small_dense.h (Cholesky with triangular inverse,
// cyclic Jacobi for Hermitian matrices) on seeded random matrices: eigen-
// residuals, orthonormality, sorted eigenvalues, and X^dag G X = I for the
// inverse Cholesky factor.  Built and run by tests/test_small_dense.py.
#include "small_dense.h"
#include <cstdio>
#include <random>
using namespace nk::dense;
int main() {
  std::mt19937_64 g(1); std::normal_distribution<double> N(0, 1);
  double worst_e = 0, worst_o = 0, worst_c = 0;
  for (int p : {1, 2, 3, 7, 24, 40, 64}) {
    std::vector<cd> a(p * p), a0;
    for (int j = 0; j < p; ++j) for (int i = 0; i <= j; ++i) { cd v(N(g), i == j ? 0.0 : N(g)); a[i + j * p] = v; a[j + i * p] = std::conj(v); }
    a0 = a;
    std::vector<double> w; std::vector<cd> q;
    jacobi_herm(a, p, w, q);
    // residual |A0 q_j - w_j q_j| and orthonormality
    for (int j = 0; j < p; ++j) {
      double r = 0; for (int i = 0; i < p; ++i) { cd s = 0; for (int k = 0; k < p; ++k) s += a0[i + k * p] * q[k + j * p]; r += std::norm(s - w[j] * q[i + j * p]); }
      worst_e = std::max(worst_e, std::sqrt(r));
      for (int l = 0; l < p; ++l) { cd s = 0; for (int i = 0; i < p; ++i) s += std::conj(q[i + l * p]) * q[i + j * p]; worst_o = std::max(worst_o, std::abs(s - (l == j ? 1.0 : 0.0))); }
      if (j) if (w[j] < w[j - 1]) { printf("not sorted\n"); return 1; }
    }
    // Cholesky: G = B^dag B for random B (p x p) + I
    std::vector<cd> b(p * p), gm(p * p, 0.0);
    for (auto& v : b) v = cd(N(g), N(g));
    for (int j = 0; j < p; ++j) for (int i = 0; i < p; ++i) { cd s = 0; for (int k = 0; k < p; ++k) s += std::conj(b[k + i * p]) * b[k + j * p]; gm[i + j * p] = s + (i == j ? 1.0 : 0.0); }
    auto g0 = gm;
    if (!chol_inv_upper(gm, p)) { printf("chol failed\n"); return 1; }
    // X = C^{-1}: check X^dag G X = I
    for (int i = 0; i < p; ++i) for (int j = 0; j < p; ++j) {
      cd s = 0; for (int k = 0; k < p; ++k) for (int l = 0; l < p; ++l) s += std::conj(gm[k + i * p]) * g0[k + l * p] * gm[l + j * p];
      worst_c = std::max(worst_c, std::abs(s - (i == j ? 1.0 : 0.0)));
    }
  }
  printf("jacobi resid %.2e orth %.2e chol %.2e\n", worst_e, worst_o, worst_c);
  return (worst_e < 1e-12 && worst_o < 1e-12 && worst_c < 1e-10) ? 0 : 1;
}
