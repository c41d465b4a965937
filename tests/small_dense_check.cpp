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
  if (!(worst_e < 1e-12 && worst_o < 1e-12 && worst_c < 1e-10)) return 1;
  // general eigen-decomposition: random complex matrices, nearly Hermitian
  // ones (a Hermitian matrix plus a small non-Hermitian part, like the
  // projected two-sided Rayleigh matrices), triangular ones (already in
  // Schur form; a random triangular matrix of order 64 has eigenvectors so
  // ill-conditioned that no left vectors are accurate, so its off-diagonal
  // part is scaled down) and ones with a repeated eigenvalue of a
  // diagonalisable matrix
  double worst_r = 0, worst_l = 0, worst_b = 0;
  int cases = 0;
  for (int kind = 0; kind < 4; ++kind) {
    for (int p : {1, 2, 3, 7, 24, 40, 64}) {
      std::vector<cd> a(p * p);
      for (auto& v : a) v = cd(N(g), N(g));
      if (kind == 1) {
        for (int j = 0; j < p; ++j) for (int i = 0; i < j; ++i) { a[j + i * p] = std::conj(a[i + j * p]) + 0.05 * cd(N(g), N(g)); }
        for (int i = 0; i < p; ++i) a[i + i * p] = cd(a[i + i * p].real(), 0.05 * N(g));
      } else if (kind == 2) {  // upper triangular, off-diagonal part scaled so the eigenvectors stay well conditioned
        for (int j = 0; j < p; ++j) for (int i = 0; i < p; ++i) {
          if (i > j) a[i + j * p] = 0.0;
          else if (i < j) a[i + j * p] *= 0.3 / std::sqrt((double)p);
        }
      } else if (kind == 3) {  // S diag(1, 1, 2, 3, ...) S^-1 with S random
        std::vector<cd> sm(p * p), si;
        for (auto& v : sm) v = cd(N(g), N(g));
        if (!lu_inverse(sm, p, si)) { printf("lu failed\n"); return 1; }
        for (int i = 0; i < p; ++i) for (int j = 0; j < p; ++j) {
          cd t = 0; for (int k = 0; k < p; ++k) t += sm[i + k * p] * double(k < 2 ? 1 : k) * si[k + j * p];
          a[i + j * p] = t;
        }
      }
      double an = 0; for (auto& v : a) an += std::norm(v); an = std::sqrt(an);
      std::vector<cd> w, vr, vl;
      if (!eig_general(a, p, w, vr, vl)) { printf("eig_general failed kind %d p %d\n", kind, p); return 1; }
      ++cases;
      for (int j = 0; j < p; ++j) {
        double r = 0, l = 0, ln = 0;
        for (int i = 0; i < p; ++i) {
          cd s = 0, t = 0;
          for (int k = 0; k < p; ++k) { s += a[i + k * p] * vr[k + j * p]; t += std::conj(vl[k + j * p]) * a[k + i * p]; }
          r += std::norm(s - w[j] * vr[i + j * p]);
          l += std::norm(t - w[j] * std::conj(vl[i + j * p]));
          ln += std::norm(vl[i + j * p]);
        }
        worst_r = std::max(worst_r, std::sqrt(r) / an);
        worst_l = std::max(worst_l, std::sqrt(l / ln) / an);
        for (int m = 0; m < p; ++m) {
          cd s = 0; for (int i = 0; i < p; ++i) s += std::conj(vl[i + m * p]) * vr[i + j * p];
          worst_b = std::max(worst_b, std::abs(s - (m == j ? 1.0 : 0.0)));
        }
      }
    }
  }
  printf("eig_general (%d matrices): right resid %.2e left resid %.2e biorth %.2e\n", cases, worst_r, worst_l, worst_b);
  return (worst_r < 1e-12 && worst_l < 1e-10 && worst_b < 1e-9) ? 0 : 1;
}
