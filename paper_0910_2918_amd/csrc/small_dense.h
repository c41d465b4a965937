// Host routines on small dense complex matrices (order p <= 128), column-major
// a[i + j * p]: Cholesky factorisation with the inverse of its triangle, and the
// cyclic Jacobi eigen-decomposition of a Hermitian matrix.  They serve the
// block eigensolver, whose p x p Gram and Rayleigh matrices cost O(p^3) per
// pass, negligible beside the O(n p) vector work that runs in kernels.
// Plain C++ with no HIP dependency.
#pragma once

#include <cmath>
#include <complex>
#include <vector>

namespace nk {
namespace dense {

using cd = std::complex<double>;

// G = C^dag C with C upper triangular (G Hermitian positive definite).  On
// success g holds C^{-1} (upper triangular) and the call returns true; it
// returns false when a pivot is not positive.
inline bool chol_inv_upper(std::vector<cd>& g, int p) {
  std::vector<cd> c(static_cast<size_t>(p) * p, cd(0.0, 0.0));
  for (int j = 0; j < p; ++j) {
    for (int i = 0; i <= j; ++i) {
      cd s = g[i + static_cast<size_t>(j) * p];
      for (int k = 0; k < i; ++k) s -= std::conj(c[k + static_cast<size_t>(i) * p]) * c[k + static_cast<size_t>(j) * p];
      if (i == j) {
        if (!(s.real() > 0.0) || !std::isfinite(s.real())) return false;
        c[j + static_cast<size_t>(j) * p] = std::sqrt(s.real());
      } else {
        c[i + static_cast<size_t>(j) * p] = s / c[i + static_cast<size_t>(i) * p];
      }
    }
  }
  // inverse of the upper triangle, column by column: C X = I
  std::vector<cd> x(static_cast<size_t>(p) * p, cd(0.0, 0.0));
  for (int j = 0; j < p; ++j) {
    for (int i = j; i >= 0; --i) {
      cd s = (i == j) ? cd(1.0, 0.0) : cd(0.0, 0.0);
      for (int k = i + 1; k <= j; ++k) s -= c[i + static_cast<size_t>(k) * p] * x[k + static_cast<size_t>(j) * p];
      x[i + static_cast<size_t>(j) * p] = s / c[i + static_cast<size_t>(i) * p];
    }
  }
  g.swap(x);
  return true;
}

// Eigen-decomposition of Hermitian a (overwritten): w ascending, q the
// eigenvectors as columns (unitary).  Cyclic Jacobi: each rotation in the
// (r, s) plane is a phase that makes a_rs real followed by a real rotation
// that zeroes it.
inline void jacobi_herm(std::vector<cd>& a, int p, std::vector<double>& w, std::vector<cd>& q) {
  auto A = [&](int i, int j) -> cd& { return a[i + static_cast<size_t>(j) * p]; };
  q.assign(static_cast<size_t>(p) * p, cd(0.0, 0.0));
  for (int i = 0; i < p; ++i) q[i + static_cast<size_t>(i) * p] = 1.0;
  double total = 0.0;
  for (int j = 0; j < p; ++j)
    for (int i = 0; i < p; ++i) total += std::norm(A(i, j));
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int j = 0; j < p; ++j)
      for (int i = 0; i < j; ++i) off += std::norm(A(i, j));
    if (off <= 1e-32 * total) break;
    for (int r = 0; r < p - 1; ++r) {
      for (int s = r + 1; s < p; ++s) {
        const cd ars = A(r, s);
        const double mag = std::abs(ars);
        if (mag == 0.0) continue;
        const cd ph = ars / mag;  // a_rs = mag * ph
        const double arr = A(r, r).real(), ass = A(s, s).real();
        // real symmetric 2x2 [[arr, mag], [mag, ass]]: rotation angle zeroing mag
        const double tau = (ass - arr) / (2.0 * mag);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = t * cs;
        // unitary J on columns r, s:  J = [[cs, sn * ph], [-sn * conj(ph), cs]]
        //   columns: new_r = cs * col_r - sn * conj(ph) * col_s, new_s = sn * ph * col_r + cs * col_s
        // A <- J^dag A J
        for (int k = 0; k < p; ++k) {  // A J (columns)
          const cd akr = A(k, r), aks = A(k, s);
          A(k, r) = cs * akr - sn * std::conj(ph) * aks;
          A(k, s) = sn * ph * akr + cs * aks;
        }
        for (int k = 0; k < p; ++k) {  // J^dag (A J) (rows)
          const cd ark = A(r, k), ask = A(s, k);
          A(r, k) = cs * ark - sn * ph * ask;
          A(s, k) = sn * std::conj(ph) * ark + cs * ask;
        }
        A(r, s) = 0.0;
        A(s, r) = 0.0;
        A(r, r) = A(r, r).real();
        A(s, s) = A(s, s).real();
        for (int k = 0; k < p; ++k) {  // Q <- Q J
          const cd qkr = q[k + static_cast<size_t>(r) * p], qks = q[k + static_cast<size_t>(s) * p];
          q[k + static_cast<size_t>(r) * p] = cs * qkr - sn * std::conj(ph) * qks;
          q[k + static_cast<size_t>(s) * p] = sn * ph * qkr + cs * qks;
        }
      }
    }
  }
  // sort ascending
  std::vector<int> idx(p);
  for (int i = 0; i < p; ++i) idx[i] = i;
  for (int i = 1; i < p; ++i)
    for (int j = i; j > 0 && A(idx[j], idx[j]).real() < A(idx[j - 1], idx[j - 1]).real(); --j) std::swap(idx[j], idx[j - 1]);
  w.resize(p);
  std::vector<cd> qs(static_cast<size_t>(p) * p);
  for (int j = 0; j < p; ++j) {
    w[j] = A(idx[j], idx[j]).real();
    for (int i = 0; i < p; ++i) qs[i + static_cast<size_t>(j) * p] = q[i + static_cast<size_t>(idx[j]) * p];
  }
  q.swap(qs);
}

}  // namespace dense
}  // namespace nk
