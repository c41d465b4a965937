// Host routines on small dense complex matrices (order p <= 128), column-major
// a[i + j * p]: Cholesky factorisation with the inverse of its triangle, the
// cyclic Jacobi eigen-decomposition of a Hermitian matrix, LU inversion and
// the eigen-decomposition (right and left vectors) of a general matrix.  They serve the
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

// LU with partial pivoting of a (overwritten) and the inverse in inv; false
// when a pivot is exactly zero (a singular matrix).
inline bool lu_inverse(std::vector<cd> a, int p, std::vector<cd>& inv) {
  auto A = [&](int i, int j) -> cd& { return a[i + static_cast<size_t>(j) * p]; };
  std::vector<int> perm(p);
  for (int i = 0; i < p; ++i) perm[i] = i;
  for (int k = 0; k < p; ++k) {
    int piv = k;
    for (int i = k + 1; i < p; ++i)
      if (std::abs(A(i, k)) > std::abs(A(piv, k))) piv = i;
    if (A(piv, k) == cd(0.0, 0.0)) return false;
    if (piv != k) {
      for (int j = 0; j < p; ++j) std::swap(A(k, j), A(piv, j));
      std::swap(perm[k], perm[piv]);
    }
    for (int i = k + 1; i < p; ++i) {
      A(i, k) /= A(k, k);
      for (int j = k + 1; j < p; ++j) A(i, j) -= A(i, k) * A(k, j);
    }
  }
  inv.assign(static_cast<size_t>(p) * p, cd(0.0, 0.0));
  for (int c = 0; c < p; ++c) {  // solve A x = e_{perm^-1(c)}: P A = L U, so rows of the unit vector permute
    std::vector<cd> x(p, cd(0.0, 0.0));
    for (int i = 0; i < p; ++i) x[i] = perm[i] == c ? cd(1.0, 0.0) : cd(0.0, 0.0);
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < i; ++j) x[i] -= A(i, j) * x[j];
    for (int i = p - 1; i >= 0; --i) {
      for (int j = i + 1; j < p; ++j) x[i] -= A(i, j) * x[j];
      x[i] /= A(i, i);
    }
    for (int i = 0; i < p; ++i) inv[i + static_cast<size_t>(c) * p] = x[i];
  }
  return true;
}

// Eigen-decomposition of a general complex matrix a (not overwritten):
// eigenvalues w, right eigenvectors as the columns of vr (a vr_i = w_i vr_i,
// unit norm) and left eigenvectors as the columns of vl (vl_i^dag a =
// w_i vl_i^dag) with vl^dag vr = I.  Householder reduction to Hessenberg
// form, then the shifted QR iteration (Wilkinson shifts, an exceptional
// shift every tenth step without deflation) to the complex Schur form
// T = Z^dag a Z; the eigenvectors of T by back substitution, mapped by Z;
// vl = vr^{-dag}.  Returns false if the iteration does not converge or the
// eigenvectors are linearly dependent (a defective matrix).
inline bool eig_general(const std::vector<cd>& a0, int p, std::vector<cd>& w, std::vector<cd>& vr,
                        std::vector<cd>& vl) {
  std::vector<cd> h = a0;
  auto H = [&](int i, int j) -> cd& { return h[i + static_cast<size_t>(j) * p]; };
  std::vector<cd> z(static_cast<size_t>(p) * p, cd(0.0, 0.0));
  auto Z = [&](int i, int j) -> cd& { return z[i + static_cast<size_t>(j) * p]; };
  for (int i = 0; i < p; ++i) Z(i, i) = 1.0;
  double anorm = 0.0;
  for (const cd& v : h) anorm += std::norm(v);
  anorm = std::sqrt(anorm);
  // Hessenberg reduction: reflector I - 2 u u^dag on rows/columns k+1 .. p-1
  for (int k = 0; k + 2 < p; ++k) {
    double xn = 0.0;
    for (int i = k + 1; i < p; ++i) xn += std::norm(H(i, k));
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const cd x0 = H(k + 1, k);
    const cd ph = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : cd(1.0, 0.0);
    std::vector<cd> u(p, cd(0.0, 0.0));
    u[k + 1] = x0 + ph * xn;
    for (int i = k + 2; i < p; ++i) u[i] = H(i, k);
    double un = 0.0;
    for (int i = k + 1; i < p; ++i) un += std::norm(u[i]);
    un = std::sqrt(un);
    if (un == 0.0) continue;
    for (int i = k + 1; i < p; ++i) u[i] /= un;
    for (int j = 0; j < p; ++j) {  // rows: H <- (I - 2 u u^dag) H
      cd s = 0.0;
      for (int i = k + 1; i < p; ++i) s += std::conj(u[i]) * H(i, j);
      for (int i = k + 1; i < p; ++i) H(i, j) -= 2.0 * u[i] * s;
    }
    for (int i = 0; i < p; ++i) {  // columns: H <- H (I - 2 u u^dag), Z likewise
      cd s = 0.0, t = 0.0;
      for (int j = k + 1; j < p; ++j) {
        s += H(i, j) * u[j];
        t += Z(i, j) * u[j];
      }
      for (int j = k + 1; j < p; ++j) {
        H(i, j) -= 2.0 * s * std::conj(u[j]);
        Z(i, j) -= 2.0 * t * std::conj(u[j]);
      }
    }
    for (int i = k + 2; i < p; ++i) H(i, k) = 0.0;
  }
  // QR iteration on the active block [lo, hi]
  const double eps = 1e-15;
  int hi = p - 1, its = 0, total = 0;
  while (hi > 0) {
    int l = hi;
    while (l > 0) {
      const double sc = std::abs(H(l, l)) + std::abs(H(l - 1, l - 1));
      if (std::abs(H(l, l - 1)) <= eps * (sc > 0.0 ? sc : anorm)) break;
      --l;
    }
    if (l > 0) H(l, l - 1) = 0.0;
    if (l == hi) {
      --hi;
      its = 0;
      continue;
    }
    if (++total > 100 * p) return false;
    ++its;
    // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block nearer H(hi, hi)
    cd mu;
    if (its % 10 == 0) {
      mu = H(hi, hi) + cd(std::abs(H(hi, hi - 1)), 0.0) * 0.75;
    } else {
      const cd a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
      const cd tr = a + d, det = a * d - b * c;
      const cd disc = std::sqrt(tr * tr * 0.25 - det);
      const cd l1 = tr * 0.5 + disc, l2 = tr * 0.5 - disc;
      mu = std::abs(l1 - d) < std::abs(l2 - d) ? l1 : l2;
    }
    // one explicit-shift QR step on [l, hi] by Givens rotations, applied to
    // the whole matrix (Schur form) and accumulated in Z
    for (int i = l; i <= hi; ++i) H(i, i) -= mu;
    std::vector<double> cs(hi - l);
    std::vector<cd> sn(hi - l);
    for (int k = l; k < hi; ++k) {
      const cd f = H(k, k), g = H(k + 1, k);
      const double r = std::sqrt(std::norm(f) + std::norm(g));
      double c;
      cd s;
      if (r == 0.0) {
        c = 1.0;
        s = 0.0;
      } else {
        c = std::abs(f) / r;
        const cd fs = std::abs(f) > 0.0 ? f / std::abs(f) : cd(1.0, 0.0);
        s = fs * std::conj(g) / r;
      }
      cs[k - l] = c;
      sn[k - l] = s;
      // rows k, k+1: [c, s; -conj(s), c] applied from the left
      for (int j = k; j < p; ++j) {
        const cd x = H(k, j), y = H(k + 1, j);
        H(k, j) = c * x + s * y;
        H(k + 1, j) = -std::conj(s) * x + c * y;
      }
    }
    for (int k = l; k < hi; ++k) {  // columns k, k+1: the conjugate transpose from the right
      const double c = cs[k - l];
      const cd s = sn[k - l];
      const int rmax = std::min(k + 2, hi);
      for (int i = 0; i <= rmax; ++i) {
        const cd x = H(i, k), y = H(i, k + 1);
        H(i, k) = c * x + std::conj(s) * y;
        H(i, k + 1) = -s * x + c * y;
      }
      for (int i = 0; i < p; ++i) {
        const cd x = Z(i, k), y = Z(i, k + 1);
        Z(i, k) = c * x + std::conj(s) * y;
        Z(i, k + 1) = -s * x + c * y;
      }
    }
    for (int i = l; i <= hi; ++i) H(i, i) += mu;
  }
  // eigenvectors of the upper triangular T = h by back substitution
  w.resize(p);
  for (int i = 0; i < p; ++i) w[i] = H(i, i);
  vr.assign(static_cast<size_t>(p) * p, cd(0.0, 0.0));
  const double small = 1e-300 + eps * anorm;
  for (int k = 0; k < p; ++k) {
    std::vector<cd> x(p, cd(0.0, 0.0));
    x[k] = 1.0;
    for (int i = k - 1; i >= 0; --i) {
      cd s = 0.0;
      for (int j = i + 1; j <= k; ++j) s += H(i, j) * x[j];
      cd den = H(i, i) - w[k];
      if (std::abs(den) < small) den = small;
      x[i] = -s / den;
    }
    double nn = 0.0;
    std::vector<cd> v(p, cd(0.0, 0.0));
    for (int i = 0; i < p; ++i) {
      for (int j = 0; j <= k; ++j) v[i] += Z(i, j) * x[j];
      nn += std::norm(v[i]);
    }
    nn = std::sqrt(nn);
    for (int i = 0; i < p; ++i) vr[i + static_cast<size_t>(k) * p] = v[i] / nn;
  }
  std::vector<cd> inv;
  if (!lu_inverse(vr, p, inv)) return false;
  vl.assign(static_cast<size_t>(p) * p, cd(0.0, 0.0));  // vl = inv^dag
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) vl[i + static_cast<size_t>(j) * p] = std::conj(inv[j + static_cast<size_t>(i) * p]);
  for (const cd& v : vl)
    if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return false;
  return true;
}

}  // namespace dense
}  // namespace nk
