// The critical eigenpairs that deflation treats exactly (Sec. 2), for the
// Hermitian case mu = 0: the m eigenvalues of H = gamma5 Dw(0) smallest in
// modulus, with orthonormal eigenvectors (left = right).  The paper takes them
// from earlier work; the method here is Chebyshev-filtered subspace iteration
// on H^2, which is positive semi-definite, so the wanted eigenvalues are its
// smallest and the filter damps the interval above them:
//   * a block of p >= m vectors is filtered by the degree-d Chebyshev
//     polynomial of H^2 mapped so that [a2, b2] goes to [-1, 1], where b2
//     bounds the spectrum of H^2 ((|4 + m_w| + 8)^2) and a2 is the largest
//     Ritz value of H^2 in the current block;
//   * the block is orthonormalised by Cholesky QR, twice;
//   * Rayleigh-Ritz with H^2 (no spurious interior Ritz values, unlike with
//     the indefinite H) rotates it to Ritz vectors, whose eigenvalue of H is
//     their Rayleigh quotient;
//   * it stops when the m leading residuals |H r - lambda r| are below
//     tol * sqrt(b2).
// Vector work (stencil, Chebyshev steps, Gram matrices, block combinations)
// runs in kernels; the p x p Cholesky and Jacobi steps run on the host.  The
// iteration works in the library's packed device layout, one stencil launch
// per vector: every other step is an inner product or a linear combination,
// which a fixed reordering of the entries leaves unchanged, so the start
// block is packed once and the result unpacked once.
#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "nk_internal.h"
#include "small_dense.h"

namespace nk {

namespace {

constexpr int ET = 256;

// out = a * hy + b * y + c * yold (yold may be NULL: no third term; out may be yold)
__global__ void __launch_bounds__(ET) k_cheb(const C64* __restrict__ hy, const C64* __restrict__ y, const C64* yold,
                                             C64* out, double a, double b, double c, size_t n) {
  const size_t e = (size_t)blockIdx.x * ET + threadIdx.x;
  if (e >= n) return;
  const C64 h = hy[e], v = y[e];
  double re = a * h.re + b * v.re, im = a * h.im + b * v.im;
  if (yold) {
    const C64 o = yold[e];
    re += c * o.re;
    im += c * o.im;
  }
  out[e] = mk(re, im);
}

using dense::cd;

struct EigWork {
  size_t n;
  int p, nb;
  C64* part;  // p * nb partial sums
  C64* dg;    // p * p Gram / Rayleigh matrix
  C64* dm;    // p * p combination coefficients
  C64* zero;  // one zero vector
  hipStream_t st;
};

// h[i + j * p] = a_i^dag a_j for the p columns of a: the upper triangle on the
// device (column j against columns 0 .. j), the lower one by Hermitian symmetry
int gram(const EigWork& w, const C64* a, std::vector<cd>& h) {
  const int p = w.p;
  for (int j = 0; j < p; ++j)
    if (int e = defl_dots(a, j + 1, w.n, a + (size_t)j * w.n, w.part, w.dg + (size_t)j * p, w.st)) return e;
  std::vector<C64> t((size_t)p * p);
  NK_HIP(hipMemcpyAsync(t.data(), w.dg, t.size() * sizeof(C64), hipMemcpyDeviceToHost, w.st));
  NK_HIP(hipStreamSynchronize(w.st));
  h.assign(t.size(), cd(0.0, 0.0));
  for (int j = 0; j < p; ++j)
    for (int i = 0; i <= j; ++i) {
      const cd v(t[i + (size_t)j * p].re, t[i + (size_t)j * p].im);
      h[i + (size_t)j * p] = i == j ? cd(v.real(), 0.0) : v;
      h[j + (size_t)i * p] = i == j ? cd(v.real(), 0.0) : std::conj(v);
    }
  return NK_OK;
}

// out_j = sum_i y_i m[i + j * p] for j < q (out must not overlap y)
int combine(const EigWork& w, const C64* y, const std::vector<cd>& m, int q, C64* out) {
  std::vector<C64> t((size_t)w.p * q);
  for (size_t i = 0; i < t.size(); ++i) t[i] = mk(-m[i].real(), -m[i].imag());  // mode 0 subtracts
  NK_HIP(hipMemcpyAsync(w.dm, t.data(), t.size() * sizeof(C64), hipMemcpyHostToDevice, w.st));
  const DeflSigns none{};
  for (int j = 0; j < q; ++j)
    if (int e = defl_combine(y, w.p, w.n, w.dm + (size_t)j * w.p, none, 0, w.zero, out + (size_t)j * w.n, w.st))
      return e;
  NK_HIP(hipStreamSynchronize(w.st));  // t stays alive until the copy has been consumed
  return NK_OK;
}

// y <- y C^{-1} with y^dag y = C^dag C, twice; tmp is a block of the same size
int orthonormalise(const EigWork& w, C64* y, C64* tmp) {
  std::vector<cd> g;
  for (int pass = 0; pass < 2; ++pass) {
    C64* src = pass == 0 ? y : tmp;
    C64* dst = pass == 0 ? tmp : y;
    if (int e = gram(w, src, g)) return e;
    if (!dense::chol_inv_upper(g, w.p)) {
      set_error("eigensolver: the block lost rank (Gram matrix not positive definite)");
      return NK_EINVAL;
    }
    if (int e = combine(w, src, g, w.p, dst)) return e;
  }
  return NK_OK;
}

}  // namespace

int eig_hermitian(nk_lattice* lat, double m_w, int m, int p, int degree, double tol, int maxit, const C64* v0,
                  double* lam, C64* r_out, int* passes, double* resid, hipStream_t st) {
  const size_t n = (size_t)12 * lat->g.V;
  const int nb = defl_partials(n);
  const size_t blk = (size_t)p * n;
  if (lat->eig.ensure((4 * blk + n + (size_t)p * nb + 2 * (size_t)p * p) * sizeof(C64))) return NK_ENOMEM;
  C64* bufs[4];
  for (int i = 0; i < 4; ++i) bufs[i] = lat->eig.as<C64>() + i * blk;
  EigWork w;
  w.n = n;
  w.p = p;
  w.nb = nb;
  w.zero = bufs[3] + blk;
  w.part = w.zero + n;
  w.dg = w.part + (size_t)p * nb;
  w.dm = w.dg + (size_t)p * p;
  w.st = st;
  NK_HIP(hipMemsetAsync(w.zero, 0, n * sizeof(C64), st));
  C64* V = bufs[0];   // current orthonormal block
  C64* Y = bufs[1];   // filter iterate
  C64* Wb = bufs[2];  // H V, or H^2 Y inside the filter
  C64* T = bufs[3];   // H Y inside the filter, orthonormalisation scratch
  const double hb = std::fabs(4.0 + m_w) + 8.0, b2 = hb * hb;
  const dim3 grid((unsigned)((blk + ET - 1) / ET));
  auto applyH = [&](const C64* x, C64* y) -> int {
    for (int i = 0; i < p; ++i)
      if (int e = nk_apply_dw_packed_device(lat, m_w, 0.0, 1, x + (size_t)i * n, y + (size_t)i * n, st)) return e;
    return NK_OK;
  };

  std::vector<double> t2, th(p), res(p);
  // Rayleigh-Ritz with H^2 on the orthonormal V; leaves V rotated, Wb = H V,
  // th the Rayleigh quotients of H and res the residual norms
  auto rayleigh_ritz = [&]() -> int {
    if (int e = applyH(V, Wb)) return e;
    std::vector<cd> g, q;
    if (int e = gram(w, Wb, g)) return e;  // V^dag H^2 V = (H V)^dag (H V), exactly Hermitian by construction
    dense::jacobi_herm(g, p, t2, q);
    if (int e = combine(w, V, q, p, T)) return e;
    std::swap(V, T);
    if (int e = combine(w, Wb, q, p, T)) return e;
    std::swap(Wb, T);
    // Rayleigh quotients v_i^dag H v_i, then the residual vectors H v_i - th_i v_i (in T) and their norms
    for (int i = 0; i < p; ++i)
      if (int e = defl_dots(V + (size_t)i * n, 1, n, Wb + (size_t)i * n, w.part, w.dg + i, st)) return e;
    std::vector<C64> d(p);
    NK_HIP(hipMemcpyAsync(d.data(), w.dg, p * sizeof(C64), hipMemcpyDeviceToHost, st));
    NK_HIP(hipStreamSynchronize(st));
    std::vector<C64> hth(p);
    for (int i = 0; i < p; ++i) {
      th[i] = d[i].re;
      hth[i] = mk(th[i], 0.0);
    }
    NK_HIP(hipMemcpyAsync(w.dm, hth.data(), p * sizeof(C64), hipMemcpyHostToDevice, st));
    const DeflSigns none{};
    for (int i = 0; i < p; ++i) {
      if (int e = defl_combine(V + (size_t)i * n, 1, n, w.dm + i, none, 0, Wb + (size_t)i * n, T + (size_t)i * n, st))
        return e;
      if (int e = defl_dots(T + (size_t)i * n, 1, n, T + (size_t)i * n, w.part, w.dg + i, st)) return e;
    }
    NK_HIP(hipMemcpyAsync(d.data(), w.dg, p * sizeof(C64), hipMemcpyDeviceToHost, st));
    NK_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < p; ++i) res[i] = std::sqrt(std::max(d[i].re, 0.0));
    return NK_OK;
  };

  if (int e = nk_spinor_pack_device(lat, v0, V, p, st)) return e;
  if (int e = orthonormalise(w, V, T)) return e;
  if (int e = rayleigh_ritz()) return e;
  int it = 0;
  double worst = *std::max_element(res.begin(), res.begin() + m);
  while (it < maxit && worst > tol * hb) {
    ++it;
    double a2 = t2[p - 1];
    if (!(a2 < b2)) a2 = 0.5 * b2;
    const double c = 0.5 * (a2 + b2), e = 0.5 * (b2 - a2);
    // Y_1 = (H^2 V - c V) / e; then Y_{j+1} = 2 (H^2 Y_j - c Y_j) / e - Y_{j-1}, with Y_{j+1} written over Y_{j-1}
    C64* prev = V;
    C64* cur = Y;
    if (int er = applyH(V, T)) return er;
    if (int er = applyH(T, Wb)) return er;
    hipLaunchKernelGGL(k_cheb, grid, dim3(ET), 0, st, Wb, V, (const C64*)nullptr, cur, 1.0 / e, -c / e, 0.0, blk);
    for (int j = 2; j <= degree; ++j) {
      if (int er = applyH(cur, T)) return er;
      if (int er = applyH(T, Wb)) return er;
      hipLaunchKernelGGL(k_cheb, grid, dim3(ET), 0, st, Wb, cur, prev, prev, 2.0 / e, -2.0 * c / e, -1.0, blk);
      std::swap(prev, cur);
    }
    NK_HIP(hipGetLastError());
    // the filtered block is in cur; make it V (Y takes the other buffer)
    if (cur != V) {
      Y = V;
      V = cur;
    }
    if (int er = orthonormalise(w, V, T)) return er;
    if (int er = rayleigh_ritz()) return er;
    worst = *std::max_element(res.begin(), res.begin() + m);
  }
  if (int e = nk_spinor_unpack_device(lat, V, r_out, m, st)) return e;
  NK_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < m; ++i) lam[i] = th[i];
  *passes = it;
  *resid = worst;
  return worst <= tol * hb ? NK_OK : NK_WARN_NOTCONV;
}

}  // namespace nk
