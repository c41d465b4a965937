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
//     the indefinite H over the whole block) rotates it to Ritz vectors;
//     then Rayleigh-Ritz with H on the leading q >= m of them (q grows past
//     m while their H^2 values repeat) splits the pairs lambda, -lambda that
//     H^2 cannot tell apart (the free field's spectrum is exactly symmetric);
//     the eigenvalue of H of each vector is its Rayleigh quotient;
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

// h[i + j * q] = a_i^dag b_j for the first q columns of a and of b
int gram2(const EigWork& w, const C64* a, const C64* b, int q, std::vector<cd>& h) {
  for (int j = 0; j < q; ++j)
    if (int e = defl_dots(a, q, w.n, b + (size_t)j * w.n, w.part, w.dg + (size_t)j * q, w.st)) return e;
  std::vector<C64> t((size_t)q * q);
  NK_HIP(hipMemcpyAsync(t.data(), w.dg, t.size() * sizeof(C64), hipMemcpyDeviceToHost, w.st));
  NK_HIP(hipStreamSynchronize(w.st));
  h.resize(t.size());
  for (size_t i = 0; i < t.size(); ++i) h[i] = cd(t[i].re, t[i].im);
  return NK_OK;
}

// the squared norms of the p columns of a
int col_norms2(const EigWork& w, const C64* a, std::vector<double>& out) {
  for (int i = 0; i < w.p; ++i)
    if (int e = defl_dots(a + (size_t)i * w.n, 1, w.n, a + (size_t)i * w.n, w.part, w.dg + i, w.st)) return e;
  std::vector<C64> d(w.p);
  NK_HIP(hipMemcpyAsync(d.data(), w.dg, w.p * sizeof(C64), hipMemcpyDeviceToHost, w.st));
  NK_HIP(hipStreamSynchronize(w.st));
  out.resize(w.p);
  for (int i = 0; i < w.p; ++i) out[i] = std::max(d[i].re, 0.0);
  return NK_OK;
}

}  // namespace

// The critical eigenpairs of A = gamma5 Dw(mu) for any mu (Sec. 2, the
// deflation paragraph): the m eigenvalues nearest the imaginary axis, with
// right vectors R (A R = R Lambda) and left vectors L (L^dag A = Lambda
// L^dag), L^dag R = I.  Two-sided filtered subspace iteration:
//   * a right block V and a left block W of p vectors are filtered by the
//     degree-d Chebyshev polynomial in A^2 (V) and in (A^dag)^2 = A(-mu)^2
//     (W), mapped so that [a2, b2] goes to [-1, 1]: b2 bounds |lambda|^2
//     ((|4 + m_w| + 6 + 2 cosh mu)^2: the mass term plus the six spatial and
//     two temporal hops), a2 is the largest Re sigma of the current Ritz
//     values of A^2 (below).  The eigenvalues of A near the imaginary axis have the
//     smallest Re lambda^2 (often below zero), outside that interval, so
//     the filter amplifies them, as long as the spectrum keeps small
//     imaginary parts where |Re lambda| is large (mu of order 0.1-1 on
//     these lattices: |Im lambda| < 0.14 against |Re lambda| up to 6);
//   * both blocks are orthonormalised (Cholesky QR, twice);
//   * two-sided Rayleigh-Ritz in two steps.  First with A^2: with
//     G = W^dag V and K2 = (A^dag W)^dag (A V) = W^dag A^2 V, the p x p
//     eigenproblem of G^{-1} K2 gives values sigma, right coefficients Y and
//     left ones U with U^dag Y = I, so the block rotated to V Y and
//     W G^{-dag} U is biorthonormal, sorted by Re sigma.  Then with A itself
//     on the leading q >= m of these vectors (q grows past m while sigma
//     repeats): the eigenvalues theta of their q x q W^dag A V, which split
//     pairs lambda, -lambda that A^2 cannot tell apart.  Rayleigh-Ritz with
//     A on the whole block would not do: A is indefinite, and a mixture of
//     eigenvectors of large positive and negative eigenvalue has a Rayleigh
//     quotient near zero, a spurious critical value with a large residual
//     (at mu = 0 the iteration then never converges);
//   * the leading q vectors are sorted by |Re theta|, and the iteration
//     stops when the m leading residuals |A r - theta r| / |r| and
//     |A^dag l - conj(theta) l| / |l| are below tol * sqrt(b2).
// Vector work runs in kernels; the p x p steps (LU inverse, Hessenberg QR
// eigen-decomposition) run on the host.
int eig_critical(nk_lattice* lat, double m_w, double mu, int m, int p, int degree, double tol, int maxit,
                 const C64* v0, double* lam, C64* r_out, C64* l_out, int* passes, double* resid, hipStream_t st) {
  const size_t n = (size_t)12 * lat->g.V;
  const int nb = defl_partials(n);
  const size_t blk = (size_t)p * n;
  // dg: p x p; dm: p x p combination coefficients and 2 p per-column scalars
  if (lat->eig.ensure((6 * blk + n + (size_t)p * nb + 2 * (size_t)p * p + 2 * (size_t)p) * sizeof(C64)))
    return NK_ENOMEM;
  C64* V = lat->eig.as<C64>();
  C64* Wl = V + blk;     // left block
  C64* AV = Wl + blk;    // A V
  C64* AW = AV + blk;    // A^dag W
  C64* Y = AW + blk;     // filter iterate
  C64* T = Y + blk;      // scratch
  EigWork w;
  w.n = n;
  w.p = p;
  w.nb = nb;
  w.zero = T + blk;
  w.part = w.zero + n;
  w.dg = w.part + (size_t)p * nb;
  w.dm = w.dg + (size_t)p * p;
  w.st = st;
  NK_HIP(hipMemsetAsync(w.zero, 0, n * sizeof(C64), st));
  const double hb = std::fabs(4.0 + m_w) + 6.0 + 2.0 * std::cosh(mu), b2 = hb * hb;
  const dim3 grid((unsigned)((blk + ET - 1) / ET));
  auto applyA = [&](double mv, const C64* x, C64* y) -> int {
    for (int i = 0; i < p; ++i)
      if (int e = nk_apply_dw_packed_device(lat, m_w, mv, 1, x + (size_t)i * n, y + (size_t)i * n, st)) return e;
    return NK_OK;
  };
  std::vector<cd> th(p), sg(p);
  std::vector<double> rv(p), rw(p), vn(p);
  // the q x q eigenproblem of Gi K (Gi = I when null): values, right and left
  // coefficient matrices (the left ones already mapped by Gi^dag)
  auto small_eig = [&](const std::vector<cd>& K, const std::vector<cd>* Gi, int q, std::vector<cd>& val,
                       std::vector<cd>& yr, std::vector<cd>& zl) -> int {
    std::vector<cd> M = K;
    if (Gi) {
      std::fill(M.begin(), M.end(), cd(0.0, 0.0));
      for (int j = 0; j < q; ++j)
        for (int k = 0; k < q; ++k) {
          const cd kk = K[k + (size_t)j * q];
          for (int i = 0; i < q; ++i) M[i + (size_t)j * q] += (*Gi)[i + (size_t)k * q] * kk;
        }
    }
    std::vector<cd> ul;
    if (!dense::eig_general(M, q, val, yr, ul)) {
      set_error("eigensolver: the projected %d x %d eigenproblem did not converge", q, q);
      return NK_EINVAL;
    }
    if (!Gi) {
      zl = ul;
      return NK_OK;
    }
    zl.assign((size_t)q * q, cd(0.0, 0.0));
    for (int j = 0; j < q; ++j)
      for (int k = 0; k < q; ++k) {
        const cd u = ul[k + (size_t)j * q];
        for (int i = 0; i < q; ++i) zl[i + (size_t)j * q] += std::conj((*Gi)[k + (size_t)i * q]) * u;
      }
    return NK_OK;
  };
  // the columns of yr and zl reordered as idx lists them, into p x p
  // coefficient matrices that leave the columns past q unchanged
  auto reorder = [&](const std::vector<cd>& yr, const std::vector<cd>& zl, int q, const std::vector<int>& idx,
                     std::vector<cd>& Ys, std::vector<cd>& Zs) {
    Ys.assign((size_t)p * p, cd(0.0, 0.0));
    Zs.assign((size_t)p * p, cd(0.0, 0.0));
    for (int j = 0; j < p; ++j) {
      if (j < q) {
        for (int i = 0; i < q; ++i) {
          Ys[i + (size_t)j * p] = yr[i + (size_t)idx[j] * q];
          Zs[i + (size_t)j * p] = zl[i + (size_t)idx[j] * q];
        }
      } else {
        Ys[j + (size_t)j * p] = 1.0;
        Zs[j + (size_t)j * p] = 1.0;
      }
    }
  };
  auto rotate = [&](const std::vector<cd>& Ys, const std::vector<cd>& Zs) -> int {
    if (int e = combine(w, V, Ys, p, T)) return e;
    std::swap(V, T);
    if (int e = combine(w, AV, Ys, p, T)) return e;
    std::swap(AV, T);
    if (int e = combine(w, Wl, Zs, p, T)) return e;
    std::swap(Wl, T);
    if (int e = combine(w, AW, Zs, p, T)) return e;
    std::swap(AW, T);
    return NK_OK;
  };
  // the two Rayleigh-Ritz steps on orthonormal V and W; leaves them rotated
  // (W^dag V = I), sg the Ritz values of A^2, th those of A on the leading
  // q, rv and rw the relative residuals and vn the squared norms of the right
  // Ritz vectors
  auto rayleigh_ritz = [&]() -> int {
    if (int e = applyA(mu, V, AV)) return e;
    if (int e = applyA(-mu, Wl, AW)) return e;
    std::vector<cd> G, K2, Gi, val, yr, zl, Ys, Zs;
    if (int e = gram2(w, Wl, V, p, G)) return e;
    if (int e = gram2(w, AW, AV, p, K2)) return e;
    if (!dense::lu_inverse(G, p, Gi)) {
      set_error("eigensolver: the left and right blocks became orthogonal (W^dag V singular)");
      return NK_EINVAL;
    }
    if (int e = small_eig(K2, &Gi, p, val, yr, zl)) return e;
    std::vector<int> idx(p);
    for (int i = 0; i < p; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return val[x].real() < val[y].real(); });
    for (int j = 0; j < p; ++j) sg[j] = val[idx[j]];
    reorder(yr, zl, p, idx, Ys, Zs);
    if (int e = rotate(Ys, Zs)) return e;
    int q = m;
    while (q < p && std::fabs(sg[q].real() - sg[q - 1].real()) <= 1e-8 * std::fabs(sg[q].real())) ++q;
    std::vector<cd> Kq;
    if (int e = gram2(w, Wl, AV, q, Kq)) return e;  // W^dag V = I on these columns
    if (int e = small_eig(Kq, nullptr, q, val, yr, zl)) return e;
    idx.resize(q);
    for (int i = 0; i < q; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(),
                     [&](int x, int y) { return std::fabs(val[x].real()) < std::fabs(val[y].real()); });
    for (int j = 0; j < q; ++j) th[j] = val[idx[j]];
    for (int j = q; j < p; ++j) th[j] = std::sqrt(sg[j]);  // only for completeness: past q, A^2 values
    reorder(yr, zl, q, idx, Ys, Zs);
    if (int e = rotate(Ys, Zs)) return e;
    // residual vectors A r - theta r (into T) and A^dag l - conj(theta) l (into Y), leading m
    std::vector<C64> tv(m), tw(m);
    for (int i = 0; i < m; ++i) {
      tv[i] = mk(th[i].real(), th[i].imag());
      tw[i] = mk(th[i].real(), -th[i].imag());
    }
    const DeflSigns none{};
    NK_HIP(hipMemcpyAsync(w.dm, tv.data(), m * sizeof(C64), hipMemcpyHostToDevice, st));
    NK_HIP(hipMemcpyAsync(w.dm + m, tw.data(), m * sizeof(C64), hipMemcpyHostToDevice, st));
    for (int i = 0; i < m; ++i) {
      if (int e = defl_combine(V + (size_t)i * n, 1, n, w.dm + i, none, 0, AV + (size_t)i * n, T + (size_t)i * n, st))
        return e;
      if (int e = defl_combine(Wl + (size_t)i * n, 1, n, w.dm + m + i, none, 0, AW + (size_t)i * n,
                               Y + (size_t)i * n, st))
        return e;
    }
    std::vector<double> a2, b2v, wn;
    if (int e = col_norms2(w, T, a2)) return e;
    if (int e = col_norms2(w, Y, b2v)) return e;
    if (int e = col_norms2(w, V, vn)) return e;
    if (int e = col_norms2(w, Wl, wn)) return e;
    for (int i = 0; i < m; ++i) {
      rv[i] = std::sqrt(a2[i] / std::max(vn[i], 1e-300));
      rw[i] = std::sqrt(b2v[i] / std::max(wn[i], 1e-300));
    }
    NK_HIP(hipStreamSynchronize(st));  // tv and tw stay alive until their copies have been consumed
    return NK_OK;
  };
  // the degree-d Chebyshev filter in A(mv)^2 applied to the block x (which
  // ends up holding the result); uses Y, T and the block `hy`
  auto filter = [&](double mv, C64*& x, C64* hy, double a2) -> int {
    const double c = 0.5 * (a2 + b2), e = 0.5 * (b2 - a2);
    C64* prev = x;
    C64* cur = Y;
    if (int er = applyA(mv, x, T)) return er;
    if (int er = applyA(mv, T, hy)) return er;
    hipLaunchKernelGGL(k_cheb, grid, dim3(ET), 0, st, hy, x, (const C64*)nullptr, cur, 1.0 / e, -c / e, 0.0, blk);
    for (int j = 2; j <= degree; ++j) {
      if (int er = applyA(mv, cur, T)) return er;
      if (int er = applyA(mv, T, hy)) return er;
      hipLaunchKernelGGL(k_cheb, grid, dim3(ET), 0, st, hy, cur, prev, prev, 2.0 / e, -2.0 * c / e, -1.0, blk);
      std::swap(prev, cur);
    }
    NK_HIP(hipGetLastError());
    if (cur != x) {  // the filtered block is in cur; x takes it, Y the other buffer
      Y = x;
      x = cur;
    }
    return NK_OK;
  };

  if (int e = nk_spinor_pack_device(lat, v0, V, p, st)) return e;
  NK_HIP(hipMemcpyAsync(Wl, V, blk * sizeof(C64), hipMemcpyDeviceToDevice, st));
  if (int e = orthonormalise(w, V, T)) return e;
  if (int e = orthonormalise(w, Wl, T)) return e;
  if (int e = rayleigh_ritz()) return e;
  auto worst_of = [&]() {
    double x = 0.0;
    for (int i = 0; i < m; ++i) x = std::max(x, std::max(rv[i], rw[i]));
    return x;
  };
  int it = 0;
  double worst = worst_of();
  while (it < maxit && worst > tol * hb) {
    ++it;
    double a2 = 0.0;
    for (int i = 0; i < p; ++i) a2 = std::max(a2, sg[i].real());
    if (!(a2 < b2)) a2 = 0.5 * b2;
    if (int er = filter(mu, V, AV, a2)) return er;
    if (int er = filter(-mu, Wl, AW, a2)) return er;
    if (int er = orthonormalise(w, V, T)) return er;
    if (int er = orthonormalise(w, Wl, T)) return er;
    if (int er = rayleigh_ritz()) return er;
    worst = worst_of();
  }
  // unit right vectors, the left ones scaled to keep l_i^dag r_i = 1
  std::vector<C64> sc(2 * (size_t)m);
  for (int i = 0; i < m; ++i) {
    const double c = std::sqrt(vn[i]);
    sc[i] = mk(-1.0 / c, 0.0);  // the combine kernel subtracts: out = 0 - (-1/c) v
    sc[m + i] = mk(-c, 0.0);
  }
  NK_HIP(hipMemcpyAsync(w.dm, sc.data(), sc.size() * sizeof(C64), hipMemcpyHostToDevice, st));
  const DeflSigns none{};
  for (int i = 0; i < m; ++i) {
    if (int e = defl_combine(V + (size_t)i * n, 1, n, w.dm + i, none, 0, w.zero, T + (size_t)i * n, st)) return e;
    if (int e = defl_combine(Wl + (size_t)i * n, 1, n, w.dm + m + i, none, 0, w.zero, Y + (size_t)i * n, st))
      return e;
  }
  if (int e = nk_spinor_unpack_device(lat, T, r_out, m, st)) return e;
  if (int e = nk_spinor_unpack_device(lat, Y, l_out, m, st)) return e;
  NK_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < m; ++i) {
    lam[2 * i] = th[i].real();
    lam[2 * i + 1] = th[i].imag();
  }
  *passes = it;
  *resid = worst;
  return worst <= tol * hb ? NK_OK : NK_WARN_NOTCONV;
}

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
    // then with H itself on the leading nq >= m vectors (nq grows past m
    // while the H^2 values repeat), which splits pairs lambda, -lambda that
    // H^2 cannot tell apart; sorted by |theta|
    int nq = m;
    while (nq < p && std::fabs(t2[nq] - t2[nq - 1]) <= 1e-8 * std::fabs(t2[nq])) ++nq;
    std::vector<cd> kq, qq;
    if (int e = gram2(w, V, Wb, nq, kq)) return e;
    for (int j = 0; j < nq; ++j)
      for (int i = 0; i <= j; ++i) {
        const cd h = 0.5 * (kq[i + (size_t)j * nq] + std::conj(kq[j + (size_t)i * nq]));
        kq[i + (size_t)j * nq] = i == j ? cd(h.real(), 0.0) : h;
        kq[j + (size_t)i * nq] = i == j ? cd(h.real(), 0.0) : std::conj(h);
      }
    std::vector<double> tq;
    dense::jacobi_herm(kq, nq, tq, qq);
    std::vector<int> idx(nq);
    for (int i = 0; i < nq; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return std::fabs(tq[x]) < std::fabs(tq[y]); });
    q.assign((size_t)p * p, cd(0.0, 0.0));
    for (int j = 0; j < p; ++j) {
      if (j < nq) {
        for (int i = 0; i < nq; ++i) q[i + (size_t)j * p] = qq[i + (size_t)idx[j] * nq];
      } else {
        q[j + (size_t)j * p] = 1.0;
      }
    }
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
