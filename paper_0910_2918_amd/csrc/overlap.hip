// The overlap operator Dov(mu) = 1 + gamma5 sgn(gamma5 Dw(mu)) (Sec. 1,
// Eq. (1)), its adjoint Dov^dag v = v + sgn(gamma5 Dw(-mu)) gamma5 v, and the
// conjugate-gradient method on the normal equations (CGNR) for Dov y = b.
// The sign applications are the library's own (nested or plain, as the
// parameters say); the kernels here are the elementwise gamma5 combinations
// and the CG vector updates, on canonical-layout vectors, where the spin index
// of entry e is (e mod 12) / 3 and gamma5 = diag(1, 1, -1, -1).
#include <cmath>
#include <vector>

#include "nk_internal.h"

namespace nk {

namespace {

constexpr int OT = 256;

__device__ __forceinline__ double g5f(size_t e) { return (e % 12) >= 6 ? -1.0 : 1.0; }

// out = x + gamma5 s
__global__ void __launch_bounds__(OT) k_ov_add_g5(const C64* __restrict__ x, const C64* __restrict__ s,
                                                  C64* __restrict__ out, size_t n) {
  const size_t e = (size_t)blockIdx.x * OT + threadIdx.x;
  if (e >= n) return;
  const double f = g5f(e);
  const C64 a = x[e], b = s[e];
  out[e] = mk(a.re + f * b.re, a.im + f * b.im);
}

// out = gamma5 x
__global__ void __launch_bounds__(OT) k_ov_g5(const C64* __restrict__ x, C64* __restrict__ out, size_t n) {
  const size_t e = (size_t)blockIdx.x * OT + threadIdx.x;
  if (e >= n) return;
  const double f = g5f(e);
  const C64 a = x[e];
  out[e] = mk(f * a.re, f * a.im);
}

// out = x + s (out may be s: each entry is read before it is written)
__global__ void __launch_bounds__(OT) k_ov_add(const C64* __restrict__ x, const C64* s, C64* out, size_t n) {
  const size_t e = (size_t)blockIdx.x * OT + threadIdx.x;
  if (e >= n) return;
  out[e] = x[e] + s[e];
}

// y += a p, r -= a w  (a real)
__global__ void __launch_bounds__(OT) k_cg_step(C64* __restrict__ y, C64* __restrict__ r, const C64* __restrict__ p,
                                                const C64* __restrict__ w, double a, size_t n) {
  const size_t e = (size_t)blockIdx.x * OT + threadIdx.x;
  if (e >= n) return;
  const C64 pv = p[e], wv = w[e], yv = y[e], rv = r[e];
  y[e] = mk(yv.re + a * pv.re, yv.im + a * pv.im);
  r[e] = mk(rv.re - a * wv.re, rv.im - a * wv.im);
}

// p = z + b p  (b real; each entry reads p before writing it)
__global__ void __launch_bounds__(OT) k_cg_dir(C64* p, const C64* __restrict__ z, double b, size_t n) {
  const size_t e = (size_t)blockIdx.x * OT + threadIdx.x;
  if (e >= n) return;
  const C64 pv = p[e], zv = z[e];
  p[e] = mk(zv.re + b * pv.re, zv.im + b * pv.im);
}

dim3 grid_of(size_t n) { return dim3((unsigned)((n + OT - 1) / OT)); }

int worse(int a, int b) { return b > a ? b : a; }

}  // namespace

int overlap_apply(nk_lattice* lat, const nk_sign_params* p, int dagger, const OvDefl& d, const C64* x, C64* y,
                  C64* tmp, nk_sign_info* info, hipStream_t st) {
  const size_t n = (size_t)12 * lat->g.V * p->nrhs;
  int e;
  if (!dagger) {
    // tmp = sgn(A) x, deflated with (lambda, R, L) when given
    e = d.m > 0 ? nk_sign_apply_deflated_device(lat, p, d.m, d.lam, d.R, d.L, x, tmp, info, st)
                : nk_sign_apply_device(lat, p, x, tmp, info, st);
    if (e < 0) return e;
    hipLaunchKernelGGL(k_ov_add_g5, grid_of(n), dim3(OT), 0, st, x, tmp, y, n);
  } else {
    hipLaunchKernelGGL(k_ov_g5, grid_of(n), dim3(OT), 0, st, x, tmp, n);  // tmp = gamma5 x
    nk_sign_params q = *p;
    q.mu = -p->mu;  // A^dag = gamma5 Dw(-mu)
    if (d.m > 0) {
      // A^dag has the conjugate eigenvalues, right eigenvectors L and left
      // eigenvectors R (with R^dag L = I), so its deflation swaps the two
      std::vector<double> lc(d.lam, d.lam + 2 * d.m);
      for (int i = 0; i < d.m; ++i) lc[2 * i + 1] = -lc[2 * i + 1];
      e = nk_sign_apply_deflated_device(lat, &q, d.m, lc.data(), d.L, d.R, tmp, y, info, st);
    } else {
      e = nk_sign_apply_device(lat, &q, tmp, y, info, st);  // y = sgn(A^dag) gamma5 x
    }
    if (e < 0) return e;
    hipLaunchKernelGGL(k_ov_add, grid_of(n), dim3(OT), 0, st, x, y, y, n);
  }
  NK_HIP(hipGetLastError());
  NK_HIP(hipStreamSynchronize(st));
  return e;
}

int overlap_solve(nk_lattice* lat, const nk_sign_params* p, const OvDefl& d, double tol, int maxit, const C64* b,
                  C64* y, int* iters, double* resid, hipStream_t st) {
  const size_t n = (size_t)12 * lat->g.V;
  const int nb = defl_partials(n);
  if (lat->ovl.ensure((5 * n + nb + 2) * sizeof(C64))) return NK_ENOMEM;
  C64* r = lat->ovl.as<C64>();
  C64* z = r + n;
  C64* pd = z + n;
  C64* w = pd + n;
  C64* tmp = w + n;
  C64* part = tmp + n;
  C64* dn = part + nb;  // two squared norms
  *iters = 0;
  *resid = 0.0;
  auto norm2_dev = [&](const C64* v, C64* out) { return defl_dots(v, 1, n, v, part, out, st); };
  auto read = [&](int cnt, double* h) -> int {
    C64 hv[2];
    NK_HIP(hipMemcpyAsync(hv, dn, cnt * sizeof(C64), hipMemcpyDeviceToHost, st));
    NK_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < cnt; ++i) h[i] = hv[i].re;
    return NK_OK;
  };
  double hb = 0.0;
  if (int e = norm2_dev(b, dn)) return e;
  if (int e = read(1, &hb)) return e;
  if (!std::isfinite(hb)) {
    set_error("right-hand side is not finite");
    return NK_EINVAL;
  }
  NK_HIP(hipMemsetAsync(y, 0, n * sizeof(C64), st));
  if (hb == 0.0) {  // y = 0 solves Dov y = 0
    NK_HIP(hipStreamSynchronize(st));
    return NK_OK;
  }
  const double nrm_b = std::sqrt(hb);
  int warn = NK_OK;
  NK_HIP(hipMemcpyAsync(r, b, n * sizeof(C64), hipMemcpyDeviceToDevice, st));
  int e = overlap_apply(lat, p, 1, d, r, z, tmp, nullptr, st);  // z = Dov^dag r
  if (e < 0) return e;
  warn = worse(warn, e);
  NK_HIP(hipMemcpyAsync(pd, z, n * sizeof(C64), hipMemcpyDeviceToDevice, st));
  double zz = 0.0;
  if (int e2 = norm2_dev(z, dn)) return e2;
  if (int e2 = read(1, &zz)) return e2;
  double res = 1.0;
  int it = 0;
  while (it < maxit && res > tol) {
    ++it;
    e = overlap_apply(lat, p, 0, d, pd, w, tmp, nullptr, st);  // w = Dov p
    if (e < 0) return e;
    warn = worse(warn, e);
    double ww = 0.0;
    if (int e2 = norm2_dev(w, dn)) return e2;
    if (int e2 = read(1, &ww)) return e2;
    if (!(ww > 0.0) || !std::isfinite(ww)) {
      set_error("CGNR: |Dov p|^2 = %g at iteration %d", ww, it);
      return NK_EINVAL;
    }
    const double alpha = zz / ww;
    hipLaunchKernelGGL(k_cg_step, grid_of(n), dim3(OT), 0, st, y, r, pd, w, alpha, n);
    NK_HIP(hipGetLastError());
    double rr = 0.0;
    if (int e2 = norm2_dev(r, dn)) return e2;
    if (int e2 = read(1, &rr)) return e2;
    res = std::sqrt(rr) / nrm_b;
    if (res <= tol || it == maxit) break;
    e = overlap_apply(lat, p, 1, d, r, z, tmp, nullptr, st);  // z = Dov^dag r
    if (e < 0) return e;
    warn = worse(warn, e);
    double zn = 0.0;
    if (int e2 = norm2_dev(z, dn)) return e2;
    if (int e2 = read(1, &zn)) return e2;
    hipLaunchKernelGGL(k_cg_dir, grid_of(n), dim3(OT), 0, st, pd, z, zn / zz, n);
    NK_HIP(hipGetLastError());
    zz = zn;
  }
  NK_HIP(hipStreamSynchronize(st));
  *iters = it;
  *resid = res;
  if (res > tol) warn = worse(warn, NK_WARN_NOTCONV);
  return warn;
}

}  // namespace nk
