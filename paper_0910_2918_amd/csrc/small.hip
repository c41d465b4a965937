// The small problem of the sign approximation on gfx950: the k-vector z with
// sgn(A) x ~ ||x|| V_k z.
//
//  ell == 0 (non-nested, Eqs. (3)-(4)): z = sgn(H_k) e_1 by Roberts-Higham on
//  the dense k x k Ritz matrix.
//  ell  > 0 (nested, Sec. 3, Eqs. (5)-(6)): B = H_k + H_k^{-1}; an inner
//  Krylov space K_l(B, e_1) (Lanczos for Hermitian H_k, two-sided Lanczos
//  otherwise, full re-(bi)orthogonalisation); z = V_l sgn(H_l) e_1.
//
// H_k^{-1} comes from one LU factorisation of the tridiagonal H_k with
// partial pivoting (U has two super-diagonals), after which k threads solve
// H x = e_j for every column j at once and write B densely; the inner
// iteration then only needs dense mat-vecs with B (and B^dag), which spread
// over the whole GPU, instead of k-long sequential solves inside its loop.
#include <cmath>
#include <vector>

#include "nk_internal.h"

namespace nk {

constexpr int ST = 256;

__device__ __forceinline__ double cabs1s(C64 a) { return fabs(a.re) + fabs(a.im); }
__device__ __forceinline__ C64 cdiv(C64 a, C64 b) {
  const double s = fmax(fabs(b.re), fabs(b.im));
  const double br = b.re / s, bi = b.im / s;
  const double d = (br * br + bi * bi) * s;
  return mk((a.re * br + a.im * bi) / d, (a.im * br - a.re * bi) / d);
}

// LU with partial pivoting of the tridiagonal H (diag alpha, super beta,
// sub delta), one thread.  Row i of U is (1/U0i[i])^{-1}, U1[i], U2[i] on
// columns i, i+1, i+2; Lm[i] is the multiplier eliminating column i of the
// row below the pivot row; Sw[i] says whether rows i and i+1 were exchanged.
__global__ void k_tri_lu(int k, const C64* __restrict__ alpha, const C64* __restrict__ beta,
                         const C64* __restrict__ delta, C64* __restrict__ Lm, int* __restrict__ Sw,
                         C64* __restrict__ U0i, C64* __restrict__ U1, C64* __restrict__ U2, int* __restrict__ sing) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const C64 z = mk(0.0, 0.0);
  C64 a0 = alpha[0], a1 = k > 1 ? beta[0] : z, a2 = z;
  int bad = 0;
  for (int i = 0; i + 1 < k; ++i) {
    const C64 b0 = delta[i], b1 = alpha[i + 1], b2 = (i + 2 < k) ? beta[i + 1] : z;
    C64 p0, p1, p2, o0, o1, o2;
    int sw;
    if (cabs1s(a0) >= cabs1s(b0)) {
      p0 = a0; p1 = a1; p2 = a2; o0 = b0; o1 = b1; o2 = b2; sw = 0;
    } else {
      p0 = b0; p1 = b1; p2 = b2; o0 = a0; o1 = a1; o2 = a2; sw = 1;
    }
    if (!(cabs1s(p0) > 0.0)) bad = 1;
    const C64 m = cdiv(o0, p0);
    U0i[i] = cdiv(mk(1.0, 0.0), p0);
    U1[i] = p1;
    U2[i] = p2;
    Lm[i] = m;
    Sw[i] = sw;
    a0 = o1 - cmul(m, p1);
    a1 = o2 - cmul(m, p2);
    a2 = z;
  }
  if (!(cabs1s(a0) > 0.0)) bad = 1;
  U0i[k - 1] = cdiv(mk(1.0, 0.0), a0);
  U1[k - 1] = z;
  U2[k - 1] = z;
  if (k >= 2) U2[k - 2] = z;
  *sing = bad;
}

// column j of H^{-1} (solve H x = e_j), then B = H + H^{-1}; B row-major k x k
__global__ void __launch_bounds__(64) k_tri_inv(int k, const C64* __restrict__ Lm, const int* __restrict__ Sw,
                                                const C64* __restrict__ U0i, const C64* __restrict__ U1,
                                                const C64* __restrict__ U2, const C64* __restrict__ alpha,
                                                const C64* __restrict__ beta, const C64* __restrict__ delta,
                                                C64* __restrict__ B) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  const C64 z = mk(0.0, 0.0);
  C64 fc = (j == 0) ? mk(1.0, 0.0) : z;
  for (int i = 0; i + 1 < k; ++i) {
    const C64 fn = (i + 1 == j) ? mk(1.0, 0.0) : z;
    const int sw = Sw[i];
    const C64 piv = sw ? fn : fc, oth = sw ? fc : fn;
    B[(size_t)i * k + j] = piv;
    fc = oth - cmul(Lm[i], piv);
  }
  B[(size_t)(k - 1) * k + j] = fc;
  C64 x1 = z, x2 = z;
  for (int i = k - 1; i >= 0; --i) {
    const C64 y = B[(size_t)i * k + j];
    const C64 xi = cmul(y - cmul(U1[i], x1) - cmul(U2[i], x2), U0i[i]);
    B[(size_t)i * k + j] = xi;
    x2 = x1;
    x1 = xi;
  }
  B[(size_t)j * k + j] = B[(size_t)j * k + j] + alpha[j];
  if (j > 0) B[(size_t)(j - 1) * k + j] = B[(size_t)(j - 1) * k + j] + beta[j - 1];
  if (j + 1 < k) B[(size_t)(j + 1) * k + j] = B[(size_t)(j + 1) * k + j] + delta[j];
}

// BH = B^dag (tiled transpose through LDS)
__global__ void k_adjoint(int k, const C64* __restrict__ B, C64* __restrict__ BH) {
  __shared__ C64 t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int yy = threadIdx.y; yy < 32; yy += 8) {
    const int r = by + yy, c = bx + threadIdx.x;
    if (r < k && c < k) t[yy][threadIdx.x] = B[(size_t)r * k + c];
  }
  __syncthreads();
  for (int yy = threadIdx.y; yy < 32; yy += 8) {
    const int r = bx + yy, c = by + threadIdx.x;
    if (r < k && c < k) BH[(size_t)r * k + c] = conj(t[threadIdx.x][yy]);
  }
}

// dense tridiagonal H (ld = k), row-major
__global__ void k_tri_dense(int k, const C64* __restrict__ alpha, const C64* __restrict__ beta,
                            const C64* __restrict__ delta, C64* __restrict__ H) {
  const size_t nn = (size_t)k * k;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / k), j = (int)(e % k);
    C64 v = mk(0.0, 0.0);
    if (i == j) v = alpha[i];
    else if (j == i + 1) v = beta[i];
    else if (i == j + 1) v = delta[j];
    H[e] = v;
  }
}

// ---------------------------------------------------------------------------
// inner Krylov on dense B.  V, W column-major (column j at j*k); u, q the
// work vectors; coefficients a[l], b[l] (super), d[l] (sub); flags[0] =
// breakdown step.
struct Inner {
  int k, herm;
  const C64* B;
  const C64* BH;
  C64* V;
  C64* W;
  C64* uraw[2];  // ping-pong raw vectors (u side)
  C64* qraw[2];  // (q side)
  C64* cproj;    // [l] projections W^dag u
  C64* dproj;    // [l] projections V^dag q
  C64* a;
  C64* b;
  C64* d;
  double* part;  // [4][nb3]
  int nb3;
  int* flags;
};

__device__ __forceinline__ void bsum(double (&v)[4]) {
  __shared__ double sh[4][ST / 64];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < 4; ++q) sh[q][threadIdx.x >> 6] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = (sh[q][0] + sh[q][1]) + (sh[q][2] + sh[q][3]);
}

// IK1: finish step i-1 (normalise), then u = B v_i - beta_{i-1} v_{i-1},
// q = B^dag w_i - delta_{i-1} w_{i-1}.  One wave per row; blockIdx.y = side.
__global__ void __launch_bounds__(ST) k_in_gemv(Inner s, int i) {
  if (s.flags[0]) return;
  const int k = s.k;
  const int side = blockIdx.y;  // 0: u = B v, 1: q = B^dag w
  const C64* src_u = s.uraw[i & 1];
  const C64* src_q = s.qraw[i & 1];
  C64* dst = side ? s.qraw[(i + 1) & 1] : s.uraw[(i + 1) & 1];
  double sv = 1.0;
  C64 sw = mk(1.0, 0.0), beta = mk(0.0, 0.0);
  double delta = 0.0;
  if (i > 0) {
    double v[4] = {0, 0, 0, 0};
    for (int bb = threadIdx.x; bb < s.nb3; bb += ST)
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] += s.part[q * s.nb3 + bb];
    bsum(v);
    C64 sd = mk(v[0], v[1]);
    if (s.herm) sd = mk(v[2], 0.0);
    const double sabs = sqrt(norm2(sd));
    if (!(sabs > 1e-14 * sqrt(v[2] * (s.herm ? v[2] : v[3])))) {
      if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) s.flags[0] = i;
      return;
    }
    delta = sqrt(sabs);
    beta = (1.0 / delta) * sd;
    sv = 1.0 / delta;
    sw = (1.0 / norm2(beta)) * beta;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
      s.b[i - 1] = beta;
      s.d[i - 1] = mk(delta, 0.0);
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = blockIdx.x * (ST / 64) + wave;
  if (r >= k) return;
  const C64* M = side ? s.BH : s.B;
  // this wave also stores the normalised row r of v_i / w_i
  const C64* xs = side ? src_q : src_u;
  const C64 scal = side ? sw : mk(sv, 0.0);
  C64 acc = mk(0.0, 0.0);
  for (int c = lane; c < k; c += 64) {
    const C64 xv = (i > 0) ? cmul(scal, xs[c]) : mk(c == 0 ? 1.0 : 0.0, 0.0);
    acc = acc + cmul(M[(size_t)r * k + c], xv);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    acc.re += __shfl_xor(acc.re, o, 64);
    acc.im += __shfl_xor(acc.im, o, 64);
  }
  if (lane == 0) {
    C64* col = (side ? s.W : s.V) + (size_t)i * k;
    const C64 xr = (i > 0) ? cmul(scal, xs[r]) : mk(r == 0 ? 1.0 : 0.0, 0.0);
    col[r] = xr;
    if (i > 0) {
      const C64* prev = (side ? s.W : s.V) + (size_t)(i - 1) * k;
      acc = acc - cmul(side ? mk(delta, 0.0) : beta, prev[r]);
    }
    dst[r] = acc;
  }
}

// IK2: projections c_j = w_j^dag u and d_j = v_j^dag q for j <= i (blockIdx.y = side)
__global__ void __launch_bounds__(ST) k_in_proj(Inner s, int i, int first) {
  if (s.flags[0]) return;
  const int j = blockIdx.x, side = blockIdx.y, k = s.k;
  const C64* basis = s.herm ? s.V + (size_t)j * k : (side ? s.V : s.W) + (size_t)j * k;
  const C64* x = side ? s.qraw[(i + 1) & 1] : s.uraw[(i + 1) & 1];
  double v[4] = {0, 0, 0, 0};
  for (int r = threadIdx.x; r < k; r += ST) {
    const C64 t = cmulc(basis[r], x[r]);
    v[0] += t.re;
    v[1] += t.im;
  }
  bsum(v);
  if (threadIdx.x == 0) {
    const C64 c = mk(v[0], v[1]);
    (side ? s.dproj : s.cproj)[j] = c;
    if (first && side == 0 && j == i) s.a[i] = s.herm ? mk(c.re, 0.0) : c;
  }
}

// IK3: u -= V c, q -= W d for the rows of this block; with `last`, partial
// sums of s = q^dag u, |u|^2, |q|^2 for the next normalisation
__global__ void __launch_bounds__(ST) k_in_sub(Inner s, int i, int last) {
  if (s.flags[0]) return;
  const int k = s.k;
  const int r = blockIdx.x * ST + threadIdx.x;
  C64* u = s.uraw[(i + 1) & 1];
  C64* q = s.qraw[(i + 1) & 1];
  double v[4] = {0, 0, 0, 0};
  if (r < k) {
    C64 du = mk(0.0, 0.0), dq = mk(0.0, 0.0);
    for (int j = 0; j <= i; ++j) {
      du = du + cmul(s.V[(size_t)j * k + r], s.cproj[j]);
      if (!s.herm) dq = dq + cmul(s.W[(size_t)j * k + r], s.dproj[j]);
    }
    const C64 un = u[r] - du;
    u[r] = un;
    C64 qn = un;
    if (!s.herm) {
      qn = q[r] - dq;
      q[r] = qn;
    }
    const C64 t = cmulc(qn, un);
    v[0] = t.re;
    v[1] = t.im;
    v[2] = norm2(un);
    v[3] = norm2(qn);
  }
  if (!last) return;
  bsum(v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) s.part[qq * s.nb3 + blockIdx.x] = v[qq];
}

// z = V y (k rows, l columns)
__global__ void k_in_lift(int k, int l, const C64* __restrict__ V, const C64* __restrict__ S, int lds,
                          C64* __restrict__ z) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= k) return;
  C64 acc = mk(0.0, 0.0);
  for (int j = 0; j < l; ++j) acc = acc + cmul(V[(size_t)j * k + r], S[(size_t)j * lds]);
  z[r] = acc;
}

// z = column 0 of S (ld = k)
__global__ void k_col0(int k, const C64* __restrict__ S, C64* __restrict__ z) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < k) z[r] = S[(size_t)r * k];
}

// ---------------------------------------------------------------------------
namespace {
DevBuf g_small;
}

int small_sign_dev(int k, int ell, int hermitian, const C64* alpha, const C64* beta, const C64* delta,
                   int rh_scaling, int rh_maxit, double rh_tol, C64* z, SmallOut* out, hipStream_t st,
                   const double* mu_sched, int mu_steps) {
  if (k <= 0) return NK_EINVAL;
  if (ell > k) ell = k;
  if (ell <= 0) {
    // non-nested: RH on dense H_k
    if (g_small.ensure((size_t)k * k * sizeof(C64))) return NK_ENOMEM;
    C64* H = g_small.as<C64>();
    hipLaunchKernelGGL(k_tri_dense, dim3(1024), dim3(256), 0, st, k, alpha, beta, delta, H);
    NK_HIP(hipGetLastError());
    int it = 0;
    double res = 0;
    int e = rh_sign_batched(1, k, &k, H, rh_scaling, rh_maxit, rh_tol, &it, &res, st, mu_sched, mu_steps);
    if (e < 0) return e;
    hipLaunchKernelGGL(k_col0, dim3((k + 255) / 256), dim3(256), 0, st, k, H, z);
    NK_HIP(hipGetLastError());
    if (out) {
      out->rh_iters = it;
      out->ell_used = 0;
      out->rh_residual = res;
    }
    return e;
  }
  // nested
  const int nb3 = (k + ST - 1) / ST;
  const size_t kk = (size_t)k * k;
  size_t bytes = 0;
  auto take = [&](size_t b) {
    size_t o = bytes;
    bytes += (b + 255) & ~(size_t)255;
    return o;
  };
  const size_t oB = take(kk * sizeof(C64));
  const size_t oBH = take(hermitian ? 0 : kk * sizeof(C64));
  const size_t oV = take((size_t)k * ell * sizeof(C64));
  const size_t oW = take(hermitian ? 0 : (size_t)k * ell * sizeof(C64));
  const size_t oR = take((size_t)4 * k * sizeof(C64));
  const size_t oF = take((size_t)5 * k * sizeof(C64) + (size_t)k * sizeof(int));
  const size_t oC = take((size_t)5 * ell * sizeof(C64));
  const size_t oP = take((size_t)4 * nb3 * sizeof(double));
  const size_t oS = take((size_t)ell * ell * sizeof(C64));
  const size_t oI = take(8 * sizeof(int));
  if (g_small.ensure(bytes)) return NK_ENOMEM;
  char* base = g_small.as<char>();
  Inner s;
  s.k = k;
  s.herm = hermitian;
  s.B = (C64*)(base + oB);
  s.BH = hermitian ? s.B : (C64*)(base + oBH);
  s.V = (C64*)(base + oV);
  s.W = hermitian ? s.V : (C64*)(base + oW);
  C64* R = (C64*)(base + oR);
  s.uraw[0] = R;
  s.uraw[1] = R + k;
  s.qraw[0] = R + 2 * k;
  s.qraw[1] = R + 3 * k;
  C64* F = (C64*)(base + oF);
  C64 *Lm = F, *U0i = F + k, *U1 = F + 2 * k, *U2 = F + 3 * k;
  int* Sw = (int*)(F + 5 * k);
  C64* Cc = (C64*)(base + oC);
  s.cproj = Cc;
  s.dproj = Cc + ell;
  s.a = Cc + 2 * ell;
  s.b = Cc + 3 * ell;
  s.d = Cc + 4 * ell;
  s.part = (double*)(base + oP);
  s.nb3 = nb3;
  C64* Hl = (C64*)(base + oS);
  int* iflags = (int*)(base + oI);
  s.flags = iflags;
  NK_HIP(hipMemsetAsync(iflags, 0, 8 * sizeof(int), st));
  NK_HIP(hipMemsetAsync(s.b, 0, 2 * ell * sizeof(C64), st));

  hipLaunchKernelGGL(k_tri_lu, dim3(1), dim3(64), 0, st, k, alpha, beta, delta, Lm, Sw, U0i, U1, U2, iflags + 1);
  hipLaunchKernelGGL(k_tri_inv, dim3((k + 63) / 64), dim3(64), 0, st, k, Lm, Sw, U0i, U1, U2, alpha, beta, delta,
                     (C64*)s.B);
  if (!hermitian) hipLaunchKernelGGL(k_adjoint, dim3((k + 31) / 32, (k + 31) / 32), dim3(32, 8), 0, st, k, s.B,
                                     (C64*)s.BH);
  NK_HIP(hipGetLastError());
  const int sides = hermitian ? 1 : 2;
  for (int i = 0; i < ell; ++i) {
    hipLaunchKernelGGL(k_in_gemv, dim3((k + 3) / 4, sides), dim3(ST), 0, st, s, i);
    hipLaunchKernelGGL(k_in_proj, dim3(i + 1, sides), dim3(ST), 0, st, s, i, 1);
    if (i + 1 < ell) {
      hipLaunchKernelGGL(k_in_sub, dim3(nb3), dim3(ST), 0, st, s, i, 0);
      hipLaunchKernelGGL(k_in_proj, dim3(i + 1, sides), dim3(ST), 0, st, s, i, 0);
      hipLaunchKernelGGL(k_in_sub, dim3(nb3), dim3(ST), 0, st, s, i, 1);
    }
  }
  NK_HIP(hipGetLastError());
  int fl[2] = {0, 0};
  NK_HIP(hipMemcpyAsync(fl, iflags, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  NK_HIP(hipStreamSynchronize(st));
  if (fl[1]) {
    set_error("nested small problem: H_k is singular");
    return NK_WARN_NOTCONV;
  }
  const int lu = fl[0] ? fl[0] : ell;
  hipLaunchKernelGGL(k_tri_dense, dim3(256), dim3(256), 0, st, lu, s.a, s.b, s.d, Hl);
  NK_HIP(hipGetLastError());
  int it = 0;
  double res = 0;
  int e = rh_sign_batched(1, lu, &lu, Hl, rh_scaling, rh_maxit, rh_tol, &it, &res, st, mu_sched, mu_steps);
  if (e < 0) return e;
  hipLaunchKernelGGL(k_in_lift, dim3((k + 255) / 256), dim3(256), 0, st, k, lu, s.V, Hl, lu, z);
  NK_HIP(hipGetLastError());
  if (out) {
    out->rh_iters = it;
    out->ell_used = lu;
    out->rh_residual = res;
  }
  return e ? e : (fl[0] ? NK_WARN_BREAKDOWN : NK_OK);
}

}  // namespace nk
