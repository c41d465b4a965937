// Deflation of critical eigenvalues (Sec. 2).  With m eigenpairs of A, right
// vectors R = [r_1 .. r_m], left vectors L = [l_1 .. l_m] and L^dag R = I,
//   sgn(A) x = R sgn(Lambda) (L^dag x) + sgn(A) (x - R L^dag x),
// so the Krylov method only sees the projected source.  The kernels here form
// c = L^dag x, the projected source x - R c and the exact part R sgn(Lambda) c,
// on canonical-layout vectors.  Every one streams its columns once from HBM;
// the sums over sites run in a fixed order (per-workgroup partials, then one
// tree per column), so the result does not depend on timing.
#include "nk_internal.h"

namespace nk {

namespace {

constexpr int DT = 256;         // threads per workgroup
constexpr int DE = 8;           // entries per thread in the dot kernel
constexpr int DCH = DT * DE;    // entries per workgroup in the dot kernel
constexpr int AE = 2;           // entries per thread in the combine kernel

__device__ __forceinline__ C64 tree_sum(C64 v, C64* red) {
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = DT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
    __syncthreads();
  }
  return red[0];
}

// part[i * nb + b] = sum over entries of chunk b of conj(a_i[e]) x[e]; i = blockIdx.y
__global__ void __launch_bounds__(DT) k_defl_dot(const C64* __restrict__ a, const C64* __restrict__ x, size_t n,
                                                 int nb, C64* __restrict__ part) {
  __shared__ C64 red[DT];
  const C64* ai = a + (size_t)blockIdx.y * n;
  const size_t base = (size_t)blockIdx.x * DCH + threadIdx.x;
  C64 av[DE], xv[DE];
#pragma unroll
  for (int j = 0; j < DE; ++j) {
    const size_t e = base + (size_t)j * DT;
    av[j] = e < n ? ai[e] : mk(0.0, 0.0);
    xv[j] = e < n ? x[e] : mk(0.0, 0.0);
  }
  C64 acc = mk(0.0, 0.0);
#pragma unroll
  for (int j = 0; j < DE; ++j) acc = acc + cmulc(av[j], xv[j]);
  const C64 s = tree_sum(acc, red);
  if (threadIdx.x == 0) part[(size_t)blockIdx.y * nb + blockIdx.x] = s;
}

// c[i] = sum_b part[i * nb + b], one workgroup per column, fixed order
__global__ void __launch_bounds__(DT) k_defl_reduce(const C64* __restrict__ part, int nb, C64* __restrict__ c) {
  __shared__ C64 red[DT];
  const C64* pi = part + (size_t)blockIdx.x * nb;
  C64 acc = mk(0.0, 0.0);
  for (int b = threadIdx.x; b < nb; b += DT) acc = acc + pi[b];
  const C64 s = tree_sum(acc, red);
  if (threadIdx.x == 0) c[blockIdx.x] = s;
}

// mode 0: out = x - sum_i c_i r_i             (the projected source)
// mode 1: out = out + sum_i s_i c_i r_i       (the exact part, s_i = sgn Re lambda_i)
// The column sum runs in order i = 0 .. m-1 for every entry.
__global__ void __launch_bounds__(DT) k_defl_axpy(const C64* __restrict__ r, size_t n, const C64* __restrict__ c,
                                                  int m, DeflSigns neg, int mode, const C64* __restrict__ x,
                                                  C64* __restrict__ out) {
  __shared__ C64 cs[NK_DEFL_MAX];
  for (int i = threadIdx.x; i < m; i += DT) {
    const C64 ci = c[i];
    const bool flip = mode == 0 || ((neg.w[i >> 6] >> (i & 63)) & 1);
    // a factor of -1 or +1 (exact), not a select between two complex values:
    // the compiler dropped the negation of such a select on the sign-bit path
    const double f = flip ? -1.0 : 1.0;
    cs[i] = mk(f * ci.re, f * ci.im);
  }
  __syncthreads();
  const size_t base = (size_t)blockIdx.x * (DT * AE) + threadIdx.x;
  C64 acc[AE];
#pragma unroll
  for (int j = 0; j < AE; ++j) {
    const size_t e = base + (size_t)j * DT;
    acc[j] = e < n ? (mode == 0 ? x[e] : out[e]) : mk(0.0, 0.0);
  }
#pragma unroll 4
  for (int i = 0; i < m; ++i) {
    const C64 ci = cs[i];
    const C64* ri = r + (size_t)i * n;
#pragma unroll
    for (int j = 0; j < AE; ++j) {
      const size_t e = base + (size_t)j * DT;
      if (e < n) acc[j] = acc[j] + cmul(ri[e], ci);
    }
  }
#pragma unroll
  for (int j = 0; j < AE; ++j) {
    const size_t e = base + (size_t)j * DT;
    if (e < n) out[e] = acc[j];
  }
}

}  // namespace

int defl_partials(size_t n) { return (int)((n + DCH - 1) / DCH); }

int defl_dots(const C64* a, int m, size_t n, const C64* x, C64* part, C64* c, hipStream_t st) {
  if (m <= 0) return NK_OK;
  const int nb = defl_partials(n);
  hipLaunchKernelGGL(k_defl_dot, dim3(nb, m), dim3(DT), 0, st, a, x, n, nb, part);
  hipLaunchKernelGGL(k_defl_reduce, dim3(m), dim3(DT), 0, st, part, nb, c);
  NK_HIP(hipGetLastError());
  return NK_OK;
}

int defl_combine(const C64* r, int m, size_t n, const C64* c, const DeflSigns& neg, int mode, const C64* x, C64* out,
                 hipStream_t st) {
  if (m < 0 || m > NK_DEFL_MAX) {
    set_error("deflation: m = %d outside [0, %d]", m, NK_DEFL_MAX);
    return NK_EINVAL;
  }
  const size_t blocks = (n + DT * AE - 1) / (DT * AE);
  hipLaunchKernelGGL(k_defl_axpy, dim3((unsigned)blocks), dim3(DT), 0, st, r, n, c, m, neg, mode, x, out);
  NK_HIP(hipGetLastError());
  return NK_OK;
}

}  // namespace nk
