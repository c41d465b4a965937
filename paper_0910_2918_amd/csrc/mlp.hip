// Learned scaling of the Roberts-Higham iteration of Eq. (4) on gfx950.
//
// The scaled iteration S <- (mu S + (mu S)^{-1}) / 2 has the limit sgn(S)
// for every mu > 0 (the scalar argument of Eq. (7) holds for mu z as well),
// so the factors change only the iteration count.  For the first T steps the
// factor is determinant scaling times a learned correction,
//   mu_t = |det S_t|^{-1/n} exp(y_t),
// with y predicted by a 16-64-64-64-T network (tanh, FP32) from cheap
// features f of S_0:
//   x = (f - mean) * inv_std,  a_l = tanh(W_l a_{l-1} + b_l) (l = 1, 2, 3),
//   y = W4 a3 + b4,
// so y = 0 is plain determinant scaling.  It is trained without labels: each
// eigenvalue of a diagonalisable S_0 follows the scalar map and
// log|det S_t| = sum_i log|z_{i,t}|, so the distance
// d_i = log |z_{i,T} - sgn Re lambda_i| after T steps follows from the
// spectrum; the loss is the smooth maximum (1/kappa) log mean exp(kappa d).
//
// Kernels: features of a batch of dense matrices, forward pass, the
// spectral loss with its gradient, backward pass (per-sample deltas, then one
// thread per weight summing over the batch in a fixed order -- deterministic),
// and Adam.  The sizes are tiny (about 9.7k parameters), so every contraction
// runs on the vector ALUs.
#include <cmath>
#include <mutex>

#include "nk_internal.h"

namespace nk {

constexpr int MI = NK_MLP_IN, MH = NK_MLP_HIDDEN, MT = NK_MLP_STEPS;
// flat parameter offsets
constexpr int OW1 = 0, OB1 = OW1 + MH * MI, OW2 = OB1 + MH, OB2 = OW2 + MH * MH, OW3 = OB2 + MH,
              OB3 = OW3 + MH * MH, OW4 = OB3 + MH, OB4 = OW4 + MT * MH, OMEAN = OB4 + MT, OISTD = OMEAN + MI;
static_assert(OMEAN == NK_MLP_NTRAIN, "trainable block size");
static_assert(OISTD + MI == NK_MLP_NPARAMS, "parameter count");
// FLOOR: squared distance below which an eigenvalue counts as converged (one
// more quadratic step takes 1e-7 to 1e-14); it also keeps the loss free of
// the sharp valleys of log 0
constexpr double KAPPA = 4.0, TINYF = 1e-30, FLOOR = 1e-14;

__device__ __forceinline__ double clampf(double v) { return fmin(50.0, fmax(-50.0, v)); }

__device__ __forceinline__ C64 cdiv1(C64 z) {  // 1 / z
  const double r = 1.0 / norm2(z);
  return mk(z.re * r, -z.im * r);
}

template <class T>
__device__ __forceinline__ T wsum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wmin(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// ---------------------------------------------------------------------------
// features of the dense n x n matrix b (row-major, leading dimension ld); one
// 256-thread workgroup per matrix, O(n^2) reads
__global__ void __launch_bounds__(256) k_rh_features(int ld, const int* __restrict__ nvec,
                                                     const C64* __restrict__ S_b, float* __restrict__ feat) {
  const int b = blockIdx.x;
  const int n = nvec[b];
  const C64* S = S_b + (size_t)b * ld * ld;
  // four consecutive lanes per row i = tid / 4 + 64 m, each adding the
  // columns j = tid % 4 + 4 q of it (row sums, Hermitian defect), met by
  // shuffles; the group's first lane keeps the row's statistics (diagonal
  // entries and the row-sum ones).  The column sums the same way, columns
  // j = tid / 4 + 64 m over rows i = tid % 4 + 4 q.
  const int gr = threadIdx.x >> 2, gl = threadIdx.x & 3;
  double fro = 0, rowmax = 0, colmax = 0, herm = 0, dsq = 0, dmax = 0, dmin = INFINITY, rmin = INFINITY;
  double npos = 0, lsum = 0, lsq = 0, radmax = 0, ncross = 0, tr_re = 0, tr_im = 0;
  for (int i0 = 0; i0 < n; i0 += 64) {
    const int i = i0 + gr;
    double rs = 0, rq = 0, hd = 0;
    if (i < n) {
#pragma unroll 4
      for (int j = gl; j < n; j += 4) {
        const C64 a = S[(size_t)i * ld + j];
        const double m = sqrt(norm2(a));
        rs += m;
        rq += m * m;
        const C64 t = a - conj(S[(size_t)j * ld + i]);
        hd += norm2(t);
      }
    }
#pragma unroll
    for (int o = 1; o < 4; o <<= 1) {
      rs += __shfl_xor(rs, o, 64);
      rq += __shfl_xor(rq, o, 64);
      hd += __shfl_xor(hd, o, 64);
    }
    if (i < n && gl == 0) {
      const C64 d = S[(size_t)i * ld + i];
      const double ad = sqrt(norm2(d));
      fro += rq;
      rowmax = fmax(rowmax, rs);
      herm += hd;
      dsq += ad * ad;
      dmax = fmax(dmax, ad);
      dmin = fmin(dmin, ad);
      rmin = fmin(rmin, fabs(d.re));
      npos += d.re > 0 ? 1.0 : 0.0;
      const double ld_ = log(ad + TINYF);
      lsum += ld_;
      lsq += ld_ * ld_;
      const double rad = rs - ad;
      radmax = fmax(radmax, rad);
      ncross += fabs(d.re) < rad ? 1.0 : 0.0;
      tr_re += d.re;
      tr_im += d.im;
    }
  }
  for (int j0 = 0; j0 < n; j0 += 64) {
    const int j = j0 + gr;
    double cs = 0;
    if (j < n) {
#pragma unroll 4
      for (int i = gl; i < n; i += 4) cs += sqrt(norm2(S[(size_t)i * ld + j]));
    }
#pragma unroll
    for (int o = 1; o < 4; o <<= 1) cs += __shfl_xor(cs, o, 64);
    if (j < n && gl == 0) colmax = fmax(colmax, cs);
  }
  __shared__ double sh[4][16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double sums[9] = {fro, herm, dsq, npos, lsum, lsq, ncross, tr_re, tr_im};
  double maxs[4] = {rowmax, colmax, dmax, radmax};
  double mins[2] = {dmin, rmin};
#pragma unroll
  for (int q = 0; q < 9; ++q) sums[q] = wsum(sums[q]);
#pragma unroll
  for (int q = 0; q < 4; ++q) maxs[q] = wmax(maxs[q]);
#pragma unroll
  for (int q = 0; q < 2; ++q) mins[q] = wmin(mins[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < 9; ++q) sh[w][q] = sums[q];
#pragma unroll
    for (int q = 0; q < 4; ++q) sh[w][9 + q] = maxs[q];
#pragma unroll
    for (int q = 0; q < 2; ++q) sh[w][13 + q] = mins[q];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double v[15];
  for (int q = 0; q < 9; ++q) v[q] = (sh[0][q] + sh[1][q]) + (sh[2][q] + sh[3][q]);
  for (int q = 9; q < 13; ++q) v[q] = fmax(fmax(sh[0][q], sh[1][q]), fmax(sh[2][q], sh[3][q]));
  for (int q = 13; q < 15; ++q) v[q] = fmin(fmin(sh[0][q], sh[1][q]), fmin(sh[2][q], sh[3][q]));
  const double nd = (double)n;
  const double frob = sqrt(v[0]);
  const double rms = frob / sqrt(nd);
  const double lr = log(rms + TINYF);
  const double lmean = v[4] / nd;
  const double lvar = fmax(v[5] / nd - lmean * lmean, 0.0);
  const double offd = sqrt(fmax(v[0] - v[2], 0.0));
  double f[16];
  f[0] = log(nd);
  f[1] = lr;
  f[2] = log(v[9] + TINYF) - lr;
  f[3] = log(v[10] + TINYF) - lr;
  f[4] = v[7] / (nd * (rms + TINYF));
  f[5] = v[8] / (nd * (rms + TINYF));
  f[6] = log(v[11] + TINYF) - lr;
  f[7] = log(v[13] + TINYF) - lr;
  f[8] = log(v[14] + TINYF) - lr;
  f[9] = v[3] / nd;
  f[10] = lmean - lr;
  f[11] = sqrt(lvar);
  f[12] = log(sqrt(v[1]) / (frob + TINYF) + TINYF);
  f[13] = log(offd / (sqrt(v[2]) + TINYF) + TINYF);
  f[14] = log(v[12] + TINYF) - lr;
  f[15] = v[6] / nd;
  for (int q = 0; q < 16; ++q) feat[(size_t)b * MI + q] = (float)clampf(f[q]);
}

// ---------------------------------------------------------------------------
// forward pass: 4 samples per 256-thread workgroup, one thread per unit;
// act (optional) keeps a1, a2, a3 for the backward pass
__global__ void __launch_bounds__(256) k_mlp_fwd(int B, const float* __restrict__ P, const float* __restrict__ feat,
                                                 float* __restrict__ y, float* __restrict__ act) {
  __shared__ float sx[4][MI];
  __shared__ float sa[4][2][MH];
  const int sl = threadIdx.x >> 6, u = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + sl;
  const bool live = b < B;
  if (u < MI) sx[sl][u] = live ? (feat[(size_t)b * MI + u] - P[OMEAN + u]) * P[OISTD + u] : 0.f;
  __syncthreads();
  float h = P[OB1 + u];
  for (int v = 0; v < MI; ++v) h += P[OW1 + u * MI + v] * sx[sl][v];
  float a = tanhf(h);
  sa[sl][0][u] = a;
  if (live && act) act[((size_t)b * 3 + 0) * MH + u] = a;
  __syncthreads();
  h = P[OB2 + u];
  for (int v = 0; v < MH; ++v) h += P[OW2 + u * MH + v] * sa[sl][0][v];
  a = tanhf(h);
  sa[sl][1][u] = a;
  if (live && act) act[((size_t)b * 3 + 1) * MH + u] = a;
  __syncthreads();
  h = P[OB3 + u];
  for (int v = 0; v < MH; ++v) h += P[OW3 + u * MH + v] * sa[sl][1][v];
  a = tanhf(h);
  __syncthreads();
  sa[sl][0][u] = a;
  if (live && act) act[((size_t)b * 3 + 2) * MH + u] = a;
  __syncthreads();
  if (live && u < MT) {
    float o = P[OB4 + u];
    for (int v = 0; v < MH; ++v) o += P[OW4 + u * MH + v] * sa[sl][0][v];
    y[(size_t)b * MT + u] = o;
  }
}

// ---------------------------------------------------------------------------
// spectral loss of sample b (eigenvalues lam[off[b] .. off[b+1])) and its
// gradient with respect to y, scaled by gscale; one workgroup per sample,
// FP64 arithmetic.  Step t uses mu_t = exp(y_t - mean_i log|z_{i,t}|): the
// determinant scale of the eigenvalues times the learned correction.
constexpr int SPT = 4;  // eigenvalues per thread: at most 1024 per matrix

// sum over the 256 threads of the workgroup, the same value in every thread
__device__ __forceinline__ double block_sum256(double v, double* sh) {
  v = wsum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void __launch_bounds__(256) k_spec_loss(const int* __restrict__ off, const C64* __restrict__ lam,
                                                   const float* __restrict__ y, float gscale,
                                                   float* __restrict__ loss, float* __restrict__ dy) {
  __shared__ double sh[4];
  const int b = blockIdx.x;
  const int i0 = off[b], n = off[b + 1] - off[b];
  if (n <= 0) {  // no eigenvalues: nothing to learn from this sample
    if (threadIdx.x < MT) dy[(size_t)b * MT + threadIdx.x] = 0.f;
    if (threadIdx.x == 0) loss[b] = 0.f;
    return;
  }
  C64 z[SPT][MT + 1];
  double sg[SPT], lmu[MT];
#pragma unroll
  for (int r = 0; r < SPT; ++r) {
    const int i = threadIdx.x + r * 256;
    z[r][0] = i < n ? lam[i0 + i] : mk(1.0, 0.0);
    sg[r] = z[r][0].re > 0 ? 1.0 : -1.0;
  }
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    double ls = 0.0;
#pragma unroll
    for (int r = 0; r < SPT; ++r)
      if (threadIdx.x + r * 256 < n) ls += 0.5 * log(norm2(z[r][t]));
    lmu[t] = (double)y[(size_t)b * MT + t] - block_sum256(ls, sh) / n;
    const double mu = exp(lmu[t]);
#pragma unroll
    for (int r = 0; r < SPT; ++r) {
      const C64 wv = mu * z[r][t];
      z[r][t + 1] = 0.5 * (wv + cdiv1(wv));
    }
  }
  double dl[SPT], e[SPT], dmax = -INFINITY;
#pragma unroll
  for (int r = 0; r < SPT; ++r) {
    e[r] = norm2(z[r][MT] - mk(sg[r], 0.0));
    dl[r] = 0.5 * log(e[r] + FLOOR);
    if (threadIdx.x + r * 256 < n) dmax = fmax(dmax, dl[r]);
  }
  dmax = wmax(dmax);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = dmax;
  __syncthreads();
  const double m = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
  double ex[SPT], se = 0.0;
#pragma unroll
  for (int r = 0; r < SPT; ++r) {
    ex[r] = threadIdx.x + r * 256 < n ? exp(KAPPA * (dl[r] - m)) : 0.0;
    se += ex[r];
  }
  const double S = block_sum256(se, sh);
  // backward: gradients as complex numbers dRe + i dIm
  C64 gz[SPT];
#pragma unroll
  for (int r = 0; r < SPT; ++r) gz[r] = (ex[r] / S / (e[r] + FLOOR)) * (z[r][MT] - mk(sg[r], 0.0));
  double g[MT];
#pragma unroll
  for (int t = MT - 1; t >= 0; --t) {
    const double mu = exp(lmu[t]);
    C64 gw[SPT];
    double pg = 0.0;
#pragma unroll
    for (int r = 0; r < SPT; ++r) {
      const C64 wv = mu * z[r][t];
      const C64 dfw = 0.5 * (mk(1.0, 0.0) - cdiv1(cmul(wv, wv)));
      gw[r] = cmulc(dfw, gz[r]);  // conj(f'(w)) gz, through z_{t+1} = (w + 1/w) / 2
      pg += gw[r].re * wv.re + gw[r].im * wv.im;
    }
    const double glm = block_sum256(pg, sh);  // dL/dlog mu_t = dL/dy_t
    g[t] = glm;
    // through w = mu z_t, and through the determinant scale -mean log|z_t|
#pragma unroll
    for (int r = 0; r < SPT; ++r)  // lanes past n stay at zero
      gz[r] = threadIdx.x + r * 256 < n ? mu * gw[r] - (glm / (n * norm2(z[r][t]))) * z[r][t] : mk(0.0, 0.0);
  }
  if (threadIdx.x == 0) {
    loss[b] = (float)(m + log(S / n) / KAPPA);
#pragma unroll
    for (int t = 0; t < MT; ++t) dy[(size_t)b * MT + t] = (float)(gscale * g[t]);
  }
}

// ---------------------------------------------------------------------------
// backward, step 1: per-sample deltas of the three hidden layers
__global__ void __launch_bounds__(256) k_mlp_delta(int B, const float* __restrict__ P, const float* __restrict__ act,
                                                   const float* __restrict__ dy, float* __restrict__ delta) {
  __shared__ float sd[4][MH];
  const int sl = threadIdx.x >> 6, u = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + sl;
  const bool live = b < B;
  const size_t ab = (size_t)(live ? b : 0) * 3 * MH;
  // layer 3: (W4^T dy) * (1 - a3^2)
  float s = 0.f;
  for (int t = 0; t < MT; ++t) s += P[OW4 + t * MH + u] * (live ? dy[(size_t)b * MT + t] : 0.f);
  float a = act[ab + 2 * MH + u];
  float d = s * (1.f - a * a);
  sd[sl][u] = d;
  if (live) delta[ab + 2 * MH + u] = d;
  __syncthreads();
  // layer 2: (W3^T d3) * (1 - a2^2)
  s = 0.f;
  for (int v = 0; v < MH; ++v) s += P[OW3 + v * MH + u] * sd[sl][v];
  a = act[ab + 1 * MH + u];
  d = s * (1.f - a * a);
  __syncthreads();
  sd[sl][u] = d;
  if (live) delta[ab + 1 * MH + u] = d;
  __syncthreads();
  // layer 1: (W2^T d2) * (1 - a1^2)
  s = 0.f;
  for (int v = 0; v < MH; ++v) s += P[OW2 + v * MH + u] * sd[sl][v];
  a = act[ab + 0 * MH + u];
  d = s * (1.f - a * a);
  if (live) delta[ab + 0 * MH + u] = d;
}

// backward, step 2: one thread per trainable parameter, summing over the
// batch in order (deterministic)
__global__ void __launch_bounds__(256) k_mlp_wgrad(int B, const float* __restrict__ P, const float* __restrict__ feat,
                                                   const float* __restrict__ act, const float* __restrict__ dy,
                                                   const float* __restrict__ delta, float* __restrict__ grad) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= NK_MLP_NTRAIN) return;
  float acc = 0.f;
  if (k < OB1) {  // W1[u][v]: delta1[u] x[v]
    const int u = k / MI, v = k % MI;
    const float mv = P[OMEAN + v], iv = P[OISTD + v];
    for (int b = 0; b < B; ++b) acc += delta[((size_t)b * 3 + 0) * MH + u] * ((feat[(size_t)b * MI + v] - mv) * iv);
  } else if (k < OW2) {
    const int u = k - OB1;
    for (int b = 0; b < B; ++b) acc += delta[((size_t)b * 3 + 0) * MH + u];
  } else if (k < OB2) {  // W2[u][v]: delta2[u] a1[v]
    const int u = (k - OW2) / MH, v = (k - OW2) % MH;
    for (int b = 0; b < B; ++b) acc += delta[((size_t)b * 3 + 1) * MH + u] * act[((size_t)b * 3 + 0) * MH + v];
  } else if (k < OW3) {
    const int u = k - OB2;
    for (int b = 0; b < B; ++b) acc += delta[((size_t)b * 3 + 1) * MH + u];
  } else if (k < OB3) {  // W3[u][v]: delta3[u] a2[v]
    const int u = (k - OW3) / MH, v = (k - OW3) % MH;
    for (int b = 0; b < B; ++b) acc += delta[((size_t)b * 3 + 2) * MH + u] * act[((size_t)b * 3 + 1) * MH + v];
  } else if (k < OW4) {
    const int u = k - OB3;
    for (int b = 0; b < B; ++b) acc += delta[((size_t)b * 3 + 2) * MH + u];
  } else if (k < OB4) {  // W4[t][v]: dy[t] a3[v]
    const int t = (k - OW4) / MH, v = (k - OW4) % MH;
    for (int b = 0; b < B; ++b) acc += dy[(size_t)b * MT + t] * act[((size_t)b * 3 + 2) * MH + v];
  } else {
    const int t = k - OB4;
    for (int b = 0; b < B; ++b) acc += dy[(size_t)b * MT + t];
  }
  grad[k] = acc;
}

__global__ void k_adam(int n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float c1, float c2, float lr, float b1, float b2, float eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// y -> exp(y), the correction factor on top of determinant scaling, in FP64
// for the Roberts-Higham kernels; a non-finite or implausible prediction
// becomes -1 (the step then uses determinant scaling alone)
__global__ void k_mu_from_y(int n, const float* __restrict__ y, double* __restrict__ mu) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = (double)y[i];
  mu[i] = (v == v && fabs(v) < 30.0) ? exp(v) : -1.0;
}

// ---------------------------------------------------------------------------
// host side
namespace {
std::mutex g_model_mu;
DevBuf g_model, g_feat, g_y, g_n;
bool g_have_model = false;
}  // namespace

int mlp_features(int batch, int ld, const int* nvec_dev, const C64* S, float* feat, hipStream_t st) {
  hipLaunchKernelGGL(k_rh_features, dim3(batch), dim3(256), 0, st, ld, nvec_dev, S, feat);
  NK_HIP(hipGetLastError());
  return NK_OK;
}

int mlp_forward(int batch, const float* P, const float* feat, float* y, float* act, hipStream_t st) {
  if (batch <= 0) return NK_OK;
  hipLaunchKernelGGL(k_mlp_fwd, dim3((batch + 3) / 4), dim3(256), 0, st, batch, P, feat, y, act);
  NK_HIP(hipGetLastError());
  return NK_OK;
}

int mlp_spectral_loss(int batch, const int* off, const C64* lam, const float* y, float gscale, float* loss,
                      float* dy, hipStream_t st) {
  if (batch <= 0) return NK_OK;
  hipLaunchKernelGGL(k_spec_loss, dim3(batch), dim3(256), 0, st, off, lam, y, gscale, loss, dy);
  NK_HIP(hipGetLastError());
  return NK_OK;
}

int mlp_backward(int batch, const float* P, const float* feat, const float* act, const float* dy, float* delta,
                 float* grad, hipStream_t st) {
  if (batch > 0) hipLaunchKernelGGL(k_mlp_delta, dim3((batch + 3) / 4), dim3(256), 0, st, batch, P, act, dy, delta);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3((NK_MLP_NTRAIN + 255) / 256), dim3(256), 0, st, batch, P, feat, act, dy, delta,
                     grad);
  NK_HIP(hipGetLastError());
  return NK_OK;
}

int mlp_adam(int n, float* p, const float* g, float* m, float* v, int t, float lr, float b1, float b2, float eps,
             hipStream_t st) {
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, t)));
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, n, p, g, m, v, c1, c2, lr, b1, b2, eps);
  NK_HIP(hipGetLastError());
  return NK_OK;
}

int mlp_model_set(const float* params_host) {
  std::lock_guard<std::mutex> lock(g_model_mu);
  if (!params_host) {
    g_have_model = false;
    return NK_OK;
  }
  if (g_model.ensure(NK_MLP_NPARAMS * sizeof(float))) return NK_ENOMEM;
  NK_HIP(hipMemcpy(g_model.p, params_host, NK_MLP_NPARAMS * sizeof(float), hipMemcpyHostToDevice));
  g_have_model = true;
  return NK_OK;
}

// correction factors [batch][NK_MLP_STEPS] (device, FP64) predicted by the
// installed model for the batch of dense matrices S; *have = 0 without a model
int mlp_schedule(int batch, int ld, const int* nvec_dev, const C64* S, double* mu_dev, int* have, hipStream_t st) {
  std::lock_guard<std::mutex> lock(g_model_mu);
  *have = g_have_model ? 1 : 0;
  if (!g_have_model || batch <= 0) return NK_OK;
  if (g_feat.ensure((size_t)batch * MI * sizeof(float)) || g_y.ensure((size_t)batch * MT * sizeof(float)))
    return NK_ENOMEM;
  if (int e = mlp_features(batch, ld, nvec_dev, S, g_feat.as<float>(), st)) return e;
  if (int e = mlp_forward(batch, g_model.as<float>(), g_feat.as<float>(), g_y.as<float>(), nullptr, st)) return e;
  hipLaunchKernelGGL(k_mu_from_y, dim3((batch * MT + 255) / 256), dim3(256), 0, st, batch * MT, g_y.as<float>(),
                     mu_dev);
  NK_HIP(hipGetLastError());
  return NK_OK;
}

}  // namespace nk
