// Outer Krylov basis of Sec. 2 on gfx950: Hermitian Lanczos (mu = 0) and
// two-sided Lanczos (mu != 0), and the lift ||x|| V_k z of Eq. (3).
//
// One step is two kernels.  K1 applies the stencil (the pair A v, A^dag w for
// two-sided Lanczos) with the previous-vector subtraction and the alpha dot
// fused into its epilogue; K2 removes the alpha term, stores the new
// (unnormalised) basis vector and produces the partial sums of its norm (or of
// s = w_hat^dag v_hat).  Normalisation is lazy: column j of V_k holds
// vt_j = v_j / sv[j] and the scale is folded into the next stencil and into
// the lift.  Every reduction is deterministic: each workgroup writes one
// partial sum, and the next kernel's workgroups all reduce the partials in the
// same fixed order, so every workgroup sees bit-identical coefficients and no
// floating-point atomics are used.  Coefficients never leave the device during
// the recurrence.
#include <hip/hip_ext.h>

#include "stencil.h"

namespace nk {

constexpr int NT = 256;

#ifndef NK_SPLIT_PAIR
#define NK_SPLIT_PAIR 1  // 0: one lane per site (both fields); 1: two lanes per site (one per field)
#endif
#ifndef NK_FIELD_MAJOR
#define NK_FIELD_MAJOR 0  // with NK_SPLIT_PAIR: the first half of the grid applies A to v, the second A^dag to w
#endif

template <int NQ>
__device__ __forceinline__ void block_sum(double (&v)[NQ]) {
  __shared__ double sh[NQ][NT / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) sh[q][wid] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = (sh[q][0] + sh[q][1]) + (sh[q][2] + sh[q][3]);
}

template <int NQ>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ part, int nb, double (&v)[NQ]) {
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = 0.0;
  for (int b = threadIdx.x; b < nb; b += NT)
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] += part[q * nb + b];
  block_sum<NQ>(v);
}

// lift accumulation during a second pass: y += lc[j] * vt_j
struct LiftAcc {
  C64* y;          // device layout, FP64; null = no accumulation
  const C64* lc;   // [k] lift coefficients ||x|| z_j sv_j
  int kused;
};

// ---------------------------------------------------------------------------
// start: column 0 of V (and W) = x, partial sums of ||x||^2
template <class R, int NQ>
__global__ void __launch_bounds__(NT) k_start(int n, const C64* __restrict__ x, Cx<R>* __restrict__ v0,
                                              Cx<R>* __restrict__ w0, double* __restrict__ part, LiftAcc lift) {
  double nrm = 0.0;
  const C64 c0 = lift.y ? lift.lc[0] : mk(0.0, 0.0);
  for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
    Cx<R> a = narrow<R>(x[i]);
    v0[i] = a;
    if (w0) w0[i] = a;
    nrm += norm2(widen(a));
    if (lift.y) lift.y[i] = cmul(c0, widen(a));
  }
  double v[1] = {nrm};
  block_sum<1>(v);
  if (threadIdx.x == 0) {
    // Hermitian: [|x|^2]; two-sided: [Re s, Im s, |v|^2, |w|^2] with s = |x|^2
    if (NQ == 1) {
      part[blockIdx.x] = v[0];
    } else {
      part[0 * gridDim.x + blockIdx.x] = v[0];
      part[1 * gridDim.x + blockIdx.x] = 0.0;
      part[2 * gridDim.x + blockIdx.x] = v[0];
      part[3 * gridDim.x + blockIdx.x] = v[0];
    }
  }
}

// ---------------------------------------------------------------------------
// Hermitian Lanczos, K1: w = A v_j - beta_{j-1} v_{j-1}, partial Re(v_j^dag w)
template <class R, class LK>
__global__ void __launch_bounds__(NT) k_lan1(Geom g, LK lk, R diag, int j, const Cx<R>* __restrict__ vj,
                                             const Cx<R>* __restrict__ vjm1, Cx<R>* __restrict__ p,
                                             const double* __restrict__ partIn, int nbIn,
                                             double* __restrict__ partOut, Coefs c) {
  if (c.flags[0]) return;
  double red[1];
  reduce_partials<1>(partIn, nbIn, red);
  const double beta = sqrt(red[0]);
  if (!(beta > 0.0) || !(beta < 1e300)) {  // invariant subspace reached (or non-finite input)
    if (blockIdx.x == 0 && threadIdx.x == 0) c.flags[0] = j > 0 ? j : -1;
    return;
  }
  const double svj = 1.0 / beta;
  const double svjm1 = j > 0 ? c.sv[j - 1] : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c.sv[j] = svj;
    if (j > 0) {
      c.beta[j - 1] = mk(beta, 0.0);
      c.delta[j - 1] = mk(beta, 0.0);
    }
  }
  const double bs = beta * svjm1;
  const int s = xcd_block() * NT + threadIdx.x;
  double dot = 0.0;
  if (s < g.V) {
    Cx<R> acc[1][12];
    const Cx<R>* in[1] = {vj};
    const R one[1] = {R(1)};
    hopping<R, 1>(g, s, lk, in, one, one, acc);
#pragma unroll
    for (int cc = 0; cc < 12; ++cc) {
      const size_t i = (size_t)cc * g.V + s;
      const Cx<R> psi = vj[i];
      Cx<R> a = diag * psi - R(0.5) * acc[0][cc];
      if (cc >= 6) a = mk<R>(-a.re, -a.im);
      C64 w = svj * widen(a);
      if (j > 0) w = w - bs * widen(vjm1[i]);
      const Cx<R> wr = narrow<R>(w);
      p[i] = wr;
      const C64 wd = widen(wr), pd = widen(psi);
      dot += pd.re * wd.re + pd.im * wd.im;
    }
  }
  double v[1] = {dot * svj};
  block_sum<1>(v);
  if (threadIdx.x == 0) partOut[blockIdx.x] = v[0];
}

// Hermitian Lanczos, K2: alpha_j, vt_{j+1} = w - alpha_j v_j, partial |vt_{j+1}|^2
template <class R>
__global__ void __launch_bounds__(NT) k_lan2(int n, int j, const Cx<R>* __restrict__ p, const Cx<R>* __restrict__ vj,
                                             Cx<R>* __restrict__ vnext, const double* __restrict__ partIn, int nbIn,
                                             double* __restrict__ partOut, Coefs c, LiftAcc lift) {
  if (c.flags[0]) return;
  double red[1];
  reduce_partials<1>(partIn, nbIn, red);
  const double alpha = red[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) c.alpha[j] = mk(alpha, 0.0);
  const double as = alpha * c.sv[j];
  const bool acc = lift.y && (j + 1 < lift.kused);
  const C64 lcn = acc ? lift.lc[j + 1] : mk(0.0, 0.0);
  double nrm = 0.0;
  for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
    const C64 v = widen(p[i]) - as * widen(vj[i]);
    const Cx<R> vr = narrow<R>(v);
    vnext[i] = vr;
    const C64 vd = widen(vr);
    nrm += norm2(vd);
    if (acc) lift.y[i] = lift.y[i] + cmul(lcn, vd);
  }
  double v[1] = {nrm};
  block_sum<1>(v);
  if (threadIdx.x == 0) partOut[blockIdx.x] = v[0];
}

// ---------------------------------------------------------------------------
// two-sided Lanczos, K1: the fused pair A v_j, A^dag w_j with
//   p = A v_j - beta_{j-1} v_{j-1},  q = A^dag w_j - delta_{j-1} w_{j-1},
// partial w_j^dag (A v_j) for alpha_j.  It first finishes the previous step:
// s -> delta_{j-1} = sqrt|s|, beta_{j-1} = s / delta_{j-1}, and detects a
// serious breakdown |s| <= 1e-14 |v_hat| |w_hat|.
template <class R, class LK>
__global__ void __launch_bounds__(NT) k_bil1(Geom g, LK lk, R diag, R eft, R ebt, int j,
                                             const Cx<R>* __restrict__ vj, const Cx<R>* __restrict__ wj,
                                             const Cx<R>* __restrict__ vjm1, const Cx<R>* __restrict__ wjm1,
                                             Cx<R>* __restrict__ p, Cx<R>* __restrict__ q,
                                             const double* __restrict__ partIn, int nbIn,
                                             double* __restrict__ partOut, Coefs c) {
  if (c.flags[0]) return;
  double red[4];
  reduce_partials<4>(partIn, nbIn, red);
  const C64 sdot = mk(red[0], red[1]);
  const double sabs = sqrt(norm2(sdot));
  if (j == 0 && !(sabs > 0.0 && sabs < 1e300)) {  // zero or non-finite source
    if (blockIdx.x == 0 && threadIdx.x == 0) c.flags[0] = -1;
    return;
  }
  if (j > 0 && !(sabs > 1e-14 * sqrt(red[2] * red[3]))) {
    if (blockIdx.x == 0 && threadIdx.x == 0) c.flags[0] = j;
    return;
  }
  const double delta = sqrt(sabs);
  const C64 beta = (1.0 / delta) * sdot;
  const double svj = 1.0 / delta;
  const C64 swj = (1.0 / norm2(beta)) * beta;  // 1 / conj(beta)
  double svjm1 = 0.0;
  C64 swjm1 = mk(0.0, 0.0);
  if (j > 0) {
    svjm1 = c.sv[j - 1];
    swjm1 = c.sw[j - 1];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c.sv[j] = svj;
    c.sw[j] = swj;
    if (j > 0) {
      c.beta[j - 1] = beta;
      c.delta[j - 1] = mk(delta, 0.0);
    }
  }
  const C64 bv = svjm1 * beta;  // beta_{j-1} sv_{j-1}
  const C64 dw = delta * swjm1;                                       // delta_{j-1} sw_{j-1}
  const int s = xcd_block() * NT + threadIdx.x;
  double dre = 0.0, dim = 0.0;
  if (s < g.V) {
    Cx<R> acc[2][12];
    const Cx<R>* in[2] = {vj, wj};
    const R ef[2] = {eft, ebt};
    const R eb[2] = {ebt, eft};
    hopping<R, 2>(g, s, lk, in, ef, eb, acc);
#pragma unroll
    for (int cc = 0; cc < 12; ++cc) {
      const size_t i = (size_t)cc * g.V + s;
      const Cx<R> pv = vj[i], pw = wj[i];
      Cx<R> av = diag * pv - R(0.5) * acc[0][cc];
      Cx<R> aw = diag * pw - R(0.5) * acc[1][cc];
      if (cc >= 6) {
        av = mk<R>(-av.re, -av.im);
        aw = mk<R>(-aw.re, -aw.im);
      }
      const C64 avd = widen(av);
      const C64 t = cmulc(widen(pw), avd);
      dre += t.re;
      dim += t.im;
      C64 pp = svj * avd;
      C64 qq = cmul(swj, widen(aw));
      if (j > 0) {
        pp = pp - cmul(bv, widen(vjm1[i]));
        qq = qq - cmul(dw, widen(wjm1[i]));
      }
      p[i] = narrow<R>(pp);
      q[i] = narrow<R>(qq);
    }
  }
  double v[2] = {dre, dim};
  block_sum<2>(v);
  if (threadIdx.x == 0) {
    partOut[blockIdx.x] = v[0];
    partOut[gridDim.x + blockIdx.x] = v[1];
  }
}

// The same step with two lanes per site: the even lane computes A v_j, the
// odd lane A^dag w_j.  Both lanes read the same link addresses in the same
// instruction (one memory request), each lane needs half the registers of
// the two-field version, and twice as many waves are in flight -- at 16^4 the
// one-lane version leaves a single wave per SIMD to hide all load latency.
template <class R, class LK>
__global__ void __launch_bounds__(NT) k_bil1s(Geom g, LK lk, R diag, R eft, R ebt, int j,
                                              const Cx<R>* __restrict__ vj, const Cx<R>* __restrict__ wj,
                                              const Cx<R>* __restrict__ vjm1, const Cx<R>* __restrict__ wjm1,
                                              Cx<R>* __restrict__ p, Cx<R>* __restrict__ q,
                                              const double* __restrict__ partIn, int nbIn,
                                              double* __restrict__ partOut, Coefs c) {
  if (c.flags[0]) return;
  double red[4];
  reduce_partials<4>(partIn, nbIn, red);
  const C64 sdot = mk(red[0], red[1]);
  const double sabs = sqrt(norm2(sdot));
  if (j == 0 && !(sabs > 0.0 && sabs < 1e300)) {  // zero or non-finite source
    if (blockIdx.x == 0 && threadIdx.x == 0) c.flags[0] = -1;
    return;
  }
  if (j > 0 && !(sabs > 1e-14 * sqrt(red[2] * red[3]))) {
    if (blockIdx.x == 0 && threadIdx.x == 0) c.flags[0] = j;
    return;
  }
  const double delta = sqrt(sabs);
  const C64 beta = (1.0 / delta) * sdot;
  const double svj = 1.0 / delta;
  const C64 swj = (1.0 / norm2(beta)) * beta;  // 1 / conj(beta)
  double svjm1 = 0.0;
  C64 swjm1 = mk(0.0, 0.0);
  if (j > 0) {
    svjm1 = c.sv[j - 1];
    swjm1 = c.sw[j - 1];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c.sv[j] = svj;
    c.sw[j] = swj;
    if (j > 0) {
      c.beta[j - 1] = beta;
      c.delta[j - 1] = mk(delta, 0.0);
    }
  }
#if NK_FIELD_MAJOR
  const int half = gridDim.x >> 1;
  const int f = blockIdx.x >= half ? 1 : 0;  // 0: A v_j, 1: A^dag w_j
  int hb = blockIdx.x - f * half;
  if ((half & 7) == 0) hb = (hb & 7) * (half >> 3) + (hb >> 3);
  const int s = hb * NT + threadIdx.x;
#else
  const int f = threadIdx.x & 1;  // 0: A v_j, 1: A^dag w_j
  const int s = xcd_block() * (NT / 2) + (threadIdx.x >> 1);
#endif
  const C64 scale = f ? swj : mk(svj, 0.0);
  const C64 sub = f ? delta * swjm1 : svjm1 * beta;  // delta_{j-1} sw_{j-1} or beta_{j-1} sv_{j-1}
  const Cx<R>* in = f ? wj : vj;
  const Cx<R>* prev = f ? wjm1 : vjm1;
  Cx<R>* out = f ? q : p;
  double dre = 0.0, dim = 0.0;
  if (s < g.V) {
    Cx<R> acc[1][12];
    const Cx<R>* ins[1] = {in};
    const R ef[1] = {f ? ebt : eft};
    const R eb[1] = {f ? eft : ebt};
    hopping<R, 1>(g, s, lk, ins, ef, eb, acc);
#pragma unroll
    for (int cc = 0; cc < 12; ++cc) {
      const size_t i = (size_t)cc * g.V + s;
      Cx<R> a = diag * in[i] - R(0.5) * acc[0][cc];
      if (cc >= 6) a = mk<R>(-a.re, -a.im);
      const C64 ad = widen(a);
      C64 o = cmul(scale, ad);
      if (j > 0) o = o - cmul(sub, widen(prev[i]));
      out[i] = narrow<R>(o);
      if (f == 0) {
        const C64 t = cmulc(widen(wj[i]), ad);
        dre += t.re;
        dim += t.im;
      }
    }
  }
  double v[2] = {dre, dim};
  block_sum<2>(v);
  if (threadIdx.x == 0) {
    partOut[blockIdx.x] = v[0];
    partOut[gridDim.x + blockIdx.x] = v[1];
  }
}

// two-sided Lanczos, K2: alpha_j = conj(sw_j) sv_j (w~_j^dag A v~_j);
//   v_hat = p - alpha_j v_j,  w_hat = q - conj(alpha_j) w_j,
// partial sums of s = w_hat^dag v_hat, |v_hat|^2, |w_hat|^2.
template <class R>
__global__ void __launch_bounds__(NT) k_bil2(int n, int j, const Cx<R>* __restrict__ p, const Cx<R>* __restrict__ q,
                                             const Cx<R>* __restrict__ vj, const Cx<R>* __restrict__ wj,
                                             Cx<R>* __restrict__ vnext, Cx<R>* __restrict__ wnext,
                                             const double* __restrict__ partIn, int nbIn,
                                             double* __restrict__ partOut, Coefs c, LiftAcc lift) {
  if (c.flags[0]) return;
  double red[2];
  reduce_partials<2>(partIn, nbIn, red);
  const double svj = c.sv[j];
  const C64 swj = c.sw[j];
  const C64 alpha = cmul(conj(swj), svj * mk(red[0], red[1]));
  if (blockIdx.x == 0 && threadIdx.x == 0) c.alpha[j] = alpha;
  const C64 av = svj * alpha;
  const C64 aw = cmul(conj(alpha), swj);
  const bool acc = lift.y && (j + 1 < lift.kused);
  const C64 lcn = acc ? lift.lc[j + 1] : mk(0.0, 0.0);
  double sre = 0.0, sim = 0.0, nv = 0.0, nw = 0.0;
  // four elements per thread and iteration: all loads are issued before the
  // first store, which keeps enough bytes in flight to stream at full rate
  constexpr int U = 4;
  const int stride = gridDim.x * NT;
  for (int i0 = blockIdx.x * NT + threadIdx.x; i0 < n; i0 += U * stride) {
    Cx<R> pp[U], qq[U], vv[U], ww[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * stride;
      if (i < n) {
        pp[u] = p[i];
        qq[u] = q[i];
        vv[u] = vj[i];
        ww[u] = wj[i];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * stride;
      if (i < n) {
        const Cx<R> vr = narrow<R>(widen(pp[u]) - cmul(av, widen(vv[u])));
        const Cx<R> wr = narrow<R>(widen(qq[u]) - cmul(aw, widen(ww[u])));
        vnext[i] = vr;
        wnext[i] = wr;
        const C64 vd = widen(vr), wd = widen(wr);
        const C64 t = cmulc(wd, vd);
        sre += t.re;
        sim += t.im;
        nv += norm2(vd);
        nw += norm2(wd);
        if (acc) lift.y[i] = lift.y[i] + cmul(lcn, vd);
      }
    }
  }
  double v[4] = {sre, sim, nv, nw};
  block_sum<4>(v);
  if (threadIdx.x == 0) {
    partOut[0 * gridDim.x + blockIdx.x] = v[0];
    partOut[1 * gridDim.x + blockIdx.x] = v[1];
    partOut[2 * gridDim.x + blockIdx.x] = v[2];
    partOut[3 * gridDim.x + blockIdx.x] = v[3];
  }
}

// ---------------------------------------------------------------------------
// lift: y = sum_j lc[j] vt_j over the stored columns (FP64 accumulation)
template <class R>
__global__ void __launch_bounds__(NT) k_lift(int n, int kused, const Cx<R>* __restrict__ vk, size_t colstride,
                                             const C64* __restrict__ lc, C64* __restrict__ y) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  C64 a0 = mk(0.0, 0.0), a1 = a0, a2 = a0, a3 = a0;
  int j = 0;
  for (; j + 4 <= kused; j += 4) {
    const Cx<R> v0 = vk[(size_t)(j + 0) * colstride + i];
    const Cx<R> v1 = vk[(size_t)(j + 1) * colstride + i];
    const Cx<R> v2 = vk[(size_t)(j + 2) * colstride + i];
    const Cx<R> v3 = vk[(size_t)(j + 3) * colstride + i];
    a0 = a0 + cmul(lc[j + 0], widen(v0));
    a1 = a1 + cmul(lc[j + 1], widen(v1));
    a2 = a2 + cmul(lc[j + 2], widen(v2));
    a3 = a3 + cmul(lc[j + 3], widen(v3));
  }
  for (; j < kused; ++j) a0 = a0 + cmul(lc[j], widen(vk[(size_t)j * colstride + i]));
  y[i] = (a0 + a1) + (a2 + a3);
}

// lc[j] = ||x|| z_j sv_j with ||x|| = 1 / sv[0]
__global__ void k_lift_coef(int k, const C64* __restrict__ z, const double* __restrict__ sv, C64* __restrict__ lc) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < k) lc[j] = (sv[j] / sv[0]) * z[j];
}

// ---------------------------------------------------------------------------
// host side
size_t basis_vector_bytes(const Geom& g, int prec) {
  return (size_t)12 * g.V * (prec == NK_PREC_FP64 ? sizeof(C64) : sizeof(C32));
}

static int nb_elem(const Geom& g) {
  const int n = 12 * g.V;
  int nb = (n + NT - 1) / NT;
  return nb < 512 ? nb : 512;
}

struct BasisBuffers {
  char* vk;        // (k + 1) columns, or a ring of 3 when !store
  size_t colbytes;
  int ncols;       // k + 1 or 3
  char* wring;     // 2 slots (two-sided only)
  char* p;
  char* q;
  double* partA;   // K1 -> K2
  double* partB;   // K2 -> K1
};

static int get_buffers(nk_lattice* lat, const BasisPlan& bp, void* vk_ext, BasisBuffers& b) {
  const Geom& g = lat->g;
  b.colbytes = basis_vector_bytes(g, bp.prec);
  b.ncols = bp.store ? bp.k + 1 : 3;
  const size_t work = 4 * b.colbytes;  // p, q, 2 W slots
  if (lat->work.ensure(work + (bp.store ? 0 : 3 * b.colbytes))) return NK_ENOMEM;
  char* w = lat->work.as<char>();
  b.p = w;
  b.q = w + b.colbytes;
  b.wring = w + 2 * b.colbytes;
  b.vk = bp.store ? (char*)vk_ext : w + 4 * b.colbytes;
  const int nb1 = 2 * ((g.V + NT - 1) / NT) + 1, nb2 = nb_elem(g);
  const int nbmax = nb1 > nb2 ? nb1 : nb2;
  if (lat->part.ensure((size_t)2 * 4 * nbmax * sizeof(double))) return NK_ENOMEM;
  b.partA = lat->part.as<double>();
  b.partB = b.partA + 4 * nbmax;
  return NK_OK;
}

static int prof_event(nk_lattice* lat, hipEvent_t* ev) {
  if (lat->evnext == lat->evpool.size()) {
    hipEvent_t e;
    NK_HIP(hipEventCreate(&e));
    lat->evpool.push_back(e);
  }
  *ev = lat->evpool[lat->evnext++];
  return NK_OK;
}

int prof_collect(nk_lattice* lat, double* t_k1, double* t_k2, int* n_k1, int* n_k2) {
  *t_k1 = *t_k2 = 0.0;
  *n_k1 = *n_k2 = 0;
  for (size_t i = 0; i < lat->evkind.size(); ++i) {
    float ms = 0.f;
    NK_HIP(hipEventElapsedTime(&ms, lat->evpool[2 * i], lat->evpool[2 * i + 1]));
    if (lat->evkind[i] == 0) {
      *t_k1 += ms;
      ++*n_k1;
    } else {
      *t_k2 += ms;
      ++*n_k2;
    }
  }
  lat->evkind.clear();
  lat->evnext = 0;
  return NK_OK;
}

template <class R, class LK>
static int run_steps(nk_lattice* lat, const BasisPlan& bp, const LK& lk, const C64* x, int j0, int j1, Coefs c,
                     BasisBuffers& b, LiftAcc lift, hipStream_t st) {
  const Geom& g = lat->g;
  const int n = 12 * g.V;
  const int nb1 = (g.V + NT - 1) / NT, nb2 = nb_elem(g);
  // two lanes per site; in field-major order each half of the grid covers all sites
  const int nb1s = NK_FIELD_MAJOR ? 2 * ((g.V + NT - 1) / NT) : (2 * g.V + NT - 1) / NT;
  const R diag = (R)(4.0 + bp.m_w);
  auto col = [&](int j) -> Cx<R>* {
    const int s = bp.store ? j : (j % 3);
    return reinterpret_cast<Cx<R>*>(b.vk + (size_t)s * b.colbytes);
  };
  auto wsl = [&](int j) -> Cx<R>* { return reinterpret_cast<Cx<R>*>(b.wring + (size_t)(j & 1) * b.colbytes); };
  Cx<R>* p = reinterpret_cast<Cx<R>*>(b.p);
  Cx<R>* q = reinterpret_cast<Cx<R>*>(b.q);
  if (j0 == 0) {
    if (bp.hermitian)
      hipLaunchKernelGGL((k_start<R, 1>), dim3(nb2), dim3(NT), 0, st, n, x, col(0), (Cx<R>*)nullptr, b.partB, lift);
    else
      hipLaunchKernelGGL((k_start<R, 4>), dim3(nb2), dim3(NT), 0, st, n, x, col(0), wsl(0), b.partB, lift);
    NK_HIP(hipGetLastError());
  }
  // K1 reads the partial sums of the previous K2 (or of k_start), both nb2 wide.
  // When profiling, each launch carries its own start/stop events: the runtime
  // stamps them from the dispatch packet itself, so the elapsed time is the
  // kernel's execution and excludes queueing gaps between launches.
  for (int j = j0; j < j1; ++j) {
    for (int kind = 0; kind < 2; ++kind) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (bp.profile) {
        if (int r = prof_event(lat, &e0)) return r;
        if (int r = prof_event(lat, &e1)) return r;
      }
      if (bp.hermitian) {
        if (kind == 0)
          hipExtLaunchKernelGGL((k_lan1<R, LK>), dim3(nb1), dim3(NT), 0, st, e0, e1, 0, g, lk, diag, j, col(j),
                                j > 0 ? col(j - 1) : col(j), p, b.partB, nb2, b.partA, c);
        else
          hipExtLaunchKernelGGL((k_lan2<R>), dim3(nb2), dim3(NT), 0, st, e0, e1, 0, n, j, p, col(j), col(j + 1),
                                b.partA, nb1, b.partB, c, lift);
      } else {
        const R eft = (R)exp(bp.mu), ebt = (R)exp(-bp.mu);
        const int nbk1 = NK_SPLIT_PAIR ? nb1s : nb1;
        if (kind == 0) {
          if (NK_SPLIT_PAIR)
            hipExtLaunchKernelGGL((k_bil1s<R, LK>), dim3(nb1s), dim3(NT), 0, st, e0, e1, 0, g, lk, diag, eft, ebt, j,
                                  col(j), wsl(j), j > 0 ? col(j - 1) : col(j), j > 0 ? wsl(j - 1) : wsl(j), p, q,
                                  b.partB, nb2, b.partA, c);
          else
            hipExtLaunchKernelGGL((k_bil1<R, LK>), dim3(nb1), dim3(NT), 0, st, e0, e1, 0, g, lk, diag, eft, ebt, j,
                                  col(j), wsl(j), j > 0 ? col(j - 1) : col(j), j > 0 ? wsl(j - 1) : wsl(j), p, q,
                                  b.partB, nb2, b.partA, c);
        } else {
          hipExtLaunchKernelGGL((k_bil2<R>), dim3(nb2), dim3(NT), 0, st, e0, e1, 0, n, j, p, q, col(j), wsl(j),
                                col(j + 1), wsl(j + 1), b.partA, nbk1, b.partB, c, lift);
        }
      }
      NK_HIP(hipGetLastError());
      if (bp.profile) lat->evkind.push_back(kind);
    }
  }
  return NK_OK;
}

template <class R, class LK>
static int dispatch_run(nk_lattice* lat, const BasisPlan& bp, const LK& lk, const C64* x, int j0, int j1, Coefs c,
                        void* vk, LiftAcc lift, hipStream_t st) {
  BasisBuffers b;
  if (int e = get_buffers(lat, bp, vk, b)) return e;
  return run_steps<R, LK>(lat, bp, lk, x, j0, j1, c, b, lift, st);
}

static int run_any(nk_lattice* lat, const BasisPlan& bp, const C64* x, int j0, int j1, Coefs c, void* vk,
                   LiftAcc lift, hipStream_t st) {
  const Geom& g = lat->g;
  if (bp.prec == NK_PREC_FP64)
    return dispatch_run<double>(lat, bp, LinksPlain<double>{lat->U64.as<C64>(), g.V}, x, j0, j1, c, vk, lift, st);
  if (bp.prec == NK_PREC_FP32)
    return dispatch_run<float>(lat, bp, LinksPlain<float>{lat->U32.as<C32>(), g.V}, x, j0, j1, c, vk, lift, st);
  return dispatch_run<float>(lat, bp, LinksBF16{lat->Ubf.as<uint32_t>(), g.V}, x, j0, j1, c, vk, lift, st);
}

int basis_run(nk_lattice* lat, const BasisPlan& bp, const C64* x_canon, int j0, int j1, Coefs c, void* vk,
              hipStream_t st, int* /*unused*/) {
  return run_any(lat, bp, x_canon, j0, j1, c, vk, LiftAcc{nullptr, nullptr, 0}, st);
}

int lift_run(nk_lattice* lat, const BasisPlan& bp, int kused, const C64* z, double, Coefs c, const void* vk,
             C64* y_dev, hipStream_t st) {
  const Geom& g = lat->g;
  const int n = 12 * g.V;
  if (lat->lift.ensure((size_t)kused * sizeof(C64))) return NK_ENOMEM;
  C64* lc = lat->lift.as<C64>();
  hipLaunchKernelGGL(k_lift_coef, dim3((kused + 255) / 256), dim3(256), 0, st, kused, z, c.sv, lc);
  const size_t colstride = (size_t)n;
  if (bp.prec == NK_PREC_FP64)
    hipLaunchKernelGGL(k_lift<double>, dim3((n + NT - 1) / NT), dim3(NT), 0, st, n, kused, (const C64*)vk,
                       colstride, lc, y_dev);
  else
    hipLaunchKernelGGL(k_lift<float>, dim3((n + NT - 1) / NT), dim3(NT), 0, st, n, kused, (const C32*)vk,
                       colstride, lc, y_dev);
  NK_HIP(hipGetLastError());
  return NK_OK;
}

// second pass: rebuild the basis with a ring of three columns and accumulate
// y += lc[j] vt_j as each column appears.  The recurrence runs the same
// kernels on the same data as the first pass, so every column is bit-identical
// to the one the first pass produced.
int two_pass_lift(nk_lattice* lat, const BasisPlan& bp0, const C64* x_canon, int kused, const C64* z, Coefs c,
                  C64* y_dev, hipStream_t st) {
  if (lat->lift.ensure((size_t)kused * sizeof(C64))) return NK_ENOMEM;
  C64* lc = lat->lift.as<C64>();
  hipLaunchKernelGGL(k_lift_coef, dim3((kused + 255) / 256), dim3(256), 0, st, kused, z, c.sv, lc);
  NK_HIP(hipGetLastError());
  BasisPlan bp = bp0;
  bp.store = 0;
  return run_any(lat, bp, x_canon, 0, kused - 1, c, nullptr, LiftAcc{y_dev, lc, kused}, st);
}

}  // namespace nk
