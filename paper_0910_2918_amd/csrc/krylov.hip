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

#ifndef NK_AUTOTUNE
#define NK_AUTOTUNE 1  // choose the direction groups of K1 by timing both on first use
#endif

// v from the lane that the DPP pattern CTRL selects (a row shift or a row
// broadcast, in the rows of ROWMASK), 0.0 where the pattern has no source
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_take(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, ROWMASK, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// sum over the 64 lanes of a wave in a fixed order (DPP row shifts, then the
// row broadcasts; lane 63 ends with the total), returned in every lane
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_take<0x111, 0xf>(v);  // row_shr:1
  v += dpp_take<0x112, 0xf>(v);  // row_shr:2
  v += dpp_take<0x114, 0xf>(v);  // row_shr:4
  v += dpp_take<0x118, 0xf>(v);  // row_shr:8
  v += dpp_take<0x142, 0xa>(v);  // row_bcast:15
  v += dpp_take<0x143, 0xc>(v);  // row_bcast:31
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int NQ>
__device__ __forceinline__ void block_sum(double (&v)[NQ]) {
  __shared__ double sh[NQ][NT / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = wave_sum(v[q]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) sh[q][wid] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = (sh[q][0] + sh[q][1]) + (sh[q][2] + sh[q][3]);
}

// two consecutive partial sums (b, b + 1) of an array of nb in one 16-byte
// load, 0 for b >= nb.  Partial arrays have an even count per quantity
// (every producer launches an even number of workgroups), so pairs never
// straddle two quantities.  The load itself is unconditional (pair 0 stands
// in past the end), so a batch of them is issued back to back instead of one
// branch and one wait per load.
__device__ __forceinline__ double pair_sum(const double* __restrict__ part, int b, int nb) {
  const bool in = b < nb;
  const double2 t = *reinterpret_cast<const double2*>(part + (in ? b : 0));
  return in ? t.x + t.y : 0.0;
}

// sum of nb (even) partial sums per quantity, the same value in every
// thread; the loads go out four pairs at a time so that long partial arrays
// cost one or two L2 round trips, not one per element
template <int NQ>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ part, int nb, double (&v)[NQ]) {
  constexpr int B = 4;
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = 0.0;
  for (int b0 = 2 * threadIdx.x; b0 < nb; b0 += 2 * B * NT) {
    double t[NQ][B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int b = b0 + 2 * u * NT;
#pragma unroll
      for (int q = 0; q < NQ; ++q) t[q][u] = pair_sum(part + q * nb, b, nb);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double a = 0.0;
#pragma unroll
      for (int u = 0; u < B; ++u) a += t[q][u];
      v[q] += a;
    }
  }
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
  const int V = n / 12;
  for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
    Cx<R> a = narrow<R>(x[i]);  // x and y in the FP64 layout, v0 and w0 in that of R
    const size_t ir = sidx_of64<R>(V, i);
    v0[ir] = a;
    if (w0) w0[ir] = a;
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
// Hermitian Lanczos, K1: w = A v_j - beta_{j-1} v_{j-1}, partial Re(v_j^dag w).
// Directions split over the waves of the workgroup (hop_group), one lane per
// site, 64 sites per wave.  The previous partial sums are loaded before the
// stencil and reduced after it, so their latency hides behind the stencil
// loads.
template <class R, class LK, int NG>
__global__ void __launch_bounds__(NT) k_lan1(Geom g, LK lk, R diag, int j, const Cx<R>* __restrict__ vj,
                                             const Cx<R>* __restrict__ vjm1, Cx<R>* __restrict__ p,
                                             const double* __restrict__ partIn, int nbIn,
                                             double* __restrict__ partOut, Coefs c) {
  constexpr int M = 12 / NG;
  constexpr int NSB = (NT / 64) / NG;  // site blocks of 64 per workgroup
  __shared__ XBuf<R, NG> xb;
  const int flag = c.flags[0];
  // this thread's pair of the previous partial sums (nbIn <= 2 NT, even)
  const double pr = pair_sum(partIn, 2 * threadIdx.x, nbIn);
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gi = w % NG, sb = w / NG;
  const int s = (xcd_block() * NSB + sb) * 64 + lane;
  const bool live = s < g.V;
  Cx<R> mine[M];
  hop_group<NG>(g, live ? s : 0, lk, vj, gi, R(1), R(1), xb, w, lane, mine);  // a lane past the end hops at site 0
  // the site's own operands of the epilogue, loaded before the reduction so
  // that their latency overlaps it
  Cx<R> ein[M], eprev[M];
  {
    int se = live ? s : 0;
    asm volatile("" : "+v"(se));  // keeps these addresses out of the stencil's registers
#pragma unroll
    for (int cl = 0; cl < M; ++cl) {
      const size_t i = sidx<R>(g.V, gi * M + cl, se);
      ein[cl] = vj[i];
      eprev[cl] = j > 0 ? vjm1[i] : mk<R>(0, 0);
    }
  }
  if (flag) return;
  double red[1] = {pr};
  block_sum<1>(red);  // also completes the exchange
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
  double dot = 0.0;
  if (live) {
    int se = s;
    asm volatile("" : "+v"(se));  // keeps the epilogue addresses out of the stencil's registers
#pragma unroll
    for (int cl = 0; cl < M; ++cl) {
      const int cc = gi * M + cl;
      const Cx<R> hs = xsum<NG>(xb, sb, gi, lane, cl, mine[cl]);
      const size_t i = sidx<R>(g.V, cc, se);
      const Cx<R> psi = ein[cl];
      Cx<R> a = diag * psi - R(0.5) * hs;
      if (cc >= 6) a = mk<R>(-a.re, -a.im);
      C64 wv = svj * widen(a);
      if (j > 0) wv = wv - bs * widen(eprev[cl]);
      const Cx<R> wr = narrow<R>(wv);
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
    if (acc) {
      const size_t iy = sidx_to64<R>(n / 12, i);
      lift.y[iy] = lift.y[iy] + cmul(lcn, vd);
    }
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
// Directions split over the waves of the workgroup (hop_group); two lanes per
// site, the even lane on A v_j, the odd lane on A^dag w_j (both read the same
// link in the same instruction); 32 sites per wave.  The previous partial
// sums are loaded before the stencil and reduced after it.
template <class R, class LK, int NG>
__global__ void __launch_bounds__(NT) k_bil1(Geom g, LK lk, R diag, R eft, R ebt, int j,
                                             const Cx<R>* __restrict__ vj, const Cx<R>* __restrict__ wj,
                                             const Cx<R>* __restrict__ vjm1, const Cx<R>* __restrict__ wjm1,
                                             Cx<R>* __restrict__ p, Cx<R>* __restrict__ q,
                                             const double* __restrict__ partIn, int nbIn,
                                             double* __restrict__ partOut, Coefs c) {
  constexpr int M = 12 / NG;
  constexpr int NSB = (NT / 64) / NG;  // site blocks of 32 per workgroup
  __shared__ XBuf<R, NG> xb;
  const int flag = c.flags[0];
  double pr[4];  // this thread's pair of the previous partial sums (nbIn <= 2 NT, even)
#pragma unroll
  for (int qd = 0; qd < 4; ++qd) pr[qd] = pair_sum(partIn + qd * nbIn, 2 * threadIdx.x, nbIn);
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gi = w % NG, sb = w / NG;
  const int f = lane & 1;  // 0: A v_j, 1: A^dag w_j
  const Cx<R>* in = f ? wj : vj;
  const int s = (xcd_block() * NSB + sb) * 32 + (lane >> 1);
  const bool live = s < g.V;
  Cx<R> mine[M];
  hop_group<NG>(g, live ? s : 0, lk, in, gi, f ? ebt : eft, f ? eft : ebt, xb, w, lane, mine);  // dead lanes hop at site 0
  if (flag) return;
  __builtin_amdgcn_sched_barrier(0);  // the stencil's registers are free before these loads
  // this site's input entries go out before the block reduction, whose
  // barriers they then overlap (the previous vector's as well would take
  // two registers more than four waves per SIMD allow)
  int se = s;
  asm volatile("" : "+v"(se));  // keeps the epilogue addresses out of the stencil's registers
  Cx<R> ein[M];
#pragma unroll
  for (int cl = 0; cl < M; ++cl) {
    const size_t i = sidx<R>(g.V, gi * M + cl, live ? se : 0);
    ein[cl] = in[i];
  }
  double red[4];
#pragma unroll
  for (int qd = 0; qd < 4; ++qd) red[qd] = pr[qd];
  block_sum<4>(red);  // also completes the exchange
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
  const C64 scale = f ? swj : mk(svj, 0.0);
  const C64 sub = f ? delta * swjm1 : svjm1 * beta;  // delta_{j-1} sw_{j-1} or beta_{j-1} sv_{j-1}
  const Cx<R>* prev = f ? wjm1 : vjm1;
  Cx<R>* out = f ? q : p;
  double dre = 0.0, dim = 0.0;
  if (live) {
#pragma unroll
    for (int cl = 0; cl < M; ++cl) {
      const int cc = gi * M + cl;
      const Cx<R> hs = xsum<NG>(xb, sb, gi, lane, cl, mine[cl]);
      const size_t i = sidx<R>(g.V, cc, se);
      const Cx<R> ini = ein[cl];
      const Cx<R> wpair = pair_swap(ini);  // the odd lane's w_j at this site
      Cx<R> a = diag * ini - R(0.5) * hs;
      if (cc >= 6) a = mk<R>(-a.re, -a.im);
      const C64 ad = widen(a);
      C64 o = cmul(scale, ad);
      if (j > 0) o = o - cmul(sub, widen(prev[i]));
      out[i] = narrow<R>(o);
      if (f == 0) {
        const C64 t = cmulc(widen(wpair), ad);
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
  // four elements per thread and batch: all loads of a batch are issued
  // before its first store, which keeps enough bytes in flight to stream at
  // full rate; the first batch is issued before the partial sums of K1 are
  // reduced, so the reduction's latency overlaps the stream
  constexpr int U = 4;
  const int stride = gridDim.x * NT;
  int i0 = blockIdx.x * NT + threadIdx.x;
  Cx<R> pp[U], qq[U], vv[U], ww[U];
  auto load = [&](int ib) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = ib + u * stride;
      if (i < n) {
        pp[u] = p[i];
        qq[u] = q[i];
        vv[u] = vj[i];
        ww[u] = wj[i];
      }
    }
  };
  const int flag = c.flags[0];
  load(i0);
  if (flag) return;
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
  for (; i0 < n; i0 += U * stride) {
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
        if (acc) {
          const size_t iy = sidx_to64<R>(n / 12, i);
          lift.y[iy] = lift.y[iy] + cmul(lcn, vd);
        }
      }
    }
    if (i0 + U * stride < n) load(i0 + U * stride);
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
// Second pass of the two-sided recurrence with A alone: every coefficient is
// known from the first pass, so one kernel per step regenerates the right
// basis vector from the two before it and adds its lift term,
//   p = sv_j (A vt_j) - (sv_{j-1} beta_{j-1}) vt_{j-1},
//   vt_{j+1} = p - (sv_j alpha_j) vt_j,   y += lc_{j+1} vt_{j+1},
// with the operations, operand order and roundings of the v-lane of k_bil1
// followed by k_bil2, so every column is bit-identical to the first pass's
// (the hopping sum is the same direction-group sum of the same hops).  No
// A^dag w, no W ring, no reduction: the left vectors only fed coefficients
// that are now stored.  One lane per site, like k_lan1.
template <class R, class LK, int NG>
__global__ void __launch_bounds__(NT) k_regen(Geom g, LK lk, R diag, R eft, R ebt, int j,
                                              const Cx<R>* __restrict__ vj, const Cx<R>* __restrict__ vjm1,
                                              Cx<R>* __restrict__ vnext, Coefs c, LiftAcc lift) {
  constexpr int M = 12 / NG;
  constexpr int NSB = (NT / 64) / NG;  // site blocks of 64 per workgroup
  __shared__ XBuf<R, NG> xb;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gi = w % NG, sb = w / NG;
  const int s = (xcd_block() * NSB + sb) * 64 + lane;
  const bool live = s < g.V;
  Cx<R> mine[M];
  hop_group<NG>(g, live ? s : 0, lk, vj, gi, eft, ebt, xb, w, lane, mine);  // a lane past the end hops at site 0
  Cx<R> ein[M], eprev[M];
  {
    int se = live ? s : 0;
    asm volatile("" : "+v"(se));  // keeps these addresses out of the stencil's registers
#pragma unroll
    for (int cl = 0; cl < M; ++cl) {
      const size_t i = sidx<R>(g.V, gi * M + cl, se);
      ein[cl] = vj[i];
      eprev[cl] = j > 0 ? vjm1[i] : mk<R>(0, 0);
    }
  }
  const double svj = c.sv[j];
  const C64 scale = mk(svj, 0.0);
  const C64 sub = j > 0 ? c.sv[j - 1] * c.beta[j - 1] : mk(0.0, 0.0);
  const C64 av = svj * c.alpha[j];
  const bool acc = j + 1 < lift.kused;
  const C64 lcn = acc ? lift.lc[j + 1] : mk(0.0, 0.0);
  __syncthreads();  // completes the exchange
  if (!live) return;
  int se = s;
  asm volatile("" : "+v"(se));  // keeps the epilogue addresses out of the stencil's registers
#pragma unroll
  for (int cl = 0; cl < M; ++cl) {
    const int cc = gi * M + cl;
    const Cx<R> hs = xsum<NG>(xb, sb, gi, lane, cl, mine[cl]);
    const size_t i = sidx<R>(g.V, cc, se);
    const Cx<R> ini = ein[cl];
    Cx<R> a = diag * ini - R(0.5) * hs;
    if (cc >= 6) a = mk<R>(-a.re, -a.im);
    C64 o = cmul(scale, widen(a));
    if (j > 0) o = o - cmul(sub, widen(eprev[cl]));
    const Cx<R> p = narrow<R>(o);
    const Cx<R> vr = narrow<R>(widen(p) - cmul(av, widen(ini)));
    vnext[i] = vr;
    if (acc) {
      const size_t iy = sidx_to64<R>(g.V, i);
      lift.y[iy] = lift.y[iy] + cmul(lcn, widen(vr));
    }
  }
}

// ---------------------------------------------------------------------------
// lift: y = sum_j lc[j] vt_j over the stored columns (FP64 accumulation)
template <class R>
__global__ void __launch_bounds__(NT) k_lift(int n, int kused, const Cx<R>* __restrict__ vk, size_t colstride,
                                             const C64* __restrict__ lc, C64* __restrict__ y) {
  const int i = blockIdx.x * NT + threadIdx.x;  // y in the FP64 layout, the columns in that of R
  if (i >= n) return;
  const size_t ir = sidx_of64<R>(n / 12, i);
  C64 a0 = mk(0.0, 0.0), a1 = a0, a2 = a0, a3 = a0;
  int j = 0;
  for (; j + 4 <= kused; j += 4) {
    const Cx<R> v0 = vk[(size_t)(j + 0) * colstride + ir];
    const Cx<R> v1 = vk[(size_t)(j + 1) * colstride + ir];
    const Cx<R> v2 = vk[(size_t)(j + 2) * colstride + ir];
    const Cx<R> v3 = vk[(size_t)(j + 3) * colstride + ir];
    a0 = a0 + cmul(lc[j + 0], widen(v0));
    a1 = a1 + cmul(lc[j + 1], widen(v1));
    a2 = a2 + cmul(lc[j + 2], widen(v2));
    a3 = a3 + cmul(lc[j + 3], widen(v3));
  }
  for (; j < kused; ++j) a0 = a0 + cmul(lc[j], widen(vk[(size_t)j * colstride + ir]));
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

// workgroups of the element-wise kernels; K1 prefetches at most 2 NT
// partial sums per quantity, so this stays <= 2 NT
static int nb_elem(const Geom& g) {
  const int n = 12 * g.V;
  int nb = (n + NT - 1) / NT;
  nb += nb & 1;  // even (pairs of partial sums are read as one load)
  return nb < 2 * NT ? nb : 2 * NT;
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
  // K1 writes one partial per workgroup: at most one per 32 sites (k_bil1
  // with four direction groups)
  const int nb1 = (g.V + 31) / 32 + 1, nb2 = nb_elem(g);
  const int nbmax = nb1 > nb2 ? nb1 : nb2;
  if (lat->part.ensure((size_t)2 * 4 * nbmax * sizeof(double))) return NK_ENOMEM;
  b.partA = lat->part.as<double>();
  b.partB = b.partA + 4 * nbmax;
  return NK_OK;
}

int prof_event(nk_lattice* lat, hipEvent_t* ev) {
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

// K1 workgroups for NG direction groups: NT / 64 / NG blocks of 64 sites
// (Lanczos, one lane per site) or of 32 sites (two-sided, two lanes per site)
static int k1_blocks(const Geom& g, int hermitian, int ng) {
  const int spb = (hermitian ? 64 : 32) * ((NT / 64) / ng);
  const int nb = (g.V + spb - 1) / spb;
  return nb + (nb & 1);  // even (pairs of partial sums are read as one load)
}

// one K1 launch with NG = ng direction groups
template <class R, class LK>
static void launch_k1(int ng, const Geom& g, const BasisPlan& bp, const LK& lk, R diag, int j, const Cx<R>* vj,
                      const Cx<R>* wj, const Cx<R>* vjm1, const Cx<R>* wjm1, Cx<R>* p, Cx<R>* q,
                      const double* partIn, int nbIn, double* partOut, Coefs c, hipEvent_t e0, hipEvent_t e1,
                      hipStream_t st) {
  const int nb1 = k1_blocks(g, bp.hermitian, ng);
  const R eft = (R)exp(bp.mu), ebt = (R)exp(-bp.mu);
  if (bp.hermitian) {
    if (ng == 2)
      hipExtLaunchKernelGGL((k_lan1<R, LK, 2>), dim3(nb1), dim3(NT), 0, st, e0, e1, 0, g, lk, diag, j, vj, vjm1, p,
                            partIn, nbIn, partOut, c);
    else
      hipExtLaunchKernelGGL((k_lan1<R, LK, 4>), dim3(nb1), dim3(NT), 0, st, e0, e1, 0, g, lk, diag, j, vj, vjm1, p,
                            partIn, nbIn, partOut, c);
  } else {
    if (ng == 2)
      hipExtLaunchKernelGGL((k_bil1<R, LK, 2>), dim3(nb1), dim3(NT), 0, st, e0, e1, 0, g, lk, diag, eft, ebt, j, vj,
                            wj, vjm1, wjm1, p, q, partIn, nbIn, partOut, c);
    else
      hipExtLaunchKernelGGL((k_bil1<R, LK, 4>), dim3(nb1), dim3(NT), 0, st, e0, e1, 0, g, lk, diag, eft, ebt, j, vj,
                            wj, vjm1, wjm1, p, q, partIn, nbIn, partOut, c);
  }
}

// The autotuner: time K1 with 2 and with 4 direction groups on this lattice,
// precision and recurrence (ten launches of each after two warm-up launches,
// on scratch coefficients and valid partial sums).  Two groups are taken only
// when they are more than 5% faster, so that timing noise between close
// candidates does not change the kernel (and the rounding of the result)
// from one process to the next.  The choice is made once per handle and
// reused by every later run, so a second (two-pass) sweep runs the same
// kernels as the first.
template <class R, class LK>
static int tune_k1(nk_lattice* lat, const BasisPlan& bp, const LK& lk, BasisBuffers& b, hipStream_t st, int* ng_out) {
  const Geom& g = lat->g;
  const int nb2 = nb_elem(g);
  if (lat->tunebuf.ensure(4096)) return NK_ENOMEM;
  char* tb = lat->tunebuf.as<char>();
  Coefs c;
  c.alpha = (C64*)(tb);
  c.beta = (C64*)(tb + 256);
  c.delta = (C64*)(tb + 512);
  c.sv = (double*)(tb + 768);
  c.sw = (C64*)(tb + 1024);
  c.flags = (int*)(tb + 1280);
  std::vector<double> parts((size_t)4 * nb2, 1.0 / nb2);  // s = 1 + i, |v|^2 = |w|^2 = 1: no breakdown
  std::vector<char> zeros(2048, 0);
  NK_HIP(hipMemcpyAsync(tb, zeros.data(), zeros.size(), hipMemcpyHostToDevice, st));
  NK_HIP(hipMemcpyAsync(b.partB, parts.data(), parts.size() * sizeof(double), hipMemcpyHostToDevice, st));
  const R diag = (R)(4.0 + bp.m_w);
  auto colp = [&](int s) { return reinterpret_cast<Cx<R>*>(b.vk + (size_t)s * b.colbytes); };
  Cx<R>* w0 = reinterpret_cast<Cx<R>*>(b.wring);
  Cx<R>* w1 = reinterpret_cast<Cx<R>*>(b.wring + b.colbytes);
  hipEvent_t ev[2];
  NK_HIP(hipEventCreate(&ev[0]));
  NK_HIP(hipEventCreate(&ev[1]));
  float tms[2] = {0.f, 0.f};  // 4 groups, 2 groups
  for (int ng : {4, 2}) {
    for (int rep = 0; rep < 12; ++rep) {
      if (rep == 2) NK_HIP(hipEventRecord(ev[0], st));
      launch_k1<R, LK>(ng, g, bp, lk, diag, 1, colp(1), w1, colp(0), w0, reinterpret_cast<Cx<R>*>(b.p),
                       reinterpret_cast<Cx<R>*>(b.q), b.partB, nb2, b.partA, c, nullptr, nullptr, st);
    }
    NK_HIP(hipGetLastError());
    NK_HIP(hipEventRecord(ev[1], st));
    NK_HIP(hipEventSynchronize(ev[1]));
    NK_HIP(hipEventElapsedTime(&tms[ng == 4 ? 0 : 1], ev[0], ev[1]));
  }
  const int best_ng = tms[1] < 0.95f * tms[0] ? 2 : 4;
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  *ng_out = best_ng;
  return NK_OK;
}

template <class R, class LK>
static int run_steps(nk_lattice* lat, const BasisPlan& bp, const LK& lk, const C64* x, int j0, int j1, Coefs c,
                     BasisBuffers& b, LiftAcc lift, hipStream_t st) {
  const Geom& g = lat->g;
  const int n = 12 * g.V;
  int& ng = lat->k1_groups[bp.hermitian ? 1 : 0][bp.prec];
  if (ng == 0) {  // first run on this handle: before k_start, whose partial sums the tuning overwrites
    if (NK_AUTOTUNE && j0 == 0) {
      if (int e = tune_k1<R, LK>(lat, bp, lk, b, st, &ng)) return e;
    } else {
      ng = NK_GROUPS;
    }
  }
  const int nb1 = k1_blocks(g, bp.hermitian, ng), nb2 = nb_elem(g);
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
      const bool timed = bp.profile > 0 && j % bp.profile == 0;
      if (timed) {
        if (int r = prof_event(lat, &e0)) return r;
        if (int r = prof_event(lat, &e1)) return r;
      }
      if (kind == 0) {
        launch_k1<R, LK>(ng, g, bp, lk, diag, j, col(j), bp.hermitian ? nullptr : wsl(j), j > 0 ? col(j - 1) : col(j),
                         bp.hermitian ? nullptr : (j > 0 ? wsl(j - 1) : wsl(j)), p, q, b.partB, nb2, b.partA, c, e0,
                         e1, st);
      } else if (bp.hermitian) {
        hipExtLaunchKernelGGL((k_lan2<R>), dim3(nb2), dim3(NT), 0, st, e0, e1, 0, n, j, p, col(j), col(j + 1),
                              b.partA, nb1, b.partB, c, lift);
      } else {
        hipExtLaunchKernelGGL((k_bil2<R>), dim3(nb2), dim3(NT), 0, st, e0, e1, 0, n, j, p, q, col(j), wsl(j),
                              col(j + 1), wsl(j + 1), b.partA, nb1, b.partB, c, lift);
      }
      NK_HIP(hipGetLastError());
      if (timed) lat->evkind.push_back(kind);
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

// y = ||x|| sum_j z_j v_j over kused FP64 columns vk + j * colstride (lc: workspace [kused])
int lift_columns(int n, int kused, const C64* vk, size_t colstride, const C64* z, const double* sv, C64* lc, C64* y,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_lift_coef, dim3((kused + 255) / 256), dim3(256), 0, st, kused, z, sv, lc);
  hipLaunchKernelGGL(k_lift<double>, dim3((n + NT - 1) / NT), dim3(NT), 0, st, n, kused, vk, colstride,
                     (const C64*)lc, y);
  NK_HIP(hipGetLastError());
  return NK_OK;
}

// the second pass of the two-sided recurrence: k_regen over a ring of three
// columns, with the direction groups the first pass's stencil kernel used
template <class R, class LK>
static int regen_run(nk_lattice* lat, const BasisPlan& bp, const LK& lk, const C64* x, int kused, Coefs c,
                     LiftAcc lift, hipStream_t st) {
  const Geom& g = lat->g;
  const int n = 12 * g.V;
  BasisBuffers b;
  if (int e = get_buffers(lat, bp, nullptr, b)) return e;
  const int ng = lat->k1_groups[0][bp.prec];
  if (ng != 2 && ng != 4) {
    set_error("second pass before the first: no stencil kernel chosen for this recurrence");
    return NK_EINVAL;
  }
  auto col = [&](int j) { return reinterpret_cast<Cx<R>*>(b.vk + (size_t)(j % 3) * b.colbytes); };
  hipLaunchKernelGGL((k_start<R, 1>), dim3(nb_elem(g)), dim3(NT), 0, st, n, x, col(0), (Cx<R>*)nullptr, b.partB,
                     lift);
  const R diag = (R)(4.0 + bp.m_w);
  const R eft = (R)exp(bp.mu), ebt = (R)exp(-bp.mu);
  const int nbl = k1_blocks(g, 1, ng);  // one lane per site
  for (int j = 0; j + 1 < kused; ++j) {
    if (ng == 2)
      hipLaunchKernelGGL((k_regen<R, LK, 2>), dim3(nbl), dim3(NT), 0, st, g, lk, diag, eft, ebt, j, col(j),
                         j > 0 ? col(j - 1) : col(j), col(j + 1), c, lift);
    else
      hipLaunchKernelGGL((k_regen<R, LK, 4>), dim3(nbl), dim3(NT), 0, st, g, lk, diag, eft, ebt, j, col(j),
                         j > 0 ? col(j - 1) : col(j), col(j + 1), c, lift);
  }
  NK_HIP(hipGetLastError());
  return NK_OK;
}

// second pass: rebuild the basis with a ring of three columns and accumulate
// y += lc[j] vt_j as each column appears, every column bit-identical to the
// one the first pass produced.  Lanczos (mu = 0) runs its own two kernels
// again; two-sided Lanczos regenerates the right vectors with A alone from
// the stored coefficients (k_regen), one kernel per step.
int two_pass_lift(nk_lattice* lat, const BasisPlan& bp0, const C64* x_canon, int kused, const C64* z, Coefs c,
                  C64* y_dev, hipStream_t st) {
  if (lat->lift.ensure((size_t)kused * sizeof(C64))) return NK_ENOMEM;
  C64* lc = lat->lift.as<C64>();
  hipLaunchKernelGGL(k_lift_coef, dim3((kused + 255) / 256), dim3(256), 0, st, kused, z, c.sv, lc);
  NK_HIP(hipGetLastError());
  BasisPlan bp = bp0;
  bp.store = 0;
  const LiftAcc lift{y_dev, lc, kused};
  if (bp.hermitian) return run_any(lat, bp, x_canon, 0, kused - 1, c, nullptr, lift, st);
  const Geom& g = lat->g;
  if (bp.prec == NK_PREC_FP64)
    return regen_run<double>(lat, bp, LinksPlain<double>{lat->U64.as<C64>(), g.V}, x_canon, kused, c, lift, st);
  if (bp.prec == NK_PREC_FP32)
    return regen_run<float>(lat, bp, LinksPlain<float>{lat->U32.as<C32>(), g.V}, x_canon, kused, c, lift, st);
  return regen_run<float>(lat, bp, LinksBF16{lat->Ubf.as<uint32_t>(), g.V}, x_canon, kused, c, lift, st);
}

}  // namespace nk
