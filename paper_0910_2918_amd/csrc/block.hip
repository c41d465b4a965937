// Many sources in lockstep: the outer two-sided Lanczos basis of Sec. 2 for
// r sources at once, the small problems of Eqs. (3)-(6) batched, and the lift.
//
// Each source keeps its own recurrence and coefficients.  A step is four
// launches for all sources together:
//   k_blk1  A v_j, A^dag w_j minus the previous vectors, partial w~^dag A v~
//           (grid: site blocks x sources)
//   k_bred1 alpha_j per source (fixed-order reduction)
//   k_blk2  v_hat, w_hat (new unnormalised columns), partial s, |v|^2, |w|^2
//   k_bred2 delta, beta, the scales and the breakdown test per source
// so launches and reductions are shared by the sources, and the small
// problems run as one inner projection per source followed by one batched
// Roberts-Higham call over the uneven ell of all sources.  The links are
// read once per source: on MI355X they stay in the 256 MB Infinity Cache
// between sources (38 MB at 16^4, 75 MB at 16^3 x 32), so re-reading them
// costs no HBM traffic, while keeping them in registers for all sources
// would cut the occupancy of the stencil kernel in half.  Every reduction
// is deterministic, so a second sweep over the same data (two-pass lift)
// reproduces the first bit for bit.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "stencil.h"

namespace nk {

namespace {

constexpr int BT = 256;

struct BArgs {
  C64* base;      // per-source vectors: slot sl of source s at base + (s * nslots + sl) * n
  size_t n;       // complex entries per vector (12 V)
  int nslots, ncols, store, r, k;
  C64* alpha;     // [r][k]
  C64* beta;      // [r][k]
  C64* delta;     // [r][k]
  double* sv;     // [r][k + 1]
  C64* sw;        // [r][k + 1]
  int* flags;     // [r]: 0 running, > 0 breakdown step, -1 zero source
  double* part1;  // [r][2][nb1]
  double* part2;  // [r][4][nb2]
  int nb1, nb2;
  const C64* lc;  // lift coefficients [r][k] (second sweep), or null
  const int* kused;  // [r] (second sweep)
};

__device__ __forceinline__ C64* slot(const BArgs& a, int s, int sl) { return a.base + ((size_t)s * a.nslots + sl) * a.n; }
__device__ __forceinline__ C64* colv(const BArgs& a, int s, int j) { return slot(a, s, a.store ? j : j % 3); }
__device__ __forceinline__ C64* colw(const BArgs& a, int s, int j) { return slot(a, s, a.ncols + (j & 1)); }
__device__ __forceinline__ C64* vp(const BArgs& a, int s) { return slot(a, s, a.ncols + 2); }
__device__ __forceinline__ C64* vq(const BArgs& a, int s) { return slot(a, s, a.ncols + 3); }
__device__ __forceinline__ C64* vx(const BArgs& a, int s) { return slot(a, s, a.ncols + 4); }
__device__ __forceinline__ C64* vy(const BArgs& a, int s) { return slot(a, s, a.ncols + 5); }

template <int NQ>
__device__ __forceinline__ void bsum(double (&v)[NQ]) {
  __shared__ double sh[NQ][BT / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) sh[q][w] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = (sh[q][0] + sh[q][1]) + (sh[q][2] + sh[q][3]);
}

// v_0 = w_0 = x (column 0), partial sums [|x|^2, 0, |x|^2, |x|^2]; in the
// second sweep also y = lc_0 x
__global__ void __launch_bounds__(BT) k_bstart(BArgs a) {
  const int s = blockIdx.y;
  const C64* x = vx(a, s);
  C64* v0 = colv(a, s, 0);
  C64* w0 = colw(a, s, 0);
  C64* y = vy(a, s);
  const bool lift = a.lc != nullptr;
  const C64 c0 = lift ? a.lc[(size_t)s * a.k] : mk(0.0, 0.0);
  double nrm = 0.0;
  for (size_t i = (size_t)blockIdx.x * BT + threadIdx.x; i < a.n; i += (size_t)gridDim.x * BT) {
    const C64 v = x[i];
    v0[i] = v;
    w0[i] = v;
    nrm += norm2(v);
    if (lift) y[i] = cmul(c0, v);
  }
  double t[1] = {nrm};
  bsum<1>(t);
  if (threadIdx.x == 0) {
    double* p = a.part2 + (size_t)s * 4 * a.nb2;
    p[0 * a.nb2 + blockIdx.x] = t[0];
    p[1 * a.nb2 + blockIdx.x] = 0.0;
    p[2 * a.nb2 + blockIdx.x] = t[0];
    p[3 * a.nb2 + blockIdx.x] = t[0];
  }
}

// fixed-order sum of nb partials (one workgroup per source)
template <int NQ>
__device__ __forceinline__ void reduce_src(const double* __restrict__ p, int nb, double (&v)[NQ]) {
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = 0.0;
  for (int b = threadIdx.x; b < nb; b += BT)
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] += p[(size_t)q * nb + b];
  bsum<NQ>(v);
}

// finish step j - 1 of every source: s -> delta, beta, scales of column j,
// breakdown test (at j = 0: the source norm)
__global__ void __launch_bounds__(BT) k_bred2(BArgs a, int j) {
  const int s = blockIdx.x;
  if (a.flags[s]) return;
  double red[4];
  reduce_src<4>(a.part2 + (size_t)s * 4 * a.nb2, a.nb2, red);
  if (threadIdx.x != 0) return;
  const C64 sdot = mk(red[0], red[1]);
  const double sabs = sqrt(norm2(sdot));
  if (j == 0 && !(sabs > 0.0 && sabs < 1e300)) {
    a.flags[s] = -1;
    return;
  }
  if (j > 0 && !(sabs > 1e-14 * sqrt(red[2] * red[3]))) {
    a.flags[s] = j;
    return;
  }
  const double delta = sqrt(sabs);
  const C64 beta = (1.0 / delta) * sdot;
  a.sv[(size_t)s * (a.k + 1) + j] = 1.0 / delta;
  a.sw[(size_t)s * (a.k + 1) + j] = (1.0 / norm2(beta)) * beta;  // 1 / conj(beta)
  if (j > 0) {
    a.beta[(size_t)s * a.k + j - 1] = beta;
    a.delta[(size_t)s * a.k + j - 1] = mk(delta, 0.0);
  }
}

// alpha_j = conj(sw_j) sv_j (w~_j^dag A v~_j) of every running source
__global__ void __launch_bounds__(BT) k_bred1(BArgs a, int j) {
  const int s = blockIdx.x;
  if (a.flags[s]) return;
  double red[2];
  reduce_src<2>(a.part1 + (size_t)s * 2 * a.nb1, a.nb1, red);
  if (threadIdx.x != 0) return;
  const double svj = a.sv[(size_t)s * (a.k + 1) + j];
  const C64 swj = a.sw[(size_t)s * (a.k + 1) + j];
  a.alpha[(size_t)s * a.k + j] = cmul(conj(swj), svj * mk(red[0], red[1]));
}

// the stencil step of source blockIdx.y: p = A v_j - beta_j v_{j-1},
// q = A^dag w_j - delta_j w_{j-1} (both scaled by the lazy normalisation),
// partial w~_j^dag (A v~_j).  The body of the one-source kernel: directions
// split over the waves (hop_group), two lanes per site.  Workgroups run
// source by source, so each source keeps the one-source kernel's locality;
// the links, read once per source, stay in the Infinity Cache between
// sources.
template <int NG>
__global__ void __launch_bounds__(BT) k_blk1(Geom g, LinksPlain<double> lk, double diag, double eft, double ebt,
                                              int j, BArgs a) {
  constexpr int M = 12 / NG;
  constexpr int NSB = (BT / 64) / NG;
  __shared__ XBuf<double, NG> xb;
  const int src = blockIdx.y;
  if (a.flags[src]) return;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gi = w % NG, sb = w / NG;
  const int f = lane & 1;  // 0: A v_j, 1: A^dag w_j
  const C64* in = f ? colw(a, src, j) : colv(a, src, j);
  const int s = (xcd_block() * NSB + sb) * 32 + (lane >> 1);
  const bool live = s < g.V;
  C64 mine[M];
  hop_group<NG>(g, live ? s : 0, lk, in, gi, f ? ebt : eft, f ? eft : ebt, xb, w, lane, mine);  // dead lanes hop at site 0
  __builtin_amdgcn_sched_barrier(0);  // the stencil's registers are free before these loads
  // this site's input entries go out before the exchange's barrier, which
  // they then overlap
  int se = s;
  asm volatile("" : "+v"(se));  // keeps the epilogue addresses out of the stencil's registers
  C64 ein[M];
#pragma unroll
  for (int cl = 0; cl < M; ++cl) ein[cl] = in[sidx<double>(g.V, gi * M + cl, live ? se : 0)];
  // this source's step coefficients (uniform loads) before the barrier too
  const size_t kk = (size_t)src * (a.k + 1);
  const double svj = a.sv[kk + j];
  const C64 swj = a.sw[kk + j];
  C64 scale = f ? swj : mk(svj, 0.0), sub = mk(0.0, 0.0);
  if (j > 0) {
    const C64 bm = a.beta[(size_t)src * a.k + j - 1], dm = a.delta[(size_t)src * a.k + j - 1];
    sub = f ? cmul(dm, a.sw[kk + j - 1]) : a.sv[kk + j - 1] * bm;
  }
  __syncthreads();
  const C64* prev = f ? colw(a, src, j > 0 ? j - 1 : 0) : colv(a, src, j > 0 ? j - 1 : 0);
  C64* out = f ? vq(a, src) : vp(a, src);
  double dre = 0.0, dim = 0.0;
  if (live) {
#pragma unroll
    for (int cl = 0; cl < M; ++cl) {
      const int cc = gi * M + cl;
      const C64 hs = xsum<NG>(xb, sb, gi, lane, cl, mine[cl]);
      const size_t i = sidx<double>(g.V, cc, se);
      const C64 wpair = pair_swap(ein[cl]);  // the odd lane's w_j at this site
      C64 av = diag * ein[cl] - 0.5 * hs;
      if (cc >= 6) av = mk(-av.re, -av.im);
      C64 o = cmul(scale, av);
      if (j > 0) o = o - cmul(sub, prev[i]);
      out[i] = o;
      if (f == 0) {
        const C64 t = cmulc(wpair, av);
        dre += t.re;
        dim += t.im;
      }
    }
  }
  double v[2] = {dre, dim};
  bsum<2>(v);
  if (threadIdx.x == 0) {
    double* p1 = a.part1 + (size_t)src * 2 * a.nb1;
    p1[blockIdx.x] = v[0];
    p1[a.nb1 + blockIdx.x] = v[1];
  }
}

// The same stencil step for S sources per workgroup that share each link
// load: 2 S lanes per site (lane l: side l & 1, source (l >> 1) % S of the
// workgroup's group blockIdx.y), 32 / S sites per wave.  The lanes of a site
// ask for the same link entry in the same load instruction, which the
// memory pipeline serves once, so the links are fetched once per site for
// all S sources; each lane's arithmetic is that of the one-source kernel.
// Partial sums per source of the group.  Lanes of a source past the last or
// of a broken-down source hop like the others (on valid vectors) and write
// nothing.
template <int NG, int S>
__global__ void __launch_bounds__(BT) k_blkS(Geom g, LinksPlain<double> lk, double diag, double eft, double ebt,
                                              int j, BArgs a) {
  constexpr int M = 12 / NG;
  constexpr int NSB = (BT / 64) / NG;
  constexpr int SPW = 32 / S;  // sites per wave
  __shared__ XBuf<double, NG> xb;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gi = w % NG, sb = w / NG;
  const int f = lane & 1;  // 0: A v_j, 1: A^dag w_j
  const int sl = (lane >> 1) % S;
  const int src0 = blockIdx.y * S + sl;
  const bool have = src0 < a.r;
  const int src = have ? src0 : a.r - 1;
  const bool run = have && a.flags[src] == 0;
  const C64* in = f ? colw(a, src, j) : colv(a, src, j);
  const int s = (xcd_block() * NSB + sb) * SPW + (lane >> 1) / S;
  const bool live = s < g.V;
  C64 mine[M];
  hop_group<NG>(g, live ? s : 0, lk, in, gi, f ? ebt : eft, f ? eft : ebt, xb, w, lane, mine);  // dead lanes hop at site 0
  __syncthreads();
  const size_t kk = (size_t)src * (a.k + 1);
  const double svj = a.sv[kk + j];
  const C64 swj = a.sw[kk + j];
  C64 scale = f ? swj : mk(svj, 0.0), sub = mk(0.0, 0.0);
  if (j > 0) {
    const C64 bm = a.beta[(size_t)src * a.k + j - 1], dm = a.delta[(size_t)src * a.k + j - 1];
    sub = f ? cmul(dm, a.sw[kk + j - 1]) : a.sv[kk + j - 1] * bm;
  }
  const C64* prev = f ? colw(a, src, j > 0 ? j - 1 : 0) : colv(a, src, j > 0 ? j - 1 : 0);
  C64* out = f ? vq(a, src) : vp(a, src);
  const C64* wj = colw(a, src, j);
  double dre = 0.0, dim = 0.0;
  if (live && run) {
    int se = s;
    asm volatile("" : "+v"(se));  // keeps the epilogue addresses out of the stencil's registers
#pragma unroll
    for (int cl = 0; cl < M; ++cl) {
      const int cc = gi * M + cl;
      const C64 hs = xsum<NG>(xb, sb, gi, lane, cl, mine[cl]);
      const size_t i = sidx<double>(g.V, cc, se);
      C64 av = diag * in[i] - 0.5 * hs;
      if (cc >= 6) av = mk(-av.re, -av.im);
      C64 o = cmul(scale, av);
      if (j > 0) o = o - cmul(sub, prev[i]);
      out[i] = o;
      if (f == 0) {
        const C64 t = cmulc(wj[i], av);
        dre += t.re;
        dim += t.im;
      }
    }
  }
  double v[2 * S];
#pragma unroll
  for (int t = 0; t < S; ++t) {
    v[2 * t] = sl == t ? dre : 0.0;
    v[2 * t + 1] = sl == t ? dim : 0.0;
  }
  bsum<2 * S>(v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int t = 0; t < S; ++t) {
      const int st = blockIdx.y * S + t;
      if (st < a.r) {
        double* p1 = a.part1 + (size_t)st * 2 * a.nb1;
        p1[blockIdx.x] = v[2 * t];
        p1[a.nb1 + blockIdx.x] = v[2 * t + 1];
      }
    }
}

// v_hat = p - alpha_j v_j, w_hat = q - conj(alpha_j) w_j into column j + 1,
// partial sums of s = w_hat^dag v_hat, |v_hat|^2, |w_hat|^2; second sweep:
// y += lc_{j+1} v_hat
__global__ void __launch_bounds__(BT) k_blk2(BArgs a, int j) {
  const int s = blockIdx.y;
  if (a.flags[s]) return;
  const double svj = a.sv[(size_t)s * (a.k + 1) + j];
  const C64 swj = a.sw[(size_t)s * (a.k + 1) + j];
  const C64 alpha = a.alpha[(size_t)s * a.k + j];
  const C64 av = svj * alpha;
  const C64 aw = cmul(conj(alpha), swj);
  const C64* p = vp(a, s);
  const C64* q = vq(a, s);
  const C64* v = colv(a, s, j);
  const C64* w = colw(a, s, j);
  C64* vn = colv(a, s, j + 1);
  C64* wn = colw(a, s, j + 1);
  C64* y = vy(a, s);
  const bool lift = a.lc != nullptr && j + 1 < a.kused[s];
  const C64 lcn = lift ? a.lc[(size_t)s * a.k + j + 1] : mk(0.0, 0.0);
  double sre = 0.0, sim = 0.0, nv = 0.0, nw = 0.0;
  // four elements per thread and batch, all loads before the first store
  constexpr int U = 4;
  const size_t stride = (size_t)gridDim.x * BT;
  for (size_t i0 = (size_t)blockIdx.x * BT + threadIdx.x; i0 < a.n; i0 += U * stride) {
    C64 pp[U], qq[U], vv[U], ww[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = i0 + u * stride;
      if (i < a.n) {
        pp[u] = p[i];
        qq[u] = q[i];
        vv[u] = v[i];
        ww[u] = w[i];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = i0 + u * stride;
      if (i < a.n) {
        const C64 vr = pp[u] - cmul(av, vv[u]);
        const C64 wr = qq[u] - cmul(aw, ww[u]);
        vn[i] = vr;
        wn[i] = wr;
        const C64 t = cmulc(wr, vr);
        sre += t.re;
        sim += t.im;
        nv += norm2(vr);
        nw += norm2(wr);
        if (lift) y[i] = y[i] + cmul(lcn, vr);
      }
    }
  }
  double t4[4] = {sre, sim, nv, nw};
  bsum<4>(t4);
  if (threadIdx.x == 0) {
    double* p2 = a.part2 + (size_t)s * 4 * a.nb2;
    p2[0 * a.nb2 + blockIdx.x] = t4[0];
    p2[1 * a.nb2 + blockIdx.x] = t4[1];
    p2[2 * a.nb2 + blockIdx.x] = t4[2];
    p2[3 * a.nb2 + blockIdx.x] = t4[3];
  }
}

// dense tridiagonal H (n x n, leading dimension ld) of each source
__global__ void k_tri_dense_b(int ld, const int* __restrict__ nvec, const C64* __restrict__ abd, C64* __restrict__ H) {
  const int s = blockIdx.y;
  const int n = nvec[s];
  const C64* al = abd + (size_t)s * 3 * ld;
  const C64* be = al + ld;
  const C64* de = be + ld;
  C64* Hs = H + (size_t)s * ld * ld;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ld * ld; e += gridDim.x * blockDim.x) {
    const int i = e / ld, c = e % ld;
    C64 v = mk(0.0, 0.0);
    if (i < n && c < n) {
      if (i == c) v = al[i];
      else if (c == i + 1) v = be[i];
      else if (i == c + 1) v = de[c];
    }
    Hs[e] = v;
  }
}

// z = column 0 of S (non-nested) or V_ell times it (nested), per source
__global__ void k_bz(int kmax, int ld, const int* __restrict__ kvec, const int* __restrict__ lvec, int nested,
                     const C64* __restrict__ Vl, const C64* __restrict__ S, C64* __restrict__ z) {
  const int s = blockIdx.y;
  const int k = kvec[s], l = lvec[s];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= k) return;
  const C64* Ss = S + (size_t)s * ld * ld;
  C64 acc = mk(0.0, 0.0);
  if (nested) {
    const C64* V = Vl + (size_t)s * kmax * ld;
    for (int c = 0; c < l; ++c) acc = acc + cmul(V[(size_t)c * k + r], Ss[(size_t)c * ld]);
  } else {
    acc = Ss[(size_t)r * ld];
  }
  z[(size_t)s * kmax + r] = acc;
}

// lc_j = ||x|| z_j sv_j per source (||x|| = 1 / sv_0)
__global__ void k_blc(int k, const int* __restrict__ kvec, const C64* __restrict__ z, const double* __restrict__ sv,
                      C64* __restrict__ lc) {
  const int s = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  const double* svs = sv + (size_t)s * (k + 1);
  lc[(size_t)s * k + j] = j < kvec[s] ? (svs[j] / svs[0]) * z[(size_t)s * k + j] : mk(0.0, 0.0);
}

int nb_elem_b(size_t n) {
  const size_t nb = (n + BT - 1) / BT;
  return (int)std::min<size_t>(nb, 512);
}

// one sweep of the basis for every source: steps 0 .. kmax - 1; with
// profile = n > 0 the stencil and update launches of every n-th step carry
// HIP events (collected by prof_collect)
// one stencil step for every source: ng direction groups, grp sources per
// workgroup (1: k_blk1; 2, 4: k_blkS); a.nb1 must be blk_nb1(g, ng, grp)
void launch_blk1(const Geom& g, const LinksPlain<double>& lk, int ng, int grp, double m_w, double eft, double ebt,
                 int j, const BArgs& a, hipEvent_t e0, hipEvent_t e1, hipStream_t st) {
  const dim3 gr1(a.nb1, a.r), grS(a.nb1, (a.r + grp - 1) / grp);
#define NK_BLK(NG_, S_)                                                                                        \
  if (ng == NG_ && grp == S_) {                                                                                \
    if (S_ == 1)                                                                                               \
      hipExtLaunchKernelGGL(k_blk1<NG_>, gr1, dim3(BT), 0, st, e0, e1, 0, g, lk, 4.0 + m_w, eft, ebt, j, a);  \
    else                                                                                                       \
      hipExtLaunchKernelGGL((k_blkS<NG_, S_>), grS, dim3(BT), 0, st, e0, e1, 0, g, lk, 4.0 + m_w, eft, ebt, j, \
                            a);                                                                                \
    return;                                                                                                    \
  }
  NK_BLK(2, 1) NK_BLK(2, 2) NK_BLK(2, 4) NK_BLK(4, 1) NK_BLK(4, 2) NK_BLK(4, 4)
#undef NK_BLK
}

int sweep(nk_lattice* lat, const BArgs& a, int ng, int grp, double m_w, double mu, int kmax, int profile,
          hipStream_t st) {
  const Geom& g = lat->g;
  const LinksPlain<double> lk{lat->U64.as<C64>(), g.V};
  hipLaunchKernelGGL(k_bstart, dim3(a.nb2, a.r), dim3(BT), 0, st, a);
  hipLaunchKernelGGL(k_bred2, dim3(a.r), dim3(BT), 0, st, a, 0);
  const double eft = exp(mu), ebt = exp(-mu);
  for (int j = 0; j < kmax; ++j) {
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    const bool timed = profile > 0 && j % profile == 0;
    if (timed)
      for (auto& e : ev)
        if (int r = prof_event(lat, &e)) return r;
    launch_blk1(g, lk, ng, grp, m_w, eft, ebt, j, a, ev[0], ev[1], st);
    hipLaunchKernelGGL(k_bred1, dim3(a.r), dim3(BT), 0, st, a, j);
    hipExtLaunchKernelGGL(k_blk2, dim3(a.nb2, a.r), dim3(BT), 0, st, ev[2], ev[3], 0, a, j);
    if (timed) {
      lat->evkind.push_back(0);
      lat->evkind.push_back(1);
    }
    if (j + 1 < kmax) hipLaunchKernelGGL(k_bred2, dim3(a.r), dim3(BT), 0, st, a, j + 1);
  }
  NK_HIP(hipGetLastError());
  return NK_OK;
}

// the same sweep replayed from a HIP graph captured on first use (on a
// private stream) and cached on the handle under its launch arguments; the
// sweep has kernel launches only, so every replay is the same work as the
// direct launches, bit for bit
int sweep_graph(nk_lattice* lat, const BArgs& a, int ng, int grp, double m_w, double mu, int kmax, hipStream_t st) {
  // the key: every launch argument, field by field (no padding bytes)
  std::vector<char> kb;
  auto put = [&](const auto& v) {
    const char* c = reinterpret_cast<const char*>(&v);
    kb.insert(kb.end(), c, c + sizeof v);
  };
  put(a.base), put(a.n), put(a.nslots), put(a.ncols), put(a.store), put(a.r), put(a.k);
  put(a.alpha), put(a.beta), put(a.delta), put(a.sv), put(a.sw), put(a.flags), put(a.part1), put(a.part2);
  put(a.nb1), put(a.nb2), put(a.lc), put(a.kused), put(ng), put(grp), put(kmax), put(m_w), put(mu);
  put(lat->U64.p), put(lat->g.V);
  hipGraphExec_t exec = nullptr;
  for (auto& gr : lat->graphs)
    if (gr.key == kb) exec = gr.exec;
  if (!exec) {
    if (!lat->cap_stream) NK_HIP(hipStreamCreateWithFlags(&lat->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    NK_HIP(hipStreamBeginCapture(lat->cap_stream, hipStreamCaptureModeRelaxed));
    const int e = sweep(lat, a, ng, grp, m_w, mu, kmax, 0, lat->cap_stream);
    const hipError_t ec = hipStreamEndCapture(lat->cap_stream, &graph);
    if (e) {
      if (graph) (void)hipGraphDestroy(graph);
      return e;
    }
    NK_HIP(ec);
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    NK_HIP(ei);
    if (lat->graphs.size() >= 4) {  // keep the four most recent
      (void)hipGraphExecDestroy(lat->graphs.front().exec);
      lat->graphs.erase(lat->graphs.begin());
    }
    lat->graphs.push_back({kb, exec});
  }
  NK_HIP(hipGraphLaunch(exec, st));
  return NK_OK;
}

}  // namespace

// sources [0, r) of x_canon / y_canon with inner sizes ell[], V_k stored
// (store = 1) or rebuilt in a second sweep
static int block_range(nk_lattice* lat, const nk_sign_params* p, const int* ell, int r, int store,
                       const C64* x_canon, C64* y_canon, nk_sign_info* info, hipStream_t st) {
  const Geom& g = lat->g;
  const int k = p->k;
  const size_t n = (size_t)12 * g.V;
  const size_t colbytes = n * sizeof(C64);
  BArgs a{};
  a.n = n;
  a.ncols = store ? k + 1 : 3;
  a.nslots = a.ncols + 6;
  a.store = store;
  a.r = r;
  a.k = k;
  // direction groups of the stencil kernel: the autotuner's choice for the
  // one-source FP64 two-sided kernel when it has run on this handle
  const int tuned = lat->k1_groups[0][NK_PREC_FP64];
  const int ng = tuned ? tuned : NK_GROUPS;
  // workgroups of the stencil step with grp sources per workgroup; the
  // partial sums are sized for the most (grp = 4)
  auto nb1_of = [&](int grp) {
    const int spb = (32 / grp) * (4 / ng);
    return (g.V + spb - 1) / spb;
  };
  a.nb1 = nb1_of(4);
  a.nb2 = nb_elem_b(n);
  if (lat->bvec.ensure((size_t)r * a.nslots * colbytes)) return NK_ENOMEM;
  a.base = lat->bvec.as<C64>();
  // coefficients, partials, small-problem space
  int lmax = 1;
  for (int s = 0; s < r; ++s) lmax = std::max(lmax, ell[s]);
  const int ldS = std::max(lmax, 1);
  const int ldK = k;  // non-nested small problems are k x k
  const int nested = lmax > 0 && ell[0] > 0 ? 1 : 0;
  for (int s = 0; s < r; ++s)
    if ((ell[s] > 0) != (nested == 1)) {
      set_error("ell_per_rhs mixes nested (ell > 0) and non-nested (ell = 0) sources");
      return NK_EINVAL;
    }
  const int ld = nested ? ldS : ldK;
  size_t bytes = 0;
  auto take = [&](size_t b) {
    size_t o = bytes;
    bytes += (b + 255) & ~(size_t)255;
    return o;
  };
  const size_t oA = take((size_t)r * k * sizeof(C64)), oB = take((size_t)r * k * sizeof(C64)),
               oD = take((size_t)r * k * sizeof(C64)), oSv = take((size_t)r * (k + 1) * sizeof(double)),
               oSw = take((size_t)r * (k + 1) * sizeof(C64)), oF = take((size_t)r * sizeof(int)),
               oP1 = take((size_t)r * 2 * a.nb1 * sizeof(double)), oP2 = take((size_t)r * 4 * a.nb2 * sizeof(double)),
               oZ = take((size_t)r * k * sizeof(C64)), oLc = take((size_t)r * k * sizeof(C64)),
               oKv = take((size_t)r * sizeof(int)), oLv = take((size_t)r * sizeof(int)),
               oAbd = take((size_t)r * 3 * ld * sizeof(C64)), oS = take((size_t)r * ld * ld * sizeof(C64)),
               oVl = take(nested ? (size_t)r * k * ld * sizeof(C64) : 0);
  if (lat->bsmall.ensure(bytes)) return NK_ENOMEM;
  char* base = lat->bsmall.as<char>();
  a.alpha = (C64*)(base + oA);
  a.beta = (C64*)(base + oB);
  a.delta = (C64*)(base + oD);
  a.sv = (double*)(base + oSv);
  a.sw = (C64*)(base + oSw);
  a.flags = (int*)(base + oF);
  a.part1 = (double*)(base + oP1);
  a.part2 = (double*)(base + oP2);
  C64* z = (C64*)(base + oZ);
  C64* lc = (C64*)(base + oLc);
  int* kv = (int*)(base + oKv);
  int* lv = (int*)(base + oLv);
  C64* abd = (C64*)(base + oAbd);
  C64* S = (C64*)(base + oS);
  C64* Vl = (C64*)(base + oVl);
  a.lc = nullptr;
  a.kused = kv;

  hipEvent_t ev[4];
  for (auto& e : ev) NK_HIP(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 4; ++i) (void)hipEventDestroy(e[i]);
    }
  } guard{ev};
  NK_HIP(hipEventRecord(ev[0], st));
  for (int s = 0; s < r; ++s) {
    C64* xs = a.base + ((size_t)s * a.nslots + a.ncols + 4) * n;
    if (int e = pack_spinor<double>(g, x_canon + (size_t)s * n, xs, st)) return e;
  }
  NK_HIP(hipMemsetAsync(a.flags, 0, r * sizeof(int), st));
  NK_HIP(hipMemsetAsync(a.beta, 0, (size_t)r * k * sizeof(C64), st));
  NK_HIP(hipMemsetAsync(a.delta, 0, (size_t)r * k * sizeof(C64), st));
  // sources per workgroup of the stencil step: chosen once per handle by
  // timing the step with 1, 2 and 4 (five launches each at step 0, after the
  // start kernels; the real sweep repeats them); a larger group is taken only
  // when it is more than 5% faster, so that timing noise does not change the
  // kernel, and so the grouping of the partial sums, from one process to the
  // next
  int& grp = lat->blk_group[ng == 2 ? 0 : 1];
  if (grp == 0) {
    const LinksPlain<double> lk{lat->U64.as<C64>(), g.V};
    hipLaunchKernelGGL(k_bstart, dim3(a.nb2, a.r), dim3(BT), 0, st, a);
    hipLaunchKernelGGL(k_bred2, dim3(a.r), dim3(BT), 0, st, a, 0);
    hipEvent_t t0, t1;
    NK_HIP(hipEventCreate(&t0));
    NK_HIP(hipEventCreate(&t1));
    float best = INFINITY;
    int pick = 1;
    for (int gsz : {1, 2, 4}) {
      BArgs at = a;
      at.nb1 = nb1_of(gsz);
      launch_blk1(g, lk, ng, gsz, p->m_w, exp(p->mu), exp(-p->mu), 0, at, nullptr, nullptr, st);
      NK_HIP(hipEventRecord(t0, st));
      for (int rep = 0; rep < 5; ++rep)
        launch_blk1(g, lk, ng, gsz, p->m_w, exp(p->mu), exp(-p->mu), 0, at, nullptr, nullptr, st);
      NK_HIP(hipEventRecord(t1, st));
      NK_HIP(hipEventSynchronize(t1));
      float ms = 0.f;
      NK_HIP(hipEventElapsedTime(&ms, t0, t1));
      if (ms < 0.95f * best) {
        best = ms;
        pick = gsz;
      }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    NK_HIP(hipGetLastError());
    grp = pick;
  }
  a.nb1 = nb1_of(grp);
  // (graph replays carry no events: profiling times the direct launches)
  lat->evkind.clear();
  lat->evnext = 0;
  auto run_sweep = [&](const BArgs& args, int kmax) {
    return p->block == 2 ? sweep_graph(lat, args, ng, grp, p->m_w, p->mu, kmax, st)
                         : sweep(lat, args, ng, grp, p->m_w, p->mu, kmax, p->profile, st);
  };
  if (int e = run_sweep(a, k)) return e;
  NK_HIP(hipEventRecord(ev[1], st));

  // steps each source completed
  std::vector<int> fl(r), kus(r), lus(r);
  NK_HIP(hipMemcpyAsync(fl.data(), a.flags, r * sizeof(int), hipMemcpyDeviceToHost, st));
  NK_HIP(hipStreamSynchronize(st));
  int warn = NK_OK, brk = 0;
  for (int s = 0; s < r; ++s) {
    if (fl[s] < 0) {
      set_error("source %d has zero or non-finite norm", s);
      return NK_EINVAL;
    }
    kus[s] = fl[s] > 0 ? fl[s] : k;
    if (fl[s] > 0) {
      warn = NK_WARN_BREAKDOWN;
      brk = fl[s];
    }
  }
  // small problems: one inner projection per source, one batched Roberts-Higham
  std::vector<C64> hab((size_t)r * 3 * ld, mk(0.0, 0.0));
  if (nested) {
    std::vector<const C64*> pa(r), pb(r), pd(r);
    std::vector<int> ls(r);
    for (int s = 0; s < r; ++s) {
      pa[s] = a.alpha + (size_t)s * k;
      pb[s] = a.beta + (size_t)s * k;
      pd[s] = a.delta + (size_t)s * k;
      ls[s] = std::min(ell[s], kus[s]);
    }
    const int e = small_inner_batch(r, kus.data(), ls.data(), 0, pa.data(), pb.data(), pd.data(), hab.data(), ld, Vl,
                                    (size_t)k * ld, lus.data(), st);
    if (e < 0) return e;
    if (e > 0 && warn == NK_OK) warn = e;
    NK_HIP(hipMemcpyAsync(abd, hab.data(), hab.size() * sizeof(C64), hipMemcpyHostToDevice, st));
  } else {
    for (int s = 0; s < r; ++s) {
      lus[s] = kus[s];
      for (int t = 0; t < 3; ++t)
        NK_HIP(hipMemcpyAsync(abd + (size_t)s * 3 * ld + (size_t)t * ld,
                              (t == 0 ? a.alpha : t == 1 ? a.beta : a.delta) + (size_t)s * k, kus[s] * sizeof(C64),
                              hipMemcpyDeviceToDevice, st));
    }
  }
  NK_HIP(hipMemcpyAsync(kv, kus.data(), r * sizeof(int), hipMemcpyHostToDevice, st));
  NK_HIP(hipMemcpyAsync(lv, lus.data(), r * sizeof(int), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_tri_dense_b, dim3(64, r), dim3(256), 0, st, ld, lv, abd, S);
  NK_HIP(hipGetLastError());
  std::vector<int> its(r);
  std::vector<double> res(r);
  const int erh = rh_sign_batched(r, ld, lus.data(), S, p->rh_scaling, p->rh_maxit, p->rh_tol, its.data(), res.data(),
                                  st);
  if (erh < 0) return erh;
  if (erh > 0 && warn == NK_OK) warn = erh;
  hipLaunchKernelGGL(k_bz, dim3((k + 255) / 256, r), dim3(256), 0, st, k, ld, kv, lv, nested, Vl, S, z);
  NK_HIP(hipGetLastError());
  NK_HIP(hipEventRecord(ev[2], st));
  // lift
  if (store) {
    for (int s = 0; s < r; ++s) {
      C64* y = a.base + ((size_t)s * a.nslots + a.ncols + 5) * n;
      if (int e = lift_columns((int)n, kus[s], a.base + (size_t)s * a.nslots * n, n, z + (size_t)s * k,
                               a.sv + (size_t)s * (k + 1), lc + (size_t)s * k, y, st))
        return e;
    }
  } else {
    hipLaunchKernelGGL(k_blc, dim3((k + 255) / 256, r), dim3(256), 0, st, k, kv, z, a.sv, lc);
    NK_HIP(hipGetLastError());
    BArgs b = a;
    b.lc = lc;
    // the second sweep recomputes the coefficients bit for bit; reset the state it reads
    NK_HIP(hipMemsetAsync(a.flags, 0, r * sizeof(int), st));
    int kmax = 0;
    for (int s = 0; s < r; ++s) kmax = std::max(kmax, kus[s]);
    if (int e = run_sweep(b, kmax - 1 > 0 ? kmax - 1 : 0)) return e;
  }
  for (int s = 0; s < r; ++s) {
    const C64* y = a.base + ((size_t)s * a.nslots + a.ncols + 5) * n;
    if (int e = unpack_spinor<double>(g, y, y_canon + (size_t)s * n, st)) return e;
  }
  NK_HIP(hipEventRecord(ev[3], st));
  NK_HIP(hipStreamSynchronize(st));
  if (info) {
    float t0 = 0, t1 = 0, t2 = 0;
    NK_HIP(hipEventElapsedTime(&t0, ev[0], ev[1]));
    NK_HIP(hipEventElapsedTime(&t1, ev[1], ev[2]));
    NK_HIP(hipEventElapsedTime(&t2, ev[2], ev[3]));
    info->k_used = kus[r - 1];
    info->ell_used = nested ? lus[r - 1] : 0;
    info->rh_iters = its[r - 1];
    info->breakdown_step = brk;
    info->two_pass = store ? 0 : 1;
    info->est = std::numeric_limits<double>::quiet_NaN();
    info->rh_residual = res[r - 1];
    info->t_basis_ms = t0;
    info->t_small_ms = t1;
    info->t_lift_ms = t2;
  }
  if (p->profile) {  // per launch: each covers all r sources of this range
    double a1 = 0, a2 = 0;
    int n1 = 0, n2 = 0;
    if (int e = prof_collect(lat, &a1, &a2, &n1, &n2)) return e;
    if (info) {
      info->t_stencil_ms += a1;
      info->t_update_ms += a2;
      info->n_stencil += n1;
      info->n_update += n2;
    }
  }
  return warn;
}

int block_sign(nk_lattice* lat, const nk_sign_params* p, const C64* x_canon, C64* y_canon, nk_sign_info* info,
               hipStream_t st) {
  const int r = p->nrhs, k = p->k;
  if (p->mu == 0.0 || p->precision != NK_PREC_FP64 || p->tol > 0.0 || p->inner != NK_INNER_SAME)
    return 1;  // not covered: one at a time
  const size_t n = (size_t)12 * lat->g.V;
  std::vector<int> ell(r);
  for (int s = 0; s < r; ++s) ell[s] = std::min(p->ell_per_rhs ? p->ell_per_rhs[s] : p->ell, k);
  if (p->two_pass == NK_TWO_PASS_ON) return block_range(lat, p, ell.data(), r, 0, x_canon, y_canon, info, st);
  // store every basis when they fit; else as many sources at a time as fit
  // with stored bases (a stored basis costs one sweep, a rebuilt one two);
  // only when not even two fit, rebuild them all in a second sweep
  const size_t per_src = (size_t)(k + 7) * n * sizeof(C64);
  const size_t margin = (size_t)4 << 30;
  size_t fr = 0, tot = 0;
  NK_HIP(hipMemGetInfo(&fr, &tot));
  size_t avail = fr + lat->bvec.bytes;
  if ((size_t)r * per_src + margin > avail && lat->vk.bytes) {  // the one-source basis is not needed here
    lat->vk.release();
    NK_HIP(hipMemGetInfo(&fr, &tot));
    avail = fr + lat->bvec.bytes;
  }
  const long fit = avail > margin ? (long)((avail - margin) / per_src) : 0;
  if (fit >= r) return block_range(lat, p, ell.data(), r, 1, x_canon, y_canon, info, st);
  if (fit < 2) {
    if (p->two_pass == NK_TWO_PASS_OFF) {
      set_error("a stored basis needs %zu bytes per source; %zu available and two_pass is OFF", per_src, avail);
      return NK_ENOMEM;
    }
    return block_range(lat, p, ell.data(), r, 0, x_canon, y_canon, info, st);
  }
  int worst = NK_OK;
  for (int c0 = 0; c0 < r; c0 += (int)fit) {
    const int cnt = std::min((int)fit, r - c0);
    const int e = block_range(lat, p, ell.data() + c0, cnt, 1, x_canon + (size_t)c0 * n, y_canon + (size_t)c0 * n,
                              info, st);
    if (e < 0) return e;
    worst = std::max(worst, e);
  }
  return worst;
}

}  // namespace nk
