// Many sources in lockstep: the outer two-sided Lanczos basis of Sec. 2 for
// r sources at once, the small problems of Eqs. (3)-(6) batched, and the lift.
//
// Each source keeps its own recurrence and coefficients; what they share is
// the gauge field.  The stencil kernel (k_blk1) gives every wave of a
// workgroup one direction of 32 sites, loads that direction's two links
// into registers once, and then applies them to all r sources in turn, so
// the links cost 576 bytes per site per step for all sources together
// instead of per source.  A step is four launches for all sources:
//   k_blk1  A v_j, A^dag w_j minus the previous vectors, partial w~^dag A v~
//   k_bred1 alpha_j per source (fixed-order reduction)
//   k_blk2  v_hat, w_hat (new unnormalised columns), partial s, |v|^2, |w|^2
//   k_bred2 delta, beta, the scales and the breakdown test per source
// Every reduction is deterministic, so a second sweep over the same data
// (two-pass lift) reproduces the first bit for bit.  The small problems run
// as one inner projection per source followed by one batched
// Roberts-Higham call over the uneven ell of all sources.
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

// both hops of direction NU with the links in registers
template <int NU>
__device__ __forceinline__ void dir_hops(const Cx<double> (&uf)[9], const Cx<double> (&ub)[9], const C64* in, int V,
                                         int sf, int sb, double cf, double cb, C64 (&acc)[12]) {
  hop_with<NU, true>(uf, in, V, sf, cf, acc);
  hop_fence();
  hop_with<NU, false>(ub, in, V, sb, cb, acc);
}

// the stencil step of every running source: p = A v_j - beta_j v_{j-1},
// q = A^dag w_j - delta_j w_{j-1} (both scaled by the lazy normalisation),
// partial w~_j^dag (A v~_j).  Four waves = four directions of 32 sites, two
// lanes per site (even: A v, odd: A^dag w).
__global__ void __launch_bounds__(BT) k_blk1(Geom g, LinksPlain<double> lk, double diag, double eft, double ebt,
                                              int j, BArgs a) {
  constexpr int NG = 4, M = 3;
  __shared__ XBuf<double, NG> xb;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gi = w;  // direction of this wave
  const int f = lane & 1;
  const int s = xcd_block() * 32 + (lane >> 1);
  const bool live = s < g.V;
  const int sh = live ? s : 0;
  const SiteC x = site_coords(g, sh);
  Cx<double> uf[9], ub[9];
  int sf, sb;
  double wf, wb;
  if (gi == 0)
    hop_setup<0>(g, sh, x, lk, uf, ub, sf, sb, wf, wb);
  else if (gi == 1)
    hop_setup<1>(g, sh, x, lk, uf, ub, sf, sb, wf, wb);
  else if (gi == 2)
    hop_setup<2>(g, sh, x, lk, uf, ub, sf, sb, wf, wb);
  else
    hop_setup<3>(g, sh, x, lk, uf, ub, sf, sb, wf, wb);
  // temporal factors: A(mu) on v, A(-mu) = A(mu)^dag on w
  const double cf = gi == 3 ? wf * (f ? ebt : eft) : wf;
  const double cb = gi == 3 ? wb * (f ? eft : ebt) : wb;
  for (int src = 0; src < a.r; ++src) {
    if (a.flags[src]) continue;  // the same in every thread
    const C64* in = f ? colw(a, src, j) : colv(a, src, j);
    C64 mine[M];
    {
      C64 acc[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] = mk(0.0, 0.0);
      if (gi == 0)
        dir_hops<0>(uf, ub, in, g.V, sf, sb, cf, cb, acc);
      else if (gi == 1)
        dir_hops<1>(uf, ub, in, g.V, sf, sb, cf, cb, acc);
      else if (gi == 2)
        dir_hops<2>(uf, ub, in, g.V, sf, sb, cf, cb, acc);
      else
        dir_hops<3>(uf, ub, in, g.V, sf, sb, cf, cb, acc);
      C64 a1[1][12];
#pragma unroll
      for (int c = 0; c < 12; ++c) a1[0][c] = acc[c];
      xput<NG>(xb, w, gi, lane, a1, mine);
    }
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
    if (live) {
      int se = s;
      asm volatile("" : "+v"(se));
#pragma unroll
      for (int cl = 0; cl < M; ++cl) {
        const int cc = gi * M + cl;
        const C64 hs = xsum<NG>(xb, 0, gi, lane, cl, mine[cl]);
        const size_t i = (size_t)cc * g.V + se;
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
    double v[2] = {dre, dim};
    bsum<2>(v);  // its barriers also order this source's exchange reads before the next one's writes
    if (threadIdx.x == 0) {
      double* p1 = a.part1 + (size_t)src * 2 * a.nb1;
      p1[blockIdx.x] = v[0];
      p1[a.nb1 + blockIdx.x] = v[1];
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
  for (size_t i = (size_t)blockIdx.x * BT + threadIdx.x; i < a.n; i += (size_t)gridDim.x * BT) {
    const C64 vr = p[i] - cmul(av, v[i]);
    const C64 wr = q[i] - cmul(aw, w[i]);
    vn[i] = vr;
    wn[i] = wr;
    const C64 t = cmulc(wr, vr);
    sre += t.re;
    sim += t.im;
    nv += norm2(vr);
    nw += norm2(wr);
    if (lift) y[i] = y[i] + cmul(lcn, vr);
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

// one sweep of the basis for every source: steps 0 .. kmax - 1
int sweep(nk_lattice* lat, const BArgs& a, double m_w, double mu, int kmax, hipStream_t st) {
  const Geom& g = lat->g;
  const LinksPlain<double> lk{lat->U64.as<C64>(), g.V};
  hipLaunchKernelGGL(k_bstart, dim3(a.nb2, a.r), dim3(BT), 0, st, a);
  hipLaunchKernelGGL(k_bred2, dim3(a.r), dim3(BT), 0, st, a, 0);
  const double eft = exp(mu), ebt = exp(-mu);
  for (int j = 0; j < kmax; ++j) {
    hipLaunchKernelGGL(k_blk1, dim3(a.nb1), dim3(BT), 0, st, g, lk, 4.0 + m_w, eft, ebt, j, a);
    hipLaunchKernelGGL(k_bred1, dim3(a.r), dim3(BT), 0, st, a, j);
    hipLaunchKernelGGL(k_blk2, dim3(a.nb2, a.r), dim3(BT), 0, st, a, j);
    if (j + 1 < kmax) hipLaunchKernelGGL(k_bred2, dim3(a.r), dim3(BT), 0, st, a, j + 1);
  }
  NK_HIP(hipGetLastError());
  return NK_OK;
}

}  // namespace

int block_sign(nk_lattice* lat, const nk_sign_params* p, const C64* x_canon, C64* y_canon, nk_sign_info* info,
               hipStream_t st) {
  const Geom& g = lat->g;
  const int r = p->nrhs, k = p->k;
  if (p->mu == 0.0 || p->precision != NK_PREC_FP64 || p->tol > 0.0) return 1;  // not covered: one at a time
  const size_t n = (size_t)12 * g.V;
  const size_t colbytes = n * sizeof(C64);
  std::vector<int> ell(r);
  for (int s = 0; s < r; ++s) ell[s] = std::min(p->ell_per_rhs ? p->ell_per_rhs[s] : p->ell, k);
  // store every column when it fits, else rebuild the basis in a second sweep
  size_t fr = 0, tot = 0;
  NK_HIP(hipMemGetInfo(&fr, &tot));
  const size_t avail = fr + lat->bvec.bytes;
  const size_t margin = (size_t)4 << 30;
  const size_t store_bytes = (size_t)r * (k + 7) * colbytes;
  int store = p->two_pass == NK_TWO_PASS_ON ? 0 : (store_bytes + margin <= avail ? 1 : 0);
  if (!store && p->two_pass == NK_TWO_PASS_OFF) {
    set_error("the bases of %d sources need %zu bytes; %zu available and two_pass is OFF", r, store_bytes, avail);
    return NK_ENOMEM;
  }
  BArgs a{};
  a.n = n;
  a.ncols = store ? k + 1 : 3;
  a.nslots = a.ncols + 6;
  a.store = store;
  a.r = r;
  a.k = k;
  a.nb1 = (g.V + 31) / 32;
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
  if (int e = sweep(lat, a, p->m_w, p->mu, k, st)) return e;
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
    std::vector<C64> hl((size_t)3 * ld);
    for (int s = 0; s < r; ++s) {
      SmallOut so;
      so.hl_host = hl.data();
      so.vl_dev = Vl + (size_t)s * k * ld;
      so.inner_only = true;
      const int e = small_sign_dev(kus[s], std::min(ell[s], kus[s]), 0, a.alpha + (size_t)s * k,
                                   a.beta + (size_t)s * k, a.delta + (size_t)s * k, p->rh_scaling, p->rh_maxit,
                                   p->rh_tol, z, &so, st);
      if (e < 0) return e;
      if (e > 0 && warn == NK_OK) warn = e;
      lus[s] = so.ell_used;
      for (int t = 0; t < 3; ++t)
        std::copy(hl.begin() + (size_t)t * lus[s], hl.begin() + (size_t)(t + 1) * lus[s],
                  hab.begin() + (size_t)s * 3 * ld + (size_t)t * ld);
    }
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
    if (int e = sweep(lat, b, p->m_w, p->mu, kmax - 1 > 0 ? kmax - 1 : 0, st)) return e;
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
  return warn;
}

}  // namespace nk
