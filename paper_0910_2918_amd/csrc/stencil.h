// Per-site hopping term of the Wilson-Dirac operator Dw(mu) on gfx950.
//
// The operator (Sec. 1 of the paper names it; its explicit form is the
// standard one with the Hasenfratz-Karsch chemical potential):
//   Dw psi(x) = (4 + m_w) psi(x) - 1/2 hop(x),
//   hop(x) = sum_nu e^{+mu d_{nu t}} (1 - gamma_nu) U_nu(x) psi(x + nu)
//                 + e^{-mu d_{nu t}} (1 + gamma_nu) U_nu(x - nu)^dag psi(x - nu),
// antiperiodic in t.  In the chiral basis (1 -/+ gamma_nu) has rank two: for
// each nu there are unit complex numbers c0, c1 and lower spins p0, p1 with
//   (1 - gamma_nu) psi = [h0, h1; conj(c0) h0 at spin p0, conj(c1) h1 at spin p1],
//   h0 = psi_0 + c0 psi_p0,  h1 = psi_1 + c1 psi_p1,
// and (1 + gamma_nu) the same with c -> -c.  So each hop multiplies only a
// two-spin half spinor by the SU(3) link (spin projection), 2 x 9 complex
// products instead of 4 x 9.
#pragma once

#include "nk_internal.h"

namespace nk {

// kernel-argument bundles of NF field pointers and temporal hop factors
template <class R, int NF>
struct FieldPtrs {
  const Cx<R>* p[NF];
};
template <class R, int NF>
struct FieldPtrsW {
  Cx<R>* p[NF];
};
template <class R, int NF>
struct TFac {
  R f[NF];  // forward temporal factor
  R b[NF];  // backward temporal factor
};

// (c0, p0, c1, p1) of the projector table; c = (CR + i CI)
template <int NU>
struct Proj;
template <>
struct Proj<0> {  // gamma_1 = [[0, -i s1], [i s1, 0]]
  static constexpr int p0 = 3, p1 = 2, c0r = 0, c0i = 1, c1r = 0, c1i = 1;
};
template <>
struct Proj<1> {  // gamma_2
  static constexpr int p0 = 3, p1 = 2, c0r = 1, c0i = 0, c1r = -1, c1i = 0;
};
template <>
struct Proj<2> {  // gamma_3
  static constexpr int p0 = 2, p1 = 3, c0r = 0, c0i = 1, c1r = 0, c1i = -1;
};
template <>
struct Proj<3> {  // gamma_4 = [[0, 1], [1, 0]]
  static constexpr int p0 = 2, p1 = 3, c0r = -1, c0i = 0, c1r = -1, c1i = 0;
};

// (CR + i CI) z for a unit CR + i CI in {1, -1, i, -i}
template <int CR, int CI, class R>
__device__ __forceinline__ Cx<R> mulu(Cx<R> z) {
  if constexpr (CI == 0) {
    if constexpr (CR > 0) return z;
    else return mk<R>(-z.re, -z.im);
  } else if constexpr (CI > 0) {
    return mk<R>(-z.im, z.re);
  } else {
    return mk<R>(z.im, -z.re);
  }
}

// --- link storage -----------------------------------------------------------
// FP64: one 16-byte load per entry
template <class R>
struct LinksPlain {
  const Cx<R>* U;
  int V;
  __device__ __forceinline__ void load(int nu, int s, Cx<R> (&u)[9]) const {
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = U[(size_t)(nu * 9 + e) * V + s];
  }
};

// FP32: entries in pairs, four 16-byte loads and one 8-byte load per link
template <>
struct LinksPlain<float> {
  const Cx<float>* U;
  int V;
  __device__ __forceinline__ void load(int nu, int s, Cx<float> (&u)[9]) const {
    const float4* P = reinterpret_cast<const float4*>(U);
#pragma unroll
    for (int pe = 0; pe < 4; ++pe) {
      const float4 t = P[(size_t)(nu * 5 + pe) * V + s];
      u[2 * pe] = mk<float>(t.x, t.y);
      u[2 * pe + 1] = mk<float>(t.z, t.w);
    }
    u[8] = U[((size_t)(nu * 5 + 4) * V + s) * 2];
  }
};

__device__ __forceinline__ float bf16lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// BF16 storage of the first two rows (12 reals as 6 packed complex words,
// one 16-byte and one 8-byte load); the rows are re-orthonormalised in FP32
// and the third row is rebuilt as conj(row0 x row1), which makes the link
// exactly special unitary again.
struct LinksBF16 {
  const uint32_t* U;
  int V;
  __device__ __forceinline__ void load(int nu, int s, Cx<float> (&u)[9]) const {
    const uint4 a = reinterpret_cast<const uint4*>(U)[(size_t)nu * V + s];
    const uint2 b = reinterpret_cast<const uint2*>(U + (size_t)16 * V)[(size_t)nu * V + s];
    const uint32_t wv[6] = {a.x, a.y, a.z, a.w, b.x, b.y};
    Cx<float> r[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) r[e] = mk<float>(bf16lo(wv[e]), bf16hi(wv[e]));
    float n0 = norm2(r[0]) + norm2(r[1]) + norm2(r[2]);
    float i0 = rsqrtf(n0);
#pragma unroll
    for (int b = 0; b < 3; ++b) r[b] = i0 * r[b];
    Cx<float> d = cmulc(r[0], r[3]) + cmulc(r[1], r[4]) + cmulc(r[2], r[5]);
#pragma unroll
    for (int b = 0; b < 3; ++b) r[3 + b] = r[3 + b] - cmul(d, r[b]);
    float n1 = norm2(r[3]) + norm2(r[4]) + norm2(r[5]);
    float i1 = rsqrtf(n1);
#pragma unroll
    for (int b = 0; b < 3; ++b) r[3 + b] = i1 * r[3 + b];
#pragma unroll
    for (int e = 0; e < 6; ++e) u[e] = r[e];
    u[6] = conj(cmul(r[1], r[5]) - cmul(r[2], r[4]));
    u[7] = conj(cmul(r[2], r[3]) - cmul(r[0], r[5]));
    u[8] = conj(cmul(r[0], r[4]) - cmul(r[1], r[3]));
  }
};

template <class R>
__device__ __forceinline__ void load_spinor(const Cx<R>* __restrict__ f, int V, int s, Cx<R> (&p)[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) p[c] = f[(size_t)c * V + s];
}
// FP32: six 16-byte loads of component pairs
template <>
__device__ __forceinline__ void load_spinor<float>(const Cx<float>* __restrict__ f, int V, int s,
                                                   Cx<float> (&p)[12]) {
  const float4* P = reinterpret_cast<const float4*>(f);
#pragma unroll
  for (int cp = 0; cp < 6; ++cp) {
    const float4 t = P[(size_t)cp * V + s];
    p[2 * cp] = mk<float>(t.x, t.y);
    p[2 * cp + 1] = mk<float>(t.z, t.w);
  }
}

// Keep the accumulators materialised at this point of the program: an empty
// asm that reads and writes them stops LLVM from sinking the arithmetic of
// every hop below the last loads, which would keep all loaded values live at
// once.  It emits no instruction.
template <class R, int NF>
__device__ __forceinline__ void pin(Cx<R> (&acc)[NF][12]) {
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int c = 0; c < 12; ++c) asm volatile("" : "+v"(acc[f][c].re), "+v"(acc[f][c].im));
}

// coordinates of a device site: local (within the tile) and tile coordinates
struct SiteC {
  int cl[4], ct[4];
};

__device__ __forceinline__ SiteC site_coords(const Geom& g, int s) {
  SiteC c;
  int l = s & ((1 << g.lts) - 1);
  int T = s >> g.lts;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    c.cl[d] = l & (g.b[d] - 1);
    l >>= g.lb[d];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    c.ct[d] = T % g.nt[d];
    T /= g.nt[d];
  }
  c.ct[3] = T;
  return c;
}

// neighbour x + nu and x - nu; *wrap is set when the hop crosses the
// lattice boundary in direction nu
template <int NU>
__device__ __forceinline__ int nbr_fwd(const Geom& g, int s, const SiteC& c, bool* wrap) {
  *wrap = false;
  if (c.cl[NU] < g.b[NU] - 1) return s + g.lstr[NU];
  const int base = s - (g.b[NU] - 1) * g.lstr[NU];
  if (c.ct[NU] == g.nt[NU] - 1) {
    *wrap = true;
    return base - (g.nt[NU] - 1) * g.tstr[NU];
  }
  return base + g.tstr[NU];
}
template <int NU>
__device__ __forceinline__ int nbr_bwd(const Geom& g, int s, const SiteC& c, bool* wrap) {
  *wrap = false;
  if (c.cl[NU] > 0) return s - g.lstr[NU];
  const int base = s + (g.b[NU] - 1) * g.lstr[NU];
  if (c.ct[NU] == 0) {
    *wrap = true;
    return base + (g.nt[NU] - 1) * g.tstr[NU];
  }
  return base - g.tstr[NU];
}

#ifndef NK_HOP_FENCE
#define NK_HOP_FENCE 1  // schedule each hop on its own (bounded registers)
#endif

__device__ __forceinline__ void hop_fence() {
#if NK_HOP_FENCE
  __builtin_amdgcn_sched_barrier(0);
#endif
}

// forward hop in direction nu for NF fields: (1 - gamma) U_nu(x) psi(x + nu)
template <int NU, class R, int NF, class LK>
__device__ __forceinline__ void hop_fwd(const Geom& g, int s, const SiteC& sc0, const LK& lk,
                                        const Cx<R>* const (&in)[NF], const R (&cf)[NF], Cx<R> (&acc)[NF][12]) {
  using P = Proj<NU>;
  const int V = g.V;
  bool wrap;
  const int sf = nbr_fwd<NU>(g, s, sc0, &wrap);
  const R bf = (NU == 3 && wrap) ? R(-1) : R(1);
  Cx<R> u[9];
  Cx<R> h0[NF][3], h1[NF][3];
  hop_fence();
  lk.load(NU, s, u);
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    Cx<R> p[12];
    load_spinor(in[f], V, sf, p);
    const R sc = bf * cf[f];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      h0[f][c] = sc * (p[c] + mulu<P::c0r, P::c0i>(p[P::p0 * 3 + c]));
      h1[f][c] = sc * (p[3 + c] + mulu<P::c1r, P::c1i>(p[P::p1 * 3 + c]));
    }
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Cx<R> g0 = cmul(u[a * 3 + 0], h0[f][0]) + cmul(u[a * 3 + 1], h0[f][1]) + cmul(u[a * 3 + 2], h0[f][2]);
      Cx<R> g1 = cmul(u[a * 3 + 0], h1[f][0]) + cmul(u[a * 3 + 1], h1[f][1]) + cmul(u[a * 3 + 2], h1[f][2]);
      acc[f][a] = acc[f][a] + g0;
      acc[f][3 + a] = acc[f][3 + a] + g1;
      acc[f][P::p0 * 3 + a] = acc[f][P::p0 * 3 + a] + mulu<P::c0r, -P::c0i>(g0);
      acc[f][P::p1 * 3 + a] = acc[f][P::p1 * 3 + a] + mulu<P::c1r, -P::c1i>(g1);
    }
  }
  pin<R, NF>(acc);
}

// backward hop in direction nu for NF fields: (1 + gamma) U_nu(x - nu)^dag psi(x - nu)
template <int NU, class R, int NF, class LK>
__device__ __forceinline__ void hop_bwd(const Geom& g, int s, const SiteC& sc0, const LK& lk,
                                        const Cx<R>* const (&in)[NF], const R (&cb)[NF], Cx<R> (&acc)[NF][12]) {
  using P = Proj<NU>;
  const int V = g.V;
  bool wrap;
  const int sb = nbr_bwd<NU>(g, s, sc0, &wrap);
  const R bb = (NU == 3 && wrap) ? R(-1) : R(1);
  Cx<R> u[9];
  Cx<R> h0[NF][3], h1[NF][3];
  hop_fence();
  lk.load(NU, sb, u);
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    Cx<R> p[12];
    load_spinor(in[f], V, sb, p);
    const R sc = bb * cb[f];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      h0[f][c] = sc * (p[c] - mulu<P::c0r, P::c0i>(p[P::p0 * 3 + c]));
      h1[f][c] = sc * (p[3 + c] - mulu<P::c1r, P::c1i>(p[P::p1 * 3 + c]));
    }
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Cx<R> g0 = cmulc(u[0 * 3 + a], h0[f][0]) + cmulc(u[1 * 3 + a], h0[f][1]) + cmulc(u[2 * 3 + a], h0[f][2]);
      Cx<R> g1 = cmulc(u[0 * 3 + a], h1[f][0]) + cmulc(u[1 * 3 + a], h1[f][1]) + cmulc(u[2 * 3 + a], h1[f][2]);
      acc[f][a] = acc[f][a] + g0;
      acc[f][3 + a] = acc[f][3 + a] + g1;
      acc[f][P::p0 * 3 + a] = acc[f][P::p0 * 3 + a] - mulu<P::c0r, -P::c0i>(g0);
      acc[f][P::p1 * 3 + a] = acc[f][P::p1 * 3 + a] - mulu<P::c1r, -P::c1i>(g1);
    }
  }
  pin<R, NF>(acc);
}

// --- direction groups over the waves of a workgroup -------------------------
// The stencil kernels give each site's eight hops to NG waves of a 256-thread
// workgroup: wave w takes direction group w % NG (NG = 4: one direction,
// forward and backward hop; NG = 2: x and y, or z and t) for a block of sites.
// The partial hopping sums then meet in LDS, where each wave finishes 12 / NG
// of the 12 components, adding the groups in group order so that the result
// does not depend on timing.  Against one lane doing all eight hops, the
// eight hops of a site are in flight at once, and a workgroup covers NG times
// fewer sites, so fewer sites are in flight per XCD and the neighbour spinors
// and links they share are still in the XCD's L2 when the next site asks.
//
// No 12-component accumulator lives across the hops of a group: each hop's
// contribution goes straight to the wave's own LDS slots (the first hop
// stores, later hops add) and to the M components the wave keeps, so while a
// hop's link and spinor loads are in flight only those M components are live.
// The additions happen in the same order as with one accumulator per lane,
// ((h1 + h2) + h3) + ..., so the result is the same to the last bit.

#ifndef NK_GROUPS
#define NK_GROUPS 4  // direction groups of the stencil kernels (2 or 4)
#endif

// LDS exchange of the partial hopping sums of the 4 waves of a workgroup
template <class R, int NG>
struct XBuf {
  static constexpr int M = 12 / NG;  // components each wave finishes
  Cx<R> v[4][12 - M][64];            // per wave: the components other waves finish
};

// slot of component cc in the buffer of group gg: below gg's own range it
// keeps its index, above it moves down by M
template <int NG>
__device__ __forceinline__ constexpr int xslot(int cc, int gg) {
  constexpr int M = 12 / NG;
  return cc < gg * M ? cc : cc - M;
}

// hand one hop's contribution acc (all 12 components) of group GI to the
// exchange: components other groups finish go to the wave's LDS slots, its
// own M components to mine[]; FIRST stores, otherwise adds
template <int NG, int GI, bool FIRST, class R>
__device__ __forceinline__ void xacc(XBuf<R, NG>& xb, int w, int lane, const Cx<R> (&acc)[1][12],
                                     Cx<R> (&mine)[12 / NG]) {
  constexpr int M = 12 / NG;
#pragma unroll
  for (int cc = 0; cc < 12; ++cc) {
    if (cc / M == GI) {
      mine[cc - GI * M] = FIRST ? acc[0][cc] : mine[cc - GI * M] + acc[0][cc];
    } else {
      Cx<R>& slot = xb.v[w][xslot<NG>(cc, GI)][lane];
      slot = FIRST ? acc[0][cc] : slot + acc[0][cc];
    }
  }
}

// one hop (forward or backward in direction NU) of group GI, handed to the
// exchange
template <bool FWD, int NU, int NG, int GI, bool FIRST, class R, class LK>
__device__ __forceinline__ void hop_x(const Geom& g, int s, const SiteC& x, const LK& lk, const Cx<R>* in, R tf,
                                      XBuf<R, NG>& xb, int w, int lane, Cx<R> (&mine)[12 / NG]) {
  const Cx<R>* ins[1] = {in};
  const R f1[1] = {NU == 3 ? tf : R(1)};
  Cx<R> acc[1][12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[0][c] = mk<R>(0, 0);
  if constexpr (FWD)
    hop_fwd<NU>(g, s, x, lk, ins, f1, acc);
  else
    hop_bwd<NU>(g, s, x, lk, ins, f1, acc);
  xacc<NG, GI, FIRST>(xb, w, lane, acc, mine);
}

// hopping sum of direction group gi (wave-uniform) of one field at site s,
// left in the exchange (LDS slots of wave w and mine[]); ef/eb are the
// forward/backward temporal factors
template <int NG, class R, class LK>
__device__ __forceinline__ void hop_group(const Geom& g, int s, const LK& lk, const Cx<R>* in, int gi, R ef, R eb,
                                          XBuf<R, NG>& xb, int w, int lane, Cx<R> (&mine)[12 / NG]) {
  const SiteC x = site_coords(g, s);
  if constexpr (NG == 4) {
    if (gi == 0) {
      hop_x<true, 0, 4, 0, true>(g, s, x, lk, in, ef, xb, w, lane, mine);
      hop_x<false, 0, 4, 0, false>(g, s, x, lk, in, eb, xb, w, lane, mine);
    } else if (gi == 1) {
      hop_x<true, 1, 4, 1, true>(g, s, x, lk, in, ef, xb, w, lane, mine);
      hop_x<false, 1, 4, 1, false>(g, s, x, lk, in, eb, xb, w, lane, mine);
    } else if (gi == 2) {
      hop_x<true, 2, 4, 2, true>(g, s, x, lk, in, ef, xb, w, lane, mine);
      hop_x<false, 2, 4, 2, false>(g, s, x, lk, in, eb, xb, w, lane, mine);
    } else {
      hop_x<true, 3, 4, 3, true>(g, s, x, lk, in, ef, xb, w, lane, mine);
      hop_x<false, 3, 4, 3, false>(g, s, x, lk, in, eb, xb, w, lane, mine);
    }
  } else {
    static_assert(NG == 2, "2 or 4 direction groups");
    if (gi == 0) {
      hop_x<true, 0, 2, 0, true>(g, s, x, lk, in, ef, xb, w, lane, mine);
      hop_x<false, 0, 2, 0, false>(g, s, x, lk, in, eb, xb, w, lane, mine);
      hop_x<true, 1, 2, 0, false>(g, s, x, lk, in, ef, xb, w, lane, mine);
      hop_x<false, 1, 2, 0, false>(g, s, x, lk, in, eb, xb, w, lane, mine);
    } else {
      hop_x<true, 2, 2, 1, true>(g, s, x, lk, in, ef, xb, w, lane, mine);
      hop_x<false, 2, 2, 1, false>(g, s, x, lk, in, eb, xb, w, lane, mine);
      hop_x<true, 3, 2, 1, false>(g, s, x, lk, in, ef, xb, w, lane, mine);
      hop_x<false, 3, 2, 1, false>(g, s, x, lk, in, eb, xb, w, lane, mine);
    }
  }
}

// after a workgroup barrier: the full hopping sum of component gi * M + cl of
// the site block sb, summed over the groups in group order
template <int NG, class R>
__device__ __forceinline__ Cx<R> xsum(const XBuf<R, NG>& xb, int sb, int gi, int lane, int cl, const Cx<R>& mine) {
  constexpr int M = 12 / NG;
  const int cc = gi * M + cl;
  Cx<R> hs = mk<R>(0, 0);
#pragma unroll
  for (int gg = 0; gg < NG; ++gg) {
    if (gg == gi)
      hs = hs + mine;
    else
      hs = hs + xb.v[sb * NG + gg][xslot<NG>(cc, gg)][lane];
  }
  return hs;
}

// the value held by the other lane of a lane pair (lane ^ 1), by a DPP quad
// permutation (1, 0, 3, 2); both lanes of the pair must be active
__device__ __forceinline__ int pair_swap(int x) { return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false); }
__device__ __forceinline__ float pair_swap(float x) { return __int_as_float(pair_swap(__float_as_int(x))); }
__device__ __forceinline__ double pair_swap(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)pair_swap((int)(unsigned)b), hi = (unsigned)pair_swap((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <class R>
__device__ __forceinline__ Cx<R> pair_swap(Cx<R> z) {
  return mk<R>(pair_swap(z.re), pair_swap(z.im));
}

// gamma5 sign of component c = spin*3 + colour
__device__ __forceinline__ constexpr int g5sign(int c) { return c < 6 ? 1 : -1; }

// XCD-aware block order: consecutive logical tiles stay on one XCD (the
// hardware hands workgroup b to XCD b % 8), so neighbouring sites share an L2.
#ifndef NK_XCD_MAP
#define NK_XCD_MAP 1
#endif
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  if (!NK_XCD_MAP || (nb & 7) != 0) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

}  // namespace nk
