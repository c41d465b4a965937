// Stand-alone applications of gamma5 Dw(mu): the single operator and the
// fused pair (A v, A^dag w) of two-sided Lanczos (A^dag = A(-mu)).
#include "stencil.h"

namespace nk {

// y_f = [gamma5] ((4 + m_w) x_f - 1/2 hop(x_f)) for NF fields, device layout.
// Directions split over the waves of the workgroup (hop_group); NF lanes per
// site, lane f on field f.
template <class R, int NF, class LK, int NG>
__global__ void __launch_bounds__(256) k_apply(Geom g, LK lk, R diag, int g5, FieldPtrs<R, NF> in,
                                                FieldPtrsW<R, NF> out, TFac<R, NF> tf) {
  constexpr int M = 12 / NG;
  constexpr int SPW = 64 / NF;         // sites per wave
  constexpr int NSB = (256 / 64) / NG;  // site blocks per workgroup
  __shared__ XBuf<R, NG> xb;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gi = w % NG, sb = w / NG;
  const int f = NF == 1 ? 0 : lane & 1;
  const Cx<R>* x = NF == 1 ? in.p[0] : (f ? in.p[NF - 1] : in.p[0]);
  Cx<R>* y = NF == 1 ? out.p[0] : (f ? out.p[NF - 1] : out.p[0]);
  const R ef = NF == 1 ? tf.f[0] : (f ? tf.f[NF - 1] : tf.f[0]);
  const R eb = NF == 1 ? tf.b[0] : (f ? tf.b[NF - 1] : tf.b[0]);
  const int s = (xcd_block() * NSB + sb) * SPW + lane / NF;
  const bool live = s < g.V;
  Cx<R> mine[M];
  hop_group<NG>(g, live ? s : 0, lk, x, gi, ef, eb, xb, w, lane, mine);  // a lane past the end hops at site 0
  __builtin_amdgcn_sched_barrier(0);  // the stencil's registers are free before these loads
  // this site's input entries go out before the exchange's barrier, which
  // they then overlap
  int se = s;
  asm volatile("" : "+v"(se));  // keeps the epilogue addresses out of the stencil's registers
  Cx<R> ein[M];
#pragma unroll
  for (int cl = 0; cl < M; ++cl) ein[cl] = x[sidx<R>(g.V, gi * M + cl, live ? se : 0)];
  __syncthreads();
  if (!live) return;
#pragma unroll
  for (int cl = 0; cl < M; ++cl) {
    const int cc = gi * M + cl;
    const Cx<R> hs = xsum<NG>(xb, sb, gi, lane, cl, mine[cl]);
    const size_t i = sidx<R>(g.V, cc, se);
    Cx<R> o = diag * ein[cl] - R(0.5) * hs;
    if (g5 && cc >= 6) o = mk<R>(-o.re, -o.im);
    y[i] = o;
  }
}

// workgroups of k_apply for NF fields
static int apply_blocks(const Geom& g, int nf) {
  const int spb = (64 / nf) * ((256 / 64) / NK_GROUPS);
  return (g.V + spb - 1) / spb;
}

static int check_gauge(nk_lattice* lat) {
  if (!lat->have_gauge) {
    set_error("no gauge field set on the lattice handle");
    return NK_ENOGAUGE;
  }
  return NK_OK;
}

int apply_dw_dev(nk_lattice* lat, double m_w, double mu, int g5, const C64* x, C64* y, hipStream_t st) {
  if (int e = check_gauge(lat)) return e;
  const Geom& g = lat->g;
  FieldPtrs<double, 1> in{{x}};
  FieldPtrsW<double, 1> out{{y}};
  TFac<double, 1> tf{{exp(mu)}, {exp(-mu)}};
  LinksPlain<double> lk{lat->U64.as<C64>(), g.V};
  hipLaunchKernelGGL((k_apply<double, 1, LinksPlain<double>, NK_GROUPS>), dim3(apply_blocks(g, 1)), dim3(256), 0,
                     st, g, lk, 4.0 + m_w, g5, in, out, tf);
  NK_HIP(hipGetLastError());
  return NK_OK;
}

int apply_pair_dev(nk_lattice* lat, double m_w, double mu, const C64* v, const C64* w, C64* av, C64* adw,
                   hipStream_t st) {
  if (int e = check_gauge(lat)) return e;
  const Geom& g = lat->g;
  FieldPtrs<double, 2> in{{v, w}};
  FieldPtrsW<double, 2> out{{av, adw}};
  TFac<double, 2> tf{{exp(mu), exp(-mu)}, {exp(-mu), exp(mu)}};
  LinksPlain<double> lk{lat->U64.as<C64>(), g.V};
  hipLaunchKernelGGL((k_apply<double, 2, LinksPlain<double>, NK_GROUPS>), dim3(apply_blocks(g, 2)), dim3(256), 0,
                     st, g, lk, 4.0 + m_w, 1, in, out, tf);
  NK_HIP(hipGetLastError());
  return NK_OK;
}

}  // namespace nk
