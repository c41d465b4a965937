// Stand-alone applications of gamma5 Dw(mu): the single operator and the
// fused pair (A v, A^dag w) of two-sided Lanczos (A^dag = A(-mu)).
#include "stencil.h"

namespace nk {

// y_f = [gamma5] ((4 + m_w) x_f - 1/2 hop(x_f)) for NF fields, device layout.
template <class R, int NF, class LK>
__global__ void __launch_bounds__(256) k_apply(Geom g, LK lk, R diag, int g5, FieldPtrs<R, NF> in,
                                                FieldPtrsW<R, NF> out, TFac<R, NF> tf) {
  const int s = xcd_block() * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  Cx<R> acc[NF][12];
  hopping<R, NF>(g, s, lk, in.p, tf.f, tf.b, acc);
#pragma unroll
  for (int f = 0; f < NF; ++f) {
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      Cx<R> psi = in.p[f][(size_t)c * g.V + s];
      Cx<R> o = diag * psi - R(0.5) * acc[f][c];
      if (g5 && c >= 6) o = mk<R>(-o.re, -o.im);
      out.p[f][(size_t)c * g.V + s] = o;
    }
  }
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
  hipLaunchKernelGGL((k_apply<double, 1, LinksPlain<double>>), dim3((g.V + 255) / 256), dim3(256), 0, st, g, lk,
                     4.0 + m_w, g5, in, out, tf);
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
  hipLaunchKernelGGL((k_apply<double, 2, LinksPlain<double>>), dim3((g.V + 255) / 256), dim3(256), 0, st, g, lk,
                     4.0 + m_w, 1, in, out, tf);
  NK_HIP(hipGetLastError());
  return NK_OK;
}

// generic entry used by the precision variants and the benchmark paths
template <class R, class LK>
int apply_g5dw_prec(const Geom& g, const LK& lk, double m_w, double mu, const Cx<R>* x, Cx<R>* y,
                    hipStream_t st) {
  FieldPtrs<R, 1> in{{x}};
  FieldPtrsW<R, 1> out{{y}};
  TFac<R, 1> tf{{(R)exp(mu)}, {(R)exp(-mu)}};
  hipLaunchKernelGGL((k_apply<R, 1, LK>), dim3((g.V + 255) / 256), dim3(256), 0, st, g, lk, (R)(4.0 + m_w), 1,
                     in, out, tf);
  NK_HIP(hipGetLastError());
  return NK_OK;
}

int apply_g5dw_any(nk_lattice* lat, int prec, double m_w, double mu, const void* x, void* y, hipStream_t st) {
  if (int e = check_gauge(lat)) return e;
  const Geom& g = lat->g;
  if (prec == NK_PREC_FP64)
    return apply_g5dw_prec<double>(g, LinksPlain<double>{lat->U64.as<C64>(), g.V}, m_w, mu, (const C64*)x,
                                   (C64*)y, st);
  if (prec == NK_PREC_FP32)
    return apply_g5dw_prec<float>(g, LinksPlain<float>{lat->U32.as<C32>(), g.V}, m_w, mu, (const C32*)x,
                                  (C32*)y, st);
  return apply_g5dw_prec<float>(g, LinksBF16{lat->Ubf.as<uint32_t>(), g.V}, m_w, mu, (const C32*)x, (C32*)y,
                                st);
}

}  // namespace nk
