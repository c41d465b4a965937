// C ABI entry points (include/nk.h) and the host orchestration of one sign
// application: outer basis -> small problem -> lift (Eqs. (3)-(6)).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "hostbuf.h"
#include "nk_internal.h"

namespace nk {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

int hip_fail(hipError_t e, const char* what, const char* file, int line) {
  set_error("%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  return NK_EHIP;
}

int DevBuf::ensure(size_t need) {
  if (p && need <= bytes) return NK_OK;
  release();
  if (need == 0) return NK_OK;
  hipError_t e = hipMalloc(&p, need);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
    bytes = 0;
    set_error("hipMalloc of %zu bytes failed: %s", need, hipGetErrorString(e));
    return NK_ENOMEM;
  }
  bytes = need;
  return NK_OK;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

int HostBuf::ensure(size_t need) {
  if (h && need <= bytes) return NK_OK;
  release();
  if (need == 0) return NK_OK;
  hipError_t e = hipHostMalloc(&h, need, hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess) e = hipHostGetDevicePointer(&d, h, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release();
    set_error("pinned host allocation of %zu bytes failed: %s", need, hipGetErrorString(e));
    return NK_ENOMEM;
  }
  bytes = need;
  return NK_OK;
}

void HostBuf::release() {
  if (h) (void)hipHostFree(h);
  h = d = nullptr;
  bytes = 0;
}

// per-call coefficient block on the device
struct CoefBlock {
  Coefs c;
  C64* z;
  C64* z0;
  C64* xd;  // source in device layout (FP64)
  C64* yd;  // result in device layout (FP64)
};

static int coef_block(nk_lattice* lat, int k, CoefBlock& cb) {
  const size_t n = (size_t)12 * lat->g.V;
  const size_t bytes = (size_t)(3 * k + 2 * (k + 1) + 2 * k) * sizeof(C64) + (size_t)(k + 1) * sizeof(double) +
                       2 * n * sizeof(C64) + 64;
  if (lat->coef.ensure(bytes)) return NK_ENOMEM;
  char* p = lat->coef.as<char>();
  auto take = [&](size_t b) {
    char* r = p;
    p += (b + 15) & ~(size_t)15;
    return r;
  };
  cb.xd = (C64*)take(n * sizeof(C64));
  cb.yd = (C64*)take(n * sizeof(C64));
  cb.c.alpha = (C64*)take(k * sizeof(C64));
  cb.c.beta = (C64*)take(k * sizeof(C64));
  cb.c.delta = (C64*)take(k * sizeof(C64));
  cb.c.sw = (C64*)take((k + 1) * sizeof(C64));
  cb.z = (C64*)take(k * sizeof(C64));
  cb.z0 = (C64*)take(k * sizeof(C64));
  cb.c.sv = (double*)take((k + 1) * sizeof(double));
  cb.c.flags = (int*)take(4 * sizeof(int));
  return NK_OK;
}

static int validate_params(nk_lattice* lat, const nk_sign_params* p) {
  if (!lat || !p) {
    set_error("null handle or params");
    return NK_EINVAL;
  }
  if (!lat->have_gauge) {
    set_error("no gauge field set on the lattice handle");
    return NK_ENOGAUGE;
  }
  if (p->k < 1 || p->ell < 0 || p->nrhs < 1 || p->precision < 0 || p->precision > 2 || p->rh_maxit < 1 ||
      p->est_delay < 0 || p->est_delay >= p->k || !(p->tol >= 0.0) || p->two_pass < 0 || p->two_pass > 2 ||
      p->rh_scaling < 0 || p->rh_scaling > 2 || p->profile < 0 || p->block < 0 || p->block > 2 || p->inner < 0 ||
      p->inner > 1 || !std::isfinite(p->mu) || !std::isfinite(p->m_w)) {
    set_error("invalid sign parameters (k=%d ell=%d nrhs=%d precision=%d est_delay=%d)", p->k, p->ell, p->nrhs,
              p->precision, p->est_delay);
    return NK_EINVAL;
  }
  if (p->ell > p->k) {
    set_error("ell (%d) > k (%d)", p->ell, p->k);
    return NK_EINVAL;
  }
  if (p->tol > 0.0 && p->check_every < 1) {
    set_error("check_every must be >= 1 when tol > 0");
    return NK_EINVAL;
  }
  return NK_OK;
}

// the outer recurrence's status flag, read through pinned memory (one DMA
// and a synchronisation, no staging through pageable memory)
namespace {
HostBuf g_flag_pin;
}
static int read_flag(const int* dflag, hipStream_t st, int* out) {
  if (g_flag_pin.ensure(sizeof(int))) return NK_ENOMEM;
  NK_HIP(hipMemcpyAsync(g_flag_pin.h, dflag, sizeof(int), hipMemcpyDeviceToHost, st));
  NK_HIP(hipStreamSynchronize(st));
  *out = *g_flag_pin.host<int>();
  return NK_OK;
}

static double host_est(const std::vector<C64>& z1, const std::vector<C64>& z0) {
  double num = 0, den = 0;
  for (size_t i = 0; i < z1.size(); ++i) {
    C64 d = z1[i];
    if (i < z0.size()) d = d - z0[i];
    num += norm2(d);
    den += norm2(z1[i]);
  }
  return std::sqrt(num / den);
}

static int estimate(int kk, int ell, int herm, int d, const nk_sign_params* p, CoefBlock& cb, hipStream_t st,
                    double* est) {
  std::vector<C64> z1(kk), z0(kk - d);
  SmallOut so;
  int e = small_sign_dev(kk, ell, herm, cb.c.alpha, cb.c.beta, cb.c.delta, p->rh_scaling, p->rh_maxit, p->rh_tol,
                         cb.z0, &so, st, p->inner);
  if (e < 0) return e;
  NK_HIP(hipMemcpyAsync(z1.data(), cb.z0, kk * sizeof(C64), hipMemcpyDeviceToHost, st));
  NK_HIP(hipStreamSynchronize(st));
  e = small_sign_dev(kk - d, std::min(ell, kk - d), herm, cb.c.alpha, cb.c.beta, cb.c.delta, p->rh_scaling,
                     p->rh_maxit, p->rh_tol, cb.z0, &so, st, p->inner);
  if (e < 0) return e;
  NK_HIP(hipMemcpyAsync(z0.data(), cb.z0, (kk - d) * sizeof(C64), hipMemcpyDeviceToHost, st));
  NK_HIP(hipStreamSynchronize(st));
  *est = host_est(z1, z0);
  return NK_OK;
}

// one source: x, y canonical device vectors
static int sign_one(nk_lattice* lat, const nk_sign_params* p, int ell, const C64* x, C64* y, nk_sign_info* info,
                    hipStream_t st) {
  const Geom& g = lat->g;
  const int k = p->k;
  const int herm = p->mu == 0.0;
  CoefBlock cb;
  if (int e = coef_block(lat, k, cb)) return e;
  BasisPlan bp;
  bp.prec = p->precision;
  bp.hermitian = herm;
  bp.m_w = p->m_w;
  bp.mu = p->mu;
  bp.k = k;
  // store V_k unless two passes are requested or it does not fit
  const size_t vbytes = basis_vector_bytes(g, bp.prec) * (size_t)(k + 1);
  int two = 0;
  if (p->two_pass == NK_TWO_PASS_ON) {
    two = 1;
  } else {
    size_t fr = 0, tot = 0;
    NK_HIP(hipMemGetInfo(&fr, &tot));
    const size_t avail = fr + lat->vk.bytes;
    const size_t margin = (size_t)2 << 30;
    if (vbytes + margin > avail) {
      if (p->two_pass == NK_TWO_PASS_OFF) {
        set_error("V_k needs %zu bytes; %zu available and two_pass is OFF", vbytes, avail);
        return NK_ENOMEM;
      }
      two = 1;
    }
  }
  bp.store = two ? 0 : 1;
  bp.profile = p->profile;
  lat->evkind.clear();
  lat->evnext = 0;
  if (!two && lat->vk.ensure(vbytes)) return NK_ENOMEM;
  hipEvent_t ev[4];
  for (auto& e : ev) NK_HIP(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 4; ++i) (void)hipEventDestroy(e[i]);
    }
  } guard{ev};

  if (int e = pack_spinor<double>(g, x, cb.xd, st)) return e;
  NK_HIP(hipMemsetAsync(cb.c.flags, 0, 4 * sizeof(int), st));
  NK_HIP(hipEventRecord(ev[0], st));
  int kused = k;
  double est = std::numeric_limits<double>::quiet_NaN();
  int flag = 0;
  const int stride = p->tol > 0.0 ? p->check_every : k;
  for (int j0 = 0; j0 < k;) {
    const int j1 = std::min(k, j0 + stride);
    if (int e = basis_run(lat, bp, cb.xd, j0, j1, cb.c, lat->vk.p, st, nullptr)) return e;
    j0 = j1;
    if (p->tol > 0.0 && j1 < k) {
      if (int e = read_flag(cb.c.flags, st, &flag)) return e;
      if (flag) break;
      const int d = std::max(1, std::min(p->est_delay > 0 ? p->est_delay : 10, j1 - 1));
      if (j1 - d < 1) continue;
      double e1 = 0;
      if (int e = estimate(j1, ell, herm, d, p, cb, st, &e1)) return e;
      if (e1 < p->tol) {
        kused = j1;
        est = e1;
        break;
      }
    }
  }
  NK_HIP(hipEventRecord(ev[1], st));
  if (int e = read_flag(cb.c.flags, st, &flag)) return e;
  int warn = NK_OK;
  if (flag < 0) {
    set_error("source vector has zero or non-finite norm");
    return NK_EINVAL;
  }
  if (flag > 0) {
    kused = std::min(kused, flag);
    warn = NK_WARN_BREAKDOWN;
    if (info) info->breakdown_step = flag;
  }
  SmallOut so;
  int es = small_sign_dev(kused, std::min(ell, kused), herm, cb.c.alpha, cb.c.beta, cb.c.delta, p->rh_scaling,
                          p->rh_maxit, p->rh_tol, cb.z, &so, st, p->inner);
  if (es < 0) return es;
  if (es > 0 && warn == NK_OK) warn = es;
  // the estimate at the final k: requested explicitly (est_delay > 0), or
  // needed for the early-stop decision when the loop ran to k without its last
  // check (the in-loop checks skip j1 == k); the delay is the loop's
  if (std::isnan(est) && (p->est_delay > 0 || p->tol > 0.0)) {
    const int d = std::max(1, std::min(p->est_delay > 0 ? p->est_delay : 10, kused - 1));
    if (kused - d >= 1) {
      if (int e = estimate(kused, ell, herm, d, p, cb, st, &est)) return e;
    }
  }
  NK_HIP(hipEventRecord(ev[2], st));
  if (two) {
    if (int e = two_pass_lift(lat, bp, cb.xd, kused, cb.z, cb.c, cb.yd, st)) return e;
  } else {
    if (int e = lift_run(lat, bp, kused, cb.z, 0.0, cb.c, lat->vk.p, cb.yd, st)) return e;
  }
  if (int e = unpack_spinor<double>(g, cb.yd, y, st)) return e;
  NK_HIP(hipEventRecord(ev[3], st));
  NK_HIP(hipEventSynchronize(ev[3]));
  if (info) {
    info->k_used = kused;
    info->ell_used = so.ell_used;
    info->rh_iters = so.rh_iters;
    info->two_pass = two;
    info->est = est;
    info->rh_residual = so.rh_residual;
    float t0 = 0, t1 = 0, t2 = 0;
    (void)hipEventElapsedTime(&t0, ev[0], ev[1]);
    (void)hipEventElapsedTime(&t1, ev[1], ev[2]);
    (void)hipEventElapsedTime(&t2, ev[2], ev[3]);
    info->t_basis_ms = t0;
    info->t_small_ms = t1;
    info->t_lift_ms = t2;
  }
  if (bp.profile) {
    double a = 0, b = 0;
    int na = 0, nb = 0;
    if (int e = prof_collect(lat, &a, &b, &na, &nb)) return e;
    if (info) {
      info->t_stencil_ms += a;
      info->t_update_ms += b;
      info->n_stencil += na;
      info->n_update += nb;
    }
  }
  if (p->tol > 0.0 && !(est < p->tol) && warn == NK_OK) warn = NK_WARN_NOTCONV;
  return warn;
}

}  // namespace nk

nk_lattice::~nk_lattice() {
  for (auto& gr : graphs)
    if (gr.exec) (void)hipGraphExecDestroy(gr.exec);
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  U64.release();
  U32.release();
  Ubf.release();
  vk.release();
  work.release();
  coef.release();
  part.release();
  canon.release();
  lift.release();
  tmp.release();
  bvec.release();
  bsmall.release();
  defl.release();
  ovl.release();
  eig.release();
  for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
}

using namespace nk;

extern "C" {

void nk_sign_params_default(nk_sign_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->m_w = -1.0;
  p->mu = 0.0;
  p->k = 100;
  p->ell = 0;
  p->tol = 0.0;
  p->nrhs = 1;
  p->precision = NK_PREC_FP64;
  p->rh_scaling = NK_RH_NONE;
  p->two_pass = NK_TWO_PASS_AUTO;
  p->est_delay = 0;
  p->check_every = 50;
  p->rh_maxit = 100;
  p->rh_tol = 1e-13;
  p->ell_per_rhs = nullptr;
}

int nk_lattice_create(const int32_t dims[4], nk_lattice** out) {
  if (!dims || !out) {
    set_error("null argument");
    return NK_EINVAL;
  }
  long long V = 1;
  for (int i = 0; i < 4; ++i) {
    if (dims[i] < 2 || (dims[i] & 1)) {
      set_error("lattice extent %d in direction %d must be even and >= 2", dims[i], i);
      return NK_EINVAL;
    }
    V *= dims[i];
  }
  if (12 * V >= (1LL << 31)) {
    set_error("lattice too large (12 V must fit in 31 bits)");
    return NK_EINVAL;
  }
  nk_lattice* lat = new nk_lattice();
  const int d4[4] = {dims[0], dims[1], dims[2], dims[3]};
  geom_init(lat->g, d4);
  if (hipGetDevice(&lat->device) != hipSuccess) {
    (void)hipGetLastError();
    delete lat;
    set_error("no HIP device");
    return NK_EHIP;
  }
  *out = lat;
  return NK_OK;
}

int nk_lattice_destroy(nk_lattice* lat) {
  if (!lat) return NK_OK;
  (void)hipDeviceSynchronize();
  delete lat;
  return NK_OK;
}

int nk_gauge_set(nk_lattice* lat, const double* U) {
  if (!lat || !U) {
    set_error("null argument");
    return NK_EINVAL;
  }
  const size_t bytes = (size_t)36 * lat->g.V * sizeof(C64);
  if (lat->canon.ensure(bytes)) return NK_ENOMEM;
  NK_HIP(hipMemcpy(lat->canon.p, U, bytes, hipMemcpyHostToDevice));
  if (int e = pack_gauge(lat, lat->canon.as<C64>(), nullptr)) return e;
  NK_HIP(hipDeviceSynchronize());
  lat->have_gauge = true;
  return NK_OK;
}

int nk_gauge_set_device(nk_lattice* lat, const void* dU, nk_stream_t stream) {
  if (!lat || !dU) {
    set_error("null argument");
    return NK_EINVAL;
  }
  if (int e = pack_gauge(lat, (const C64*)dU, (hipStream_t)stream)) return e;
  lat->have_gauge = true;
  return NK_OK;
}

int nk_apply_dw_device(nk_lattice* lat, double m_w, double mu, int32_t gamma5, const void* x, void* y,
                       int32_t nrhs, nk_stream_t stream) {
  if (!lat || !x || !y || nrhs < 1 || x == y) {
    set_error("invalid argument to nk_apply_dw");
    return NK_EINVAL;
  }
  if (!lat->have_gauge) {
    set_error("no gauge field set on the lattice handle");
    return NK_ENOGAUGE;
  }
  const Geom& g = lat->g;
  const size_t n = (size_t)12 * g.V;
  if (lat->tmp.ensure(2 * n * sizeof(C64))) return NK_ENOMEM;
  C64* a = lat->tmp.as<C64>();
  C64* b = a + n;
  hipStream_t st = (hipStream_t)stream;
  for (int r = 0; r < nrhs; ++r) {
    if (int e = pack_spinor<double>(g, (const C64*)x + r * n, a, st)) return e;
    if (int e = apply_dw_dev(lat, m_w, mu, gamma5 ? 1 : 0, a, b, st)) return e;
    if (int e = unpack_spinor<double>(g, b, (C64*)y + r * n, st)) return e;
  }
  return NK_OK;
}

int nk_apply_dw(nk_lattice* lat, double m_w, double mu, int32_t gamma5, const double* x, double* y, int32_t nrhs) {
  if (!lat || !x || !y || nrhs < 1) {
    set_error("invalid argument to nk_apply_dw");
    return NK_EINVAL;
  }
  const size_t n = (size_t)12 * lat->g.V;
  if (lat->canon.ensure(2 * n * nrhs * sizeof(C64))) return NK_ENOMEM;
  C64* dx = lat->canon.as<C64>();
  C64* dy = dx + n * nrhs;
  NK_HIP(hipMemcpy(dx, x, n * nrhs * sizeof(C64), hipMemcpyHostToDevice));
  if (int e = nk_apply_dw_device(lat, m_w, mu, gamma5, dx, dy, nrhs, nullptr)) return e;
  NK_HIP(hipMemcpy(y, dy, n * nrhs * sizeof(C64), hipMemcpyDeviceToHost));
  return NK_OK;
}

int nk_apply_pair_device(nk_lattice* lat, double m_w, double mu, const void* v, const void* w, void* av, void* adw,
                         nk_stream_t stream) {
  if (!lat || !v || !w || !av || !adw) {
    set_error("invalid argument to nk_apply_pair_device");
    return NK_EINVAL;
  }
  if (!lat->have_gauge) {
    set_error("no gauge field set on the lattice handle");
    return NK_ENOGAUGE;
  }
  const Geom& g = lat->g;
  const size_t n = (size_t)12 * g.V;
  if (lat->tmp.ensure(4 * n * sizeof(C64))) return NK_ENOMEM;
  C64* t = lat->tmp.as<C64>();
  hipStream_t st = (hipStream_t)stream;
  if (int e = pack_spinor<double>(g, (const C64*)v, t, st)) return e;
  if (int e = pack_spinor<double>(g, (const C64*)w, t + n, st)) return e;
  if (int e = apply_pair_dev(lat, m_w, mu, t, t + n, t + 2 * n, t + 3 * n, st)) return e;
  if (int e = unpack_spinor<double>(g, t + 2 * n, (C64*)av, st)) return e;
  if (int e = unpack_spinor<double>(g, t + 3 * n, (C64*)adw, st)) return e;
  return NK_OK;
}

int nk_spinor_pack_device(nk_lattice* lat, const void* x, void* xp, int32_t nrhs, nk_stream_t stream) {
  if (!lat || !x || !xp || nrhs < 1 || x == xp) {
    set_error("invalid argument to nk_spinor_pack_device");
    return NK_EINVAL;
  }
  const size_t n = (size_t)12 * lat->g.V;
  for (int r = 0; r < nrhs; ++r)
    if (int e = pack_spinor<double>(lat->g, (const C64*)x + r * n, (C64*)xp + r * n, (hipStream_t)stream)) return e;
  return NK_OK;
}

int nk_spinor_unpack_device(nk_lattice* lat, const void* xp, void* x, int32_t nrhs, nk_stream_t stream) {
  if (!lat || !x || !xp || nrhs < 1 || x == xp) {
    set_error("invalid argument to nk_spinor_unpack_device");
    return NK_EINVAL;
  }
  const size_t n = (size_t)12 * lat->g.V;
  for (int r = 0; r < nrhs; ++r)
    if (int e = unpack_spinor<double>(lat->g, (const C64*)xp + r * n, (C64*)x + r * n, (hipStream_t)stream)) return e;
  return NK_OK;
}

int nk_apply_dw_packed_device(nk_lattice* lat, double m_w, double mu, int32_t gamma5, const void* xp, void* yp,
                              nk_stream_t stream) {
  if (!lat || !xp || !yp || xp == yp) {
    set_error("invalid argument to nk_apply_dw_packed_device");
    return NK_EINVAL;
  }
  return apply_dw_dev(lat, m_w, mu, gamma5 ? 1 : 0, (const C64*)xp, (C64*)yp, (hipStream_t)stream);
}

int nk_apply_pair_packed_device(nk_lattice* lat, double m_w, double mu, const void* vp, const void* wp, void* avp,
                                void* adwp, nk_stream_t stream) {
  if (!lat || !vp || !wp || !avp || !adwp || avp == adwp || avp == vp || avp == wp || adwp == vp || adwp == wp) {
    set_error("invalid argument to nk_apply_pair_packed_device");
    return NK_EINVAL;
  }
  return apply_pair_dev(lat, m_w, mu, (const C64*)vp, (const C64*)wp, (C64*)avp, (C64*)adwp, (hipStream_t)stream);
}

int nk_krylov_basis_device(nk_lattice* lat, const nk_sign_params* p, const void* x, double* alpha, double* beta,
                           double* delta, nk_sign_info* info, nk_stream_t stream) {
  if (int e = validate_params(lat, p)) return e;
  if (!x || !alpha || !beta || !delta) {
    set_error("null argument");
    return NK_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  const int k = p->k;
  CoefBlock cb;
  if (int e = coef_block(lat, k, cb)) return e;
  BasisPlan bp{p->precision, p->mu == 0.0 ? 1 : 0, p->m_w, p->mu, k, 0, 0};
  if (int e = pack_spinor<double>(lat->g, (const C64*)x, cb.xd, st)) return e;
  NK_HIP(hipMemsetAsync(cb.c.flags, 0, 4 * sizeof(int), st));
  NK_HIP(hipMemsetAsync(cb.c.alpha, 0, 3 * k * sizeof(C64), st));
  if (int e = basis_run(lat, bp, cb.xd, 0, k, cb.c, nullptr, st, nullptr)) return e;
  int flag = 0;
  NK_HIP(hipMemcpyAsync(&flag, cb.c.flags, sizeof(int), hipMemcpyDeviceToHost, st));
  NK_HIP(hipMemcpyAsync(alpha, cb.c.alpha, k * sizeof(C64), hipMemcpyDeviceToHost, st));
  NK_HIP(hipMemcpyAsync(beta, cb.c.beta, k * sizeof(C64), hipMemcpyDeviceToHost, st));
  NK_HIP(hipMemcpyAsync(delta, cb.c.delta, k * sizeof(C64), hipMemcpyDeviceToHost, st));
  NK_HIP(hipStreamSynchronize(st));
  if (flag < 0) {
    set_error("source vector has zero or non-finite norm");
    return NK_EINVAL;
  }
  const int kused = flag > 0 ? flag : k;
  // entries past k_used (and the last off-diagonal) are zero
  for (int j = kused; j < k; ++j) alpha[2 * j] = alpha[2 * j + 1] = 0.0;
  for (int j = kused - 1; j < k; ++j) beta[2 * j] = beta[2 * j + 1] = delta[2 * j] = delta[2 * j + 1] = 0.0;
  if (info) {
    std::memset(info, 0, sizeof *info);
    info->k_used = kused;
    info->breakdown_step = flag;
    info->est = std::numeric_limits<double>::quiet_NaN();
  }
  return flag > 0 ? NK_WARN_BREAKDOWN : NK_OK;
}

int nk_small_sign(int32_t k, int32_t ell, int32_t hermitian, const double* alpha, const double* beta,
                  const double* delta, const nk_sign_params* p, double* z, nk_sign_info* info) {
  if (k < 1 || ell < 0 || ell > k || !alpha || !beta || !delta || !z) {
    set_error("invalid argument to nk_small_sign");
    return NK_EINVAL;
  }
  nk_sign_params dp;
  nk_sign_params_default(&dp);
  if (!p) p = &dp;
  ScopedBuf buf;
  if (buf.ensure((size_t)4 * k * sizeof(C64))) return NK_ENOMEM;
  C64* a = buf.as<C64>();
  NK_HIP(hipMemcpy(a, alpha, k * sizeof(C64), hipMemcpyHostToDevice));
  NK_HIP(hipMemcpy(a + k, beta, k * sizeof(C64), hipMemcpyHostToDevice));
  NK_HIP(hipMemcpy(a + 2 * k, delta, k * sizeof(C64), hipMemcpyHostToDevice));
  SmallOut so;
  if (p->inner < 0 || p->inner > 1) {
    set_error("invalid inner basis %d", p->inner);
    return NK_EINVAL;
  }
  int e = small_sign_dev(k, ell, hermitian, a, a + k, a + 2 * k, p->rh_scaling, p->rh_maxit, p->rh_tol, a + 3 * k,
                         &so, nullptr, p->inner);
  if (e < 0) return e;
  NK_HIP(hipMemcpy(z, a + 3 * k, k * sizeof(C64), hipMemcpyDeviceToHost));
  if (info) {
    std::memset(info, 0, sizeof *info);
    info->k_used = k;
    info->ell_used = so.ell_used;
    info->rh_iters = so.rh_iters;
    info->rh_residual = so.rh_residual;
    info->est = std::numeric_limits<double>::quiet_NaN();
  }
  return e;
}

int nk_inner_matrix(int32_t k, int32_t ell, int32_t hermitian, const double* alpha, const double* beta,
                    const double* delta, double* a, double* b, double* d, int32_t* ell_used) {
  if (k < 1 || ell < 1 || ell > k || !alpha || !beta || !delta || !a || !b || !d || !ell_used) {
    set_error("invalid argument to nk_inner_matrix");
    return NK_EINVAL;
  }
  ScopedBuf buf;
  if (buf.ensure((size_t)4 * k * sizeof(C64))) return NK_ENOMEM;
  C64* c = buf.as<C64>();
  NK_HIP(hipMemcpy(c, alpha, k * sizeof(C64), hipMemcpyHostToDevice));
  NK_HIP(hipMemcpy(c + k, beta, k * sizeof(C64), hipMemcpyHostToDevice));
  NK_HIP(hipMemcpy(c + 2 * k, delta, k * sizeof(C64), hipMemcpyHostToDevice));
  std::vector<C64> hl((size_t)3 * ell);
  SmallOut so;
  so.hl_host = hl.data();
  so.inner_only = true;
  const int e = small_sign_dev(k, ell, hermitian, c, c + k, c + 2 * k, NK_RH_NONE, 1, 0.0, c + 3 * k, &so, nullptr);
  if (e < 0) return e;
  const int lu = so.ell_used;
  std::memset(a, 0, 2 * sizeof(double) * ell);
  std::memset(b, 0, 2 * sizeof(double) * ell);
  std::memset(d, 0, 2 * sizeof(double) * ell);
  std::memcpy(a, hl.data(), lu * sizeof(C64));
  std::memcpy(b, hl.data() + lu, lu * sizeof(C64));
  std::memcpy(d, hl.data() + 2 * lu, lu * sizeof(C64));
  *ell_used = lu;
  return e;
}

int nk_stencil_groups(nk_lattice* lat, int32_t precision, int32_t hermitian) {
  if (!lat || precision < 0 || precision > 2) {
    set_error("invalid argument to nk_stencil_groups");
    return NK_EINVAL;
  }
  return lat->k1_groups[hermitian ? 1 : 0][precision];
}

int nk_rh_model_set(const float* params) { return nk::mlp_model_set(params); }

int nk_rh_newton_schulz(int32_t enable) { return nk::rh_newton_schulz(enable); }

int nk_block_group(nk_lattice* lat, int32_t set) {
  if (!lat || !(set == 0 || set == 1 || set == 2 || set == 4)) {
    set_error("nk_block_group: a handle and set in {0, 1, 2, 4}");
    return NK_EINVAL;
  }
  const int cur = lat->blk_group[1] ? lat->blk_group[1] : lat->blk_group[0];
  if (set) lat->blk_group[0] = lat->blk_group[1] = set;
  return cur;
}

int nk_rh_tile_force(int32_t rows_per_thread, int32_t panel_threads, int32_t update_tile) {
  return nk::rh_tile_force(rows_per_thread, panel_threads, update_tile);
}

int nk_rh_tile_choice(int32_t n, int32_t batch, int32_t shape[4]) {
  if (n < 1 || batch < 1 || !shape) {
    set_error("invalid argument to nk_rh_tile_choice");
    return NK_EINVAL;
  }
  int nb = 0, rm = 0, pth = 0, tile = 0;
  const int have = nk::rh_tile_choice(n, batch, &nb, &rm, &pth, &tile);
  shape[0] = nb;
  shape[1] = rm;
  shape[2] = pth;
  shape[3] = tile;
  return have;
}

int nk_rh_features_device(int32_t batch, int32_t ld, const int32_t* n, const void* S, float* feat,
                          nk_stream_t stream) {
  if (batch < 1 || ld < 1 || !n || !S || !feat) {
    set_error("invalid argument to nk_rh_features_device");
    return NK_EINVAL;
  }
  for (int b = 0; b < batch; ++b)
    if (n[b] < 1 || n[b] > ld) {
      set_error("matrix %d has size %d outside [1, ld=%d]", b, n[b], ld);
      return NK_EINVAL;
    }
  ScopedBuf nb;
  if (nb.ensure((size_t)batch * sizeof(int))) return NK_ENOMEM;
  NK_HIP(hipMemcpyAsync(nb.p, n, batch * sizeof(int), hipMemcpyHostToDevice, stream));
  if (int e = mlp_features(batch, ld, nb.as<int>(), (const C64*)S, feat, stream)) return e;
  NK_HIP(hipStreamSynchronize(stream));  // nb is released on return
  return NK_OK;
}

int nk_mlp_forward_device(int32_t batch, const float* params, const float* feat, float* y, float* act,
                          nk_stream_t stream) {
  if (batch < 0 || !params || (batch > 0 && (!feat || !y))) {
    set_error("invalid argument to nk_mlp_forward_device");
    return NK_EINVAL;
  }
  return mlp_forward(batch, params, feat, y, act, stream);
}

int nk_rh_spectral_loss_device(int32_t batch, const int32_t* off, const void* lam, const float* y, float gscale,
                               float* loss, float* dy, nk_stream_t stream) {
  if (batch < 0 || (batch > 0 && (!off || !lam || !y || !loss || !dy))) {
    set_error("invalid argument to nk_rh_spectral_loss_device");
    return NK_EINVAL;
  }
  return mlp_spectral_loss(batch, off, (const C64*)lam, y, gscale, loss, dy, stream);
}

int nk_mlp_backward_device(int32_t batch, const float* params, const float* feat, const float* act,
                           const float* dy, float* delta, float* grad, nk_stream_t stream) {
  if (batch < 0 || !params || !grad || (batch > 0 && (!feat || !act || !dy || !delta))) {
    set_error("invalid argument to nk_mlp_backward_device");
    return NK_EINVAL;
  }
  return mlp_backward(batch, params, feat, act, dy, delta, grad, stream);
}

int nk_adam_step_device(int32_t n, float* params, const float* grad, float* m, float* v, int32_t t, float lr,
                        float beta1, float beta2, float eps, nk_stream_t stream) {
  if (n < 0 || t < 1 || (n > 0 && (!params || !grad || !m || !v))) {
    set_error("invalid argument to nk_adam_step_device");
    return NK_EINVAL;
  }
  if (n == 0) return NK_OK;
  return mlp_adam(n, params, grad, m, v, t, lr, beta1, beta2, eps, stream);
}

int nk_rh_sign(int32_t batch, int32_t ld, const int32_t* n, double* S, int32_t scaling, int32_t maxit, double tol,
               int32_t* iters) {
  if (batch < 1 || ld < 1 || !n || !S || !iters || maxit < 1 || scaling < 0 || scaling > 2) {
    set_error("invalid argument to nk_rh_sign");
    return NK_EINVAL;
  }
  for (int b = 0; b < batch; ++b)
    if (n[b] < 0 || n[b] > ld) {
      set_error("matrix %d has size %d outside [0, ld=%d]", b, n[b], ld);
      return NK_EINVAL;
    }
  ScopedBuf buf;
  const size_t bytes = (size_t)batch * ld * ld * sizeof(C64);
  if (buf.ensure(bytes)) return NK_ENOMEM;
  NK_HIP(hipMemcpy(buf.p, S, bytes, hipMemcpyHostToDevice));
  int e = rh_sign_batched(batch, ld, n, buf.as<C64>(), scaling, maxit, tol, iters, nullptr, nullptr);
  if (e < 0) return e;
  NK_HIP(hipMemcpy(S, buf.p, bytes, hipMemcpyDeviceToHost));
  return e;
}

int nk_sign_apply_device(nk_lattice* lat, const nk_sign_params* p, const void* x, void* y, nk_sign_info* info,
                         nk_stream_t stream) {
  if (int e = validate_params(lat, p)) return e;
  if (!x || !y || x == y) {
    set_error("invalid source/result pointers");
    return NK_EINVAL;
  }
  if (info) {
    std::memset(info, 0, sizeof *info);
    info->est = std::numeric_limits<double>::quiet_NaN();
  }
  const size_t n = (size_t)12 * lat->g.V;
  for (int r = 0; r < p->nrhs; ++r) {
    const int ell = p->ell_per_rhs ? p->ell_per_rhs[r] : p->ell;
    if (ell < 0 || ell > p->k) {
      set_error("ell_per_rhs[%d] = %d outside [0, k]", r, ell);
      return NK_EINVAL;
    }
  }
  if (p->block && p->nrhs > 1) {
    const int e = block_sign(lat, p, (const C64*)x, (C64*)y, info, (hipStream_t)stream);
    if (e != 1) return e;  // 1: not a case the block path covers; run the sources one after another
  }
  int worst = NK_OK;
  for (int r = 0; r < p->nrhs; ++r) {
    const int ell = p->ell_per_rhs ? p->ell_per_rhs[r] : p->ell;
    int e = sign_one(lat, p, ell, (const C64*)x + r * n, (C64*)y + r * n, info, (hipStream_t)stream);
    if (e < 0) return e;
    if (e > worst) worst = e;
  }
  return worst;
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

int nk_sign_apply_deflated_device(nk_lattice* lat, const nk_sign_params* p, int32_t m, const double* lam,
                                  const void* R, const void* L, const void* x, void* y, nk_sign_info* info,
                                  nk_stream_t stream) {
  if (int e = validate_params(lat, p)) return e;
  if (m < 0 || m > NK_DEFL_MAX) {
    set_error("m = %d deflated eigenpairs outside [0, %d]", m, NK_DEFL_MAX);
    return NK_EINVAL;
  }
  if (m == 0) return nk_sign_apply_device(lat, p, x, y, info, stream);
  const size_t n = (size_t)12 * lat->g.V;
  const size_t vb = (size_t)p->nrhs * n * sizeof(C64), cb = (size_t)m * n * sizeof(C64);
  if (!lam || !R || !L || !x || !y || overlaps(y, vb, x, vb) || overlaps(y, vb, R, cb) || overlaps(y, vb, L, cb)) {
    set_error("invalid deflation arguments (NULL, or y overlapping x, R or L)");
    return NK_EINVAL;
  }
  DeflSigns neg{};
  for (int i = 0; i < m; ++i) {
    const double re = lam[2 * i], im = lam[2 * i + 1];
    if (!std::isfinite(re) || !std::isfinite(im) || re == 0.0) {
      set_error("eigenvalue %d = (%g, %g): sgn needs a finite value off the imaginary axis", i, re, im);
      return NK_EINVAL;
    }
    if (re < 0.0) neg.w[i >> 6] |= 1ull << (i & 63);
  }
  for (int r = 0; r < p->nrhs; ++r) {
    const int ell = p->ell_per_rhs ? p->ell_per_rhs[r] : p->ell;
    if (ell < 0 || ell > p->k) {
      set_error("ell_per_rhs[%d] = %d outside [0, k]", r, ell);
      return NK_EINVAL;
    }
  }
  hipStream_t st = (hipStream_t)stream;
  const int nb = defl_partials(n);
  const size_t npart = (size_t)m * nb, nc = (size_t)p->nrhs * (m + 1);
  if (lat->defl.ensure((npart + nc + (size_t)p->nrhs * n) * sizeof(C64))) return NK_ENOMEM;
  C64* part = lat->defl.as<C64>();
  C64* c = part + npart;         // [nrhs][m] projections, then [nrhs] squared norms
  C64* nrm = c + (size_t)p->nrhs * m;
  C64* xp = nrm + p->nrhs;       // [nrhs][n] projected sources
  const C64* Rd = (const C64*)R;
  const C64* Ld = (const C64*)L;
  for (int r = 0; r < p->nrhs; ++r) {
    const C64* xr = (const C64*)x + r * n;
    C64* xpr = xp + r * n;
    if (int e = defl_dots(Ld, m, n, xr, part, c + (size_t)r * m, st)) return e;
    if (int e = defl_combine(Rd, m, n, c + (size_t)r * m, neg, 0, xr, xpr, st)) return e;
    if (int e = defl_dots(xpr, 1, n, xpr, part, nrm + r, st)) return e;
  }
  std::vector<C64> hn(p->nrhs);
  NK_HIP(hipMemcpyAsync(hn.data(), nrm, p->nrhs * sizeof(C64), hipMemcpyDeviceToHost, st));
  NK_HIP(hipStreamSynchronize(st));
  bool all = true;
  for (int r = 0; r < p->nrhs; ++r) {
    if (!std::isfinite(hn[r].re)) {
      set_error("source %d is not finite", r);
      return NK_EINVAL;
    }
    all = all && hn[r].re > 0.0;
  }
  if (info) {
    std::memset(info, 0, sizeof *info);
    info->est = std::numeric_limits<double>::quiet_NaN();
  }
  int worst = NK_OK;
  if (all) {
    worst = nk_sign_apply_device(lat, p, xp, y, info, stream);
    if (worst < 0) return worst;
  } else {
    for (int r = 0; r < p->nrhs; ++r) {
      C64* yr = (C64*)y + r * n;
      if (!(hn[r].re > 0.0)) {
        NK_HIP(hipMemsetAsync(yr, 0, n * sizeof(C64), st));
        continue;
      }
      nk_sign_params q = *p;
      q.nrhs = 1;
      q.ell = p->ell_per_rhs ? p->ell_per_rhs[r] : p->ell;
      q.ell_per_rhs = nullptr;
      const int e = nk_sign_apply_device(lat, &q, xp + r * n, yr, info, stream);
      if (e < 0) return e;
      if (e > worst) worst = e;
    }
  }
  for (int r = 0; r < p->nrhs; ++r)
    if (int e = defl_combine(Rd, m, n, c + (size_t)r * m, neg, 1, nullptr, (C64*)y + r * n, st)) return e;
  NK_HIP(hipStreamSynchronize(st));
  return worst;
}

static int ov_defl(const nk_lattice* lat, int32_t m, const double* lam, const void* R, const void* L, const void* y,
                   size_t ybytes, OvDefl* d) {
  if (m < 0 || m > NK_DEFL_MAX || (m > 0 && (!lam || !R || !L))) {
    set_error("invalid deflation arguments: m = %d, lam/R/L must be given for m > 0", m);
    return NK_EINVAL;
  }
  const size_t cb = (size_t)m * 12 * lat->g.V * sizeof(C64);
  if (m > 0 && (overlaps(y, ybytes, R, cb) || overlaps(y, ybytes, L, cb))) {
    set_error("the result overlaps R or L");
    return NK_EINVAL;
  }
  d->m = m;
  d->lam = lam;
  d->R = R;
  d->L = L;
  return NK_OK;
}

int nk_overlap_apply_device(nk_lattice* lat, const nk_sign_params* p, int32_t dagger, int32_t m, const double* lam,
                            const void* R, const void* L, const void* x, void* y, nk_sign_info* info,
                            nk_stream_t stream) {
  if (int e = validate_params(lat, p)) return e;
  const size_t n = (size_t)12 * lat->g.V * p->nrhs;
  if (!x || !y || overlaps(x, n * sizeof(C64), y, n * sizeof(C64)) || (dagger != 0 && dagger != 1)) {
    set_error("invalid overlap arguments (NULL, overlapping x and y, or dagger not 0/1)");
    return NK_EINVAL;
  }
  OvDefl d;
  if (int e = ov_defl(lat, m, lam, R, L, y, n * sizeof(C64), &d)) return e;
  if (lat->ovl.ensure(n * sizeof(C64))) return NK_ENOMEM;
  if (info) {
    std::memset(info, 0, sizeof *info);
    info->est = std::numeric_limits<double>::quiet_NaN();
  }
  return overlap_apply(lat, p, dagger, d, (const C64*)x, (C64*)y, lat->ovl.as<C64>(), info, (hipStream_t)stream);
}

int nk_overlap_solve_device(nk_lattice* lat, const nk_sign_params* p, int32_t m, const double* lam, const void* R,
                            const void* L, double tol, int32_t maxit, const void* b, void* y, int32_t* iters,
                            double* resid, nk_stream_t stream) {
  if (int e = validate_params(lat, p)) return e;
  const size_t n = (size_t)12 * lat->g.V;
  if (p->nrhs != 1 || !(tol > 0.0) || !std::isfinite(tol) || maxit < 1 || !b || !y || !iters || !resid ||
      overlaps(b, n * sizeof(C64), y, n * sizeof(C64))) {
    set_error("invalid overlap-solve arguments (nrhs must be 1, tol > 0, maxit >= 1, b and y apart)");
    return NK_EINVAL;
  }
  OvDefl d;
  if (int e = ov_defl(lat, m, lam, R, L, y, n * sizeof(C64), &d)) return e;
  int it = 0;
  double res = 0.0;
  const int e = overlap_solve(lat, p, d, tol, maxit, (const C64*)b, (C64*)y, &it, &res, (hipStream_t)stream);
  *iters = it;
  *resid = res;
  return e;
}

int nk_eig_hermitian_device(nk_lattice* lat, double m_w, int32_t m, int32_t p, int32_t degree, double tol,
                            int32_t maxit, const void* V0, double* lam, void* R, int32_t* passes, double* resid,
                            nk_stream_t stream) {
  if (!lat) {
    set_error("NULL lattice handle");
    return NK_EINVAL;
  }
  if (!lat->have_gauge) {
    set_error("no gauge field set");
    return NK_ENOGAUGE;
  }
  const size_t n = (size_t)12 * lat->g.V;
  if (m < 1 || p < m || p > 128 || (size_t)p > n || degree < 1 || degree > 1000 || !(tol > 0.0) ||
      !std::isfinite(tol) || maxit < 1 || !std::isfinite(m_w) || !V0 || !lam || !R || !passes || !resid ||
      overlaps(V0, (size_t)p * n * sizeof(C64), R, (size_t)m * n * sizeof(C64))) {
    set_error("invalid eigensolver arguments (1 <= m <= p <= 128, 1 <= degree <= 1000, tol > 0, maxit >= 1, "
              "V0 and R apart)");
    return NK_EINVAL;
  }
  int it = 0;
  double res = 0.0;
  const int e = eig_hermitian(lat, m_w, m, p, degree, tol, maxit, (const C64*)V0, lam, (C64*)R, &it, &res,
                              (hipStream_t)stream);
  *passes = it;
  *resid = res;
  return e;
}

int nk_eig_critical_device(nk_lattice* lat, double m_w, double mu, int32_t m, int32_t p, int32_t degree, double tol,
                           int32_t maxit, const void* V0, double* lam, void* R, void* L, int32_t* passes,
                           double* resid, nk_stream_t stream) {
  if (!lat) {
    set_error("NULL lattice handle");
    return NK_EINVAL;
  }
  if (!lat->have_gauge) {
    set_error("no gauge field set");
    return NK_ENOGAUGE;
  }
  const size_t n = (size_t)12 * lat->g.V;
  const size_t vb = (size_t)p * n * sizeof(C64), rb = (size_t)m * n * sizeof(C64);
  if (m < 1 || p < m || p > 128 || (size_t)p > n || degree < 1 || degree > 1000 || !(tol > 0.0) ||
      !std::isfinite(tol) || maxit < 1 || !std::isfinite(m_w) || !std::isfinite(mu) || !V0 || !lam || !R || !L ||
      !passes || !resid || overlaps(V0, vb, R, rb) || overlaps(V0, vb, L, rb) || overlaps(R, rb, L, rb)) {
    set_error("invalid eigensolver arguments (1 <= m <= p <= 128, 1 <= degree <= 1000, tol > 0, maxit >= 1, "
              "V0, R and L apart)");
    return NK_EINVAL;
  }
  int it = 0;
  double res = 0.0;
  const int e = eig_critical(lat, m_w, mu, m, p, degree, tol, maxit, (const C64*)V0, lam, (C64*)R, (C64*)L, &it,
                             &res, (hipStream_t)stream);
  *passes = it;
  *resid = res;
  return e;
}

int nk_sign_apply(nk_lattice* lat, const nk_sign_params* p, const double* x, double* y, nk_sign_info* info) {
  if (int e = validate_params(lat, p)) return e;
  if (!x || !y) {
    set_error("null argument");
    return NK_EINVAL;
  }
  const size_t n = (size_t)12 * lat->g.V * p->nrhs;
  ScopedBuf io;
  if (io.ensure(2 * n * sizeof(C64))) return NK_ENOMEM;
  C64* dx = io.as<C64>();
  C64* dy = dx + n;
  NK_HIP(hipMemcpy(dx, x, n * sizeof(C64), hipMemcpyHostToDevice));
  int e = nk_sign_apply_device(lat, p, dx, dy, info, nullptr);
  if (e < 0) return e;
  NK_HIP(hipMemcpy(y, dy, n * sizeof(C64), hipMemcpyDeviceToHost));
  return e;
}

const char* nk_last_error(void) { return g_err.c_str(); }

const char* nk_version(void) { return "nk 0.1.0 (gfx950)"; }

}  // extern "C"
