// nk_apply_dw_noalloc_device: the operator of Sec. 1 on canonical device
// vectors, as nk_apply_dw_device computes it, with its two layout
// temporaries in a fixed device array instead of the handle's allocation.
// For callers that cannot allocate device memory (HIP graph capture, tight
// serving loops).
#include <mutex>

#include "nk_internal.h"

namespace nk {

// two packed FP64 spinor fields of at most NK_NOALLOC_MAX_SITES sites: the
// packed source and the packed result.  Each device the library runs on
// holds its own copy until the process ends.
constexpr size_t kScratchElems = (size_t)2 * 12 * NK_NOALLOC_MAX_SITES;
static __device__ __align__(256) C64 scratch[kScratchElems];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// the device address of `scratch` on the current device, looked up once per
// device (the host-side name of the array is not a device address)
static int scratch_ptr(C64** out) {
  int dev = 0;
  NK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device ordinal %d out of range for the fixed workspace", dev);
    return NK_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    NK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("hipGetSymbolAddress returned a null address for the fixed workspace");
      return NK_EHIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<C64*>(g_scratch_ptr[dev]);
  return NK_OK;
}

}  // namespace nk

using namespace nk;

extern "C" int nk_apply_dw_noalloc_device(nk_lattice* lat, double m_w, double mu, int32_t gamma5, const void* x,
                                          void* y, int32_t nrhs, nk_stream_t stream) {
  if (!lat || !x || !y || nrhs < 1 || x == y) {
    set_error("invalid argument to nk_apply_dw_noalloc_device");
    return NK_EINVAL;
  }
  if (!lat->have_gauge) {
    set_error("no gauge field set on the lattice handle");
    return NK_ENOGAUGE;
  }
  const Geom& g = lat->g;
  if (g.V > NK_NOALLOC_MAX_SITES) {
    set_error("nk_apply_dw_noalloc_device: %d sites exceed the fixed workspace of %d sites", g.V,
              NK_NOALLOC_MAX_SITES);
    return NK_EINVAL;
  }
  C64* a = nullptr;
  if (int e = scratch_ptr(&a)) return e;
  const size_t n = (size_t)12 * g.V;
  C64* b = a + (size_t)12 * NK_NOALLOC_MAX_SITES;
  hipStream_t st = (hipStream_t)stream;
  // pack writes every entry of a, the stencil every entry of b: nothing from
  // an earlier call is read, so nothing needs clearing
  for (int r = 0; r < nrhs; ++r) {
    if (int e = pack_spinor<double>(g, (const C64*)x + r * n, a, st)) return e;
    if (int e = apply_dw_dev(lat, m_w, mu, gamma5 ? 1 : 0, a, b, st)) return e;
    if (int e = unpack_spinor<double>(g, b, (C64*)y + r * n, st)) return e;
  }
  return NK_OK;
}
