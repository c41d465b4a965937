// Canonical (site-major) <-> device (component-major) layouts.
#include "nk_internal.h"

namespace nk {

__device__ __forceinline__ uint32_t f2bf16(float f) {
  // round to nearest even
  uint32_t b = __float_as_uint(f);
  b += 0x7fffu + ((b >> 16) & 1u);
  return b >> 16;
}

// device index of canonical site s
__device__ __forceinline__ int dev_site(const Geom& g, int s) {
  const int x = s % g.L[0];
  int r = s / g.L[0];
  const int y = r % g.L[1];
  r /= g.L[1];
  const int z = r % g.L[2];
  const int t = r / g.L[2];
  return tiled_index(g, x, y, z, t);
}

// canonical U[site][nu][a][b] -> the three device link layouts (FP64, FP32
// in entry pairs, BF16 rows 0 and 1 as 4 + 2 packed words)
__global__ void k_pack_gauge(Geom g, const C64* __restrict__ canon, C64* __restrict__ u64, C32* __restrict__ u32,
                             uint32_t* __restrict__ ubf) {
  const int V = g.V;
  const int sc = blockIdx.x * blockDim.x + threadIdx.x;
  if (sc >= V) return;
  const int s = dev_site(g, sc);
  for (int nu = 0; nu < 4; ++nu) {
    for (int e = 0; e < 9; ++e) {
      C64 v = canon[(size_t)sc * 36 + nu * 9 + e];
      u64[(size_t)(nu * 9 + e) * V + s] = v;
      u32[((size_t)(nu * 5 + e / 2) * V + s) * 2 + (e & 1)] = narrow<float>(v);
      const uint32_t w = f2bf16((float)v.re) | (f2bf16((float)v.im) << 16);
      if (e < 4) ubf[((size_t)nu * V + s) * 4 + e] = w;
      else if (e < 6) ubf[(size_t)16 * V + ((size_t)nu * V + s) * 2 + (e - 4)] = w;
    }
    u32[((size_t)(nu * 5 + 4) * V + s) * 2 + 1] = mk(0.f, 0.f);  // unused half of entry 8's pair
  }
}

template <class R>
__global__ void k_pack_spinor(Geom g, const C64* __restrict__ canon, Cx<R>* __restrict__ dev) {
  const int sc = blockIdx.x * blockDim.x + threadIdx.x;
  if (sc >= g.V) return;
  const int s = dev_site(g, sc);
#pragma unroll
  for (int c = 0; c < 12; ++c) dev[sidx<R>(g.V, c, s)] = narrow<R>(canon[(size_t)sc * 12 + c]);
}

template <class R>
__global__ void k_unpack_spinor(Geom g, const Cx<R>* __restrict__ dev, C64* __restrict__ canon) {
  const int sc = blockIdx.x * blockDim.x + threadIdx.x;
  if (sc >= g.V) return;
  const int s = dev_site(g, sc);
#pragma unroll
  for (int c = 0; c < 12; ++c) canon[(size_t)sc * 12 + c] = widen(dev[sidx<R>(g.V, c, s)]);
}

void geom_init(Geom& g, const int dims[4]) {
  int st = 1;
  g.V = 1;
  for (int d = 0; d < 4; ++d) {
    g.L[d] = dims[d];
    g.stride[d] = st;
    st *= dims[d];
    g.V *= dims[d];
    // tiles of 16 x 4 x 4 x 4 sites where the extents allow (x first: 16,
    // else 8, 4 or 2; the others 4, else 2): a tile row holds a whole 16-site
    // x line, 256 contiguous bytes per spinor component, so x hops stay in
    // the tile and every cache line a wave touches is used in full
    const int want = d == 0 ? 16 : 4;
    int bd = 2;
    for (int t = want; t >= 4; t >>= 1)
      if (dims[d] % t == 0) {
        bd = t;
        break;
      }
    g.b[d] = bd;
    g.lb[d] = 0;
    while ((1 << g.lb[d]) < g.b[d]) ++g.lb[d];
    g.nt[d] = dims[d] / g.b[d];
  }
  int ls = 1, lts = 0;
  for (int d = 0; d < 4; ++d) {
    g.lstr[d] = ls;
    ls *= g.b[d];
    lts += g.lb[d];
  }
  g.lts = lts;
  int ts = 1 << lts;
  for (int d = 0; d < 4; ++d) {
    g.tstr[d] = ts;
    ts *= g.nt[d];
  }
}

int pack_gauge(nk_lattice* lat, const C64* canon, hipStream_t st) {
  const int V = lat->g.V;
  if (lat->U64.ensure((size_t)36 * V * sizeof(C64)) || lat->U32.ensure((size_t)40 * V * sizeof(C32)) ||
      lat->Ubf.ensure((size_t)24 * V * sizeof(uint32_t)))
    return NK_ENOMEM;
  hipLaunchKernelGGL(k_pack_gauge, dim3((V + 255) / 256), dim3(256), 0, st, lat->g, canon, lat->U64.as<C64>(),
                     lat->U32.as<C32>(), lat->Ubf.as<uint32_t>());
  NK_HIP(hipGetLastError());
  return NK_OK;
}

template <class R>
int pack_spinor(const Geom& g, const C64* canon, Cx<R>* dev, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_spinor<R>, dim3((g.V + 255) / 256), dim3(256), 0, st, g, canon, dev);
  NK_HIP(hipGetLastError());
  return NK_OK;
}

template <class R>
int unpack_spinor(const Geom& g, const Cx<R>* dev, C64* canon, hipStream_t st) {
  hipLaunchKernelGGL(k_unpack_spinor<R>, dim3((g.V + 255) / 256), dim3(256), 0, st, g, dev, canon);
  NK_HIP(hipGetLastError());
  return NK_OK;
}

template int pack_spinor<double>(const Geom&, const C64*, C64*, hipStream_t);
template int pack_spinor<float>(const Geom&, const C64*, C32*, hipStream_t);
template int unpack_spinor<double>(const Geom&, const C64*, C64*, hipStream_t);
template int unpack_spinor<float>(const Geom&, const C32*, C64*, hipStream_t);

}  // namespace nk
