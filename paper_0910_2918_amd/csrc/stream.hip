// Streaming kernels that measure what this library's own memory-bound code
// can reach on the device: read-only, copy and triad passes over complex128
// arrays, 16 bytes per lane per access, four accesses in flight per lane.
// They take no part in the sign function; the stencil's and the
// recurrences' bandwidth figures are read against them.
#include "nk_internal.h"

namespace nk {

constexpr int SNT = 256;
constexpr int SU = 4;  // accesses in flight per lane

// kind 0: partial sums of |a|^2 per workgroup into c (read-only pass)
// kind 1: c = a
// kind 2: c = a + s b (triad)
template <int KIND>
__global__ void __launch_bounds__(SNT) k_stream(size_t n, const C64* __restrict__ a, const C64* __restrict__ b,
                                                C64* __restrict__ c, double s) {
  const size_t stride = (size_t)gridDim.x * SNT;
  double acc = 0.0;
  for (size_t i0 = (size_t)blockIdx.x * SNT + threadIdx.x; i0 < n; i0 += SU * stride) {
    C64 va[SU], vb[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const size_t i = i0 + u * stride;
      if (i < n) {
        va[u] = a[i];
        if (KIND == 2) vb[u] = b[i];
      }
    }
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const size_t i = i0 + u * stride;
      if (i < n) {
        if (KIND == 0) acc += norm2(va[u]);
        if (KIND == 1) c[i] = va[u];
        if (KIND == 2) c[i] = va[u] + s * vb[u];
      }
    }
  }
  if (KIND == 0) {
    __shared__ double sh[SNT / 64];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) c[blockIdx.x] = mk((sh[0] + sh[1]) + (sh[2] + sh[3]), 0.0);
  }
}

}  // namespace nk

using namespace nk;

extern "C" int nk_stream_device(int32_t kind, int64_t n, const void* a, const void* b, void* c, int32_t blocks,
                                nk_stream_t stream) {
  if (kind < 0 || kind > 2 || n < 1 || !a || !c || (kind == 2 && !b) || blocks < 1) {
    set_error("invalid argument to nk_stream_device");
    return NK_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  const C64* pa = (const C64*)a;
  const C64* pb = (const C64*)b;
  C64* pc = (C64*)c;
  if (kind == 0)
    hipLaunchKernelGGL(k_stream<0>, dim3(blocks), dim3(SNT), 0, st, (size_t)n, pa, pb, pc, 0.0);
  else if (kind == 1)
    hipLaunchKernelGGL(k_stream<1>, dim3(blocks), dim3(SNT), 0, st, (size_t)n, pa, pb, pc, 0.0);
  else
    hipLaunchKernelGGL(k_stream<2>, dim3(blocks), dim3(SNT), 0, st, (size_t)n, pa, pb, pc, 0.5);
  NK_HIP(hipGetLastError());
  return NK_OK;
}
