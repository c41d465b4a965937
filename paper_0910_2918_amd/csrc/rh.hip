// Roberts-Higham iteration S_{n+1} = (S_n + S_n^{-1}) / 2 (Eq. (4)) for a
// batch of dense complex matrices of uneven sizes, on gfx950.
//
// Orders up to 128 run every iteration in one launch per batch (k_rh_small,
// below).  Larger ones invert each iterate by a blocked Gauss-Jordan
// elimination with partial pivoting in which rows are never moved: posof[r]
// is the column whose pivot row is r (-1 while r is unused) and rowof[c] the
// pivot row of column c, and the eliminated matrix X holds
// inv(S)[posof[r]][rowof[c]] at (r, c).  For each panel of NB columns
// c0 .. c0 + NB - 1 of the buffer `old`:
//  * k_gjp (one workgroup per matrix) eliminates the panel columns in
//    registers, each thread owning whole panel rows (loaded and stored
//    through LDS, sixteen threads to a row, where the panel fits).  Per
//    column: every lane forms a 32-bit pivot key of its unused rows (the
//    magnitude's float bits with the low 13 bits replaced by 8191 - row, so
//    the largest magnitude to ten mantissa bits wins and ties go to the
//    smaller row), a DPP maximum gives each wave's largest key, which goes to
//    LDS; after a barrier every thread knows the pivot row, whose owner
//    writes it to LDS; after a second barrier every thread updates its own
//    rows with it.  The transformed panel M (rows in place) goes to the
//    panel columns of `new`.
//  * k_gju applies the panel to every other column on the FP64 matrix cores
//    (v_mfma_f64_16x16x4f64, four real products per complex one):
//      new[r][j] = (posof[r] in the panel ? 0 : old[r][j]) + sum_t M[r][t] old[rowof[c0 + t]][j],
//    reading `old` and writing `new` (ping-pong), so no workgroup reads a
//    row that another one writes.
// The panel's thread count (and so rows per thread) and the update's output
// tile are chosen per matrix-size class by timing every feasible pair once
// (the autotuner below).  None of them changes the arithmetic: the pivot key
// is independent of the thread layout, every panel row sees the same
// operations in the same order, and every output element of the update is
// accumulated by the same matrix-core chain at the same position of a
// 16 x 16 tile whatever the output tile; so the choice never changes a bit
// of the result.  k_gjcombine maps X back through posof and rowof, forms the
// average (optionally with a positive scale mu, which leaves the limit
// unchanged) and emits partial sums of |S_{n+1} - S_n|_F^2 and
// |S_{n+1}|_F^2 for the host's stopping test.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>

#include "hostbuf.h"
#include "nk_internal.h"

namespace nk {

constexpr int PT = 1024;  // largest panel thread count
constexpr int UT = 256;   // update threads: four waves of 16 x 16 matrix-core tiles

__device__ __forceinline__ double cabs1(C64 a) { return fabs(a.re) + fabs(a.im); }

// 1 / a = conj(a) / |a|^2 with a first scaled by a power of two (exact), so
// that |a|^2 neither overflows nor underflows: one division
__device__ __forceinline__ C64 crecip1(C64 a) {
  int e;
  (void)frexp(fmax(fabs(a.re), fabs(a.im)), &e);
  const double ar = ldexp(a.re, -e), ai = ldexp(a.im, -e);
  const double q = 1.0 / (ar * ar + ai * ai);
  return mk(ldexp(ar * q, -e), ldexp(-ai * q, -e));
}

typedef double nk_d4 __attribute__((ext_vector_type(4)));

// the 32-bit pivot key of a panel row r < 4096 (never zero)
__device__ __forceinline__ unsigned gj_key(double mag, int r) {
  if (!(mag >= 0.0)) mag = 0.0;  // a NaN entry counts as a zero pivot, so some row is always chosen
  return (__float_as_uint((float)mag) & ~0x1FFFu) | (unsigned)(8191 - r);
}

// the largest of a 32-bit value over the 64 lanes of a wave (DPP row shifts,
// then the row broadcasts), in every lane
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));  // row_shr:1
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));  // row_shr:2
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));  // row_shr:4
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));  // row_shr:8
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// LDS staging of the whole panel (coalesced loads and stores) when it fits
template <int NB, int RM, int PTH>
struct GJStage {
  static constexpr bool on = (size_t)PTH * RM * (NB + 1) * sizeof(C64) <= 144 * 1024;
  static constexpr int rows = on ? PTH * RM : 1;
};

template <int NB, int RM, int PTH>
__global__ void __launch_bounds__(PTH) k_gjp(int ld, const int* __restrict__ nvec, const int* __restrict__ active,
                                            int c0, const C64* __restrict__ Aold_b, C64* __restrict__ Anew_b,
                                            int* __restrict__ rowof_b, int* __restrict__ posof_b,
                                            double* __restrict__ logdet, int* __restrict__ sing) {
  constexpr int NW = PTH / 64;
  using SG = GJStage<NB, RM, PTH>;
  const int b = blockIdx.x;
  const int n = nvec[b];
  if (!active[b] || c0 >= n) return;
  const int nbe = min(NB, n - c0);
  const size_t off = (size_t)b * ld * ld;
  const C64* Aold = Aold_b + off;
  C64* Anew = Anew_b + off;
  int* rowof = rowof_b + (size_t)b * ld;
  int* posof = posof_b + (size_t)b * ld;
  // one LDS block with the small arrays first, so that their addresses fit the
  // immediate offset of an LDS instruction
  __shared__ struct {
    C64 prow[2][NB];
    unsigned key[2][NW];
    int piv[NB];  // pivot rows of the panel, written to memory after the last column
    C64 panel[SG::rows][NB + 1];
  } sh;
  auto& s_key = sh.key;
  auto& s_prow = sh.prow;
  auto& s_piv = sh.piv;
  auto& s_panel = sh.panel;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  C64 a[RM][NB];
  bool used[RM];
  if constexpr (SG::on) {
    // sixteen consecutive threads read one row's NB entries (contiguous);
    // sixteen loads per thread go out together before any LDS write, so the
    // panel costs one memory round trip per batch, not one per entry
    constexpr int PER = SG::rows * NB / PTH, BMAX = PTH >= 1024 ? 8 : 16, BAT = PER < BMAX ? PER : BMAX;
    static_assert(PER % BAT == 0, "panel entries per thread in whole batches");
#pragma unroll
    for (int q0 = 0; q0 < PER; q0 += BAT) {
      C64 v[BAT];
#pragma unroll
      for (int q = 0; q < BAT; ++q) {
        const int e = tid + (q0 + q) * PTH, r = e / NB, t = e % NB;
        v[q] = (r < n && t < nbe) ? Aold[(size_t)r * ld + c0 + t] : mk(0.0, 0.0);
      }
#pragma unroll
      for (int q = 0; q < BAT; ++q) asm volatile("" : "+v"(v[q].re), "+v"(v[q].im));
#pragma unroll
      for (int q = 0; q < BAT; ++q) {
        const int e = tid + (q0 + q) * PTH;
        s_panel[e / NB][e % NB] = v[q];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    const int r = tid + m * PTH;
    used[m] = !(r < n) || posof[r] >= 0;  // rows past the order never pivot
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      if constexpr (SG::on)
        a[m][t] = s_panel[r][t];
      else
        a[m][t] = (r < n && t < nbe) ? Aold[(size_t)r * ld + c0 + t] : mk(0.0, 0.0);
    }
  }
  // the wave's largest pivot key of column tc over its unused rows
  auto col_key = [&](int tc) -> unsigned {
    unsigned key = 0;
#pragma unroll
    for (int m = 0; m < RM; ++m)
      if (!used[m]) {
        const unsigned kk = gj_key(cabs1(a[m][tc]), tid + m * PTH);
        key = kk > key ? kk : key;
      }
    return wave_max_u32(key);
  };
  // |det| of the panel's pivots as a running mantissa and binary exponent
  double dm = 1.0;
  int de = 0, bad = 0;
  unsigned wkey = col_key(0);  // c0 < n, so the panel has a column 0
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    if (t < nbe) {
      const int par = t & 1;
      // 1. every wave's largest key (formed during the previous column's
      //    update), then (after a barrier) the block's
      if (lane == 0) s_key[par][wid] = wkey;
      __syncthreads();
      unsigned best = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const unsigned kw = s_key[par][w];
        best = kw > best ? kw : best;
      }
      // while t < n - c0 an unused row remains, so best != 0; a zero key
      // would only leave pr = -1 (no row replaced) and a zero multiplier
      const int pr = best ? 8191 - (int)(best & 0x1FFFu) : -1;
      // 2. the pivot row's owner hands its row to every thread, then sets its
      //    own copy to -e_t, so that the common update of step 3 turns it into
      //    the scaled pivot row
#pragma unroll
      for (int m = 0; m < RM; ++m)
        if (tid + m * PTH == pr) {
#pragma unroll
          for (int u = 0; u < NB; ++u) s_prow[par][u] = a[m][u];
#pragma unroll
          for (int u = 0; u < NB; ++u) a[m][u] = mk(u == t ? -1.0 : 0.0, 0.0);
          used[m] = true;
        }
      if (tid == 0) s_piv[t] = pr;
      __syncthreads();
      // the pivot row in registers, all of it read before any use (one LDS
      // round trip, not one per entry) where the register budget allows it
      // (up to 512 threads: two waves per SIMD); the pivot itself first, so
      // that its reciprocal is formed while the rest arrives
      constexpr bool REGROW = PTH < 1024;
      C64 prow[REGROW ? NB : 1];
      if constexpr (REGROW) {
        prow[t] = s_prow[par][t];
#pragma unroll
        for (int u = 0; u < NB; ++u)
          if (u != t) prow[u] = s_prow[par][u];
        asm volatile("" : "+v"(prow[t].re), "+v"(prow[t].im));
      }
      auto prow_at = [&](int u) -> C64 {
        if constexpr (REGROW)
          return prow[u];
        else
          return s_prow[par][u];
      };
      const C64 piv = best ? prow_at(t) : mk(0.0, 0.0);
      const bool nz = cabs1(piv) > 0.0;
      if (!nz) bad = 1;
      const C64 d = nz ? crecip1(piv) : mk(0.0, 0.0);
      if (nz) {
        int ex;
        dm = frexp(dm * norm2(piv), &ex);
        de += ex;
      }
      if constexpr (REGROW) {
#pragma unroll
        for (int u = 0; u < NB; ++u)
          if (u != t) asm volatile("" : "+v"(prow[u].re), "+v"(prow[u].im));
      }
      // 3. one branch-free update for every row, with p the pivot row and
      //    g = a[t] / piv:  a[t] = -g,  a[u] = a[u] - g p[u] (u != t).
      //    Other rows: column t becomes -a[t] / piv.  The pivot row holds -e_t
      //    (step 2), so g = -1 / piv and the row becomes p / piv with 1 / piv
      //    in column t.  Column t + 1 goes first, so that the next column's
      //    key and its wave maximum overlap the rest of the update.
      C64 g[RM];
#pragma unroll
      for (int m = 0; m < RM; ++m) g[m] = cmul(a[m][t], d);
      auto upd = [&](int m, int u) {
        const C64 p = prow_at(u);
        a[m][u] = mk(fma(g[m].im, p.im, fma(-g[m].re, p.re, a[m][u].re)),
                     fma(-g[m].im, p.re, fma(-g[m].re, p.im, a[m][u].im)));
      };
      if (t + 1 < NB) {
        const int tn = t + 1 < NB ? t + 1 : t;  // (keeps the index in range where this is dead code)
#pragma unroll
        for (int m = 0; m < RM; ++m) upd(m, tn);
        wkey = col_key(tn);
      }
#pragma unroll
      for (int m = 0; m < RM; ++m) {
#pragma unroll
        for (int u = 0; u < NB; ++u) {
          if (u == t)
            a[m][u] = mk(-g[m].re, -g[m].im);
          else if (u != t + 1)
            upd(m, u);
        }
      }
    }
  }
  if constexpr (SG::on) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < RM; ++m)
#pragma unroll
      for (int t = 0; t < NB; ++t) s_panel[tid + m * PTH][t] = a[m][t];
    __syncthreads();
    // the same batches out: all LDS reads of a batch before its stores
    constexpr int PER = SG::rows * NB / PTH, BMAX = PTH >= 1024 ? 8 : 16, BAT = PER < BMAX ? PER : BMAX;
#pragma unroll
    for (int q0 = 0; q0 < PER; q0 += BAT) {
      C64 v[BAT];
#pragma unroll
      for (int q = 0; q < BAT; ++q) {
        const int e = tid + (q0 + q) * PTH;
        v[q] = s_panel[e / NB][e % NB];
      }
#pragma unroll
      for (int q = 0; q < BAT; ++q) {
        const int e = tid + (q0 + q) * PTH, r = e / NB, t = e % NB;
        if (r < n && t < nbe) Anew[(size_t)r * ld + c0 + t] = v[q];
      }
    }
  } else {
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      const int r = tid + m * PTH;
      if (r < n)
#pragma unroll
        for (int t = 0; t < NB; ++t)
          if (t < nbe) Anew[(size_t)r * ld + c0 + t] = a[m][t];
    }
  }
  if (tid < nbe) {
    const int pr = s_piv[tid];
    if (pr >= 0) {
      rowof[c0 + tid] = pr;
      posof[pr] = c0 + tid;
    }
  }
  if (tid == 0) {
    logdet[b] += 0.5 * (log(dm) + de * 0.69314718055994530942);
    if (bad) sing[b] = 1;
  }
}

// the rank-NB update of every column outside the panel, T x T output tile
// per 256-thread workgroup: four waves in a 2 x 2 arrangement, each with
// (T / 32)^2 sub-tiles of 16 x 16 on the matrix cores.  MFMA operand layout
// (16 x 16 x 4, FP64): lane l holds A[l % 16][l / 16] and B[l / 16][l % 16],
// and accumulator element i of lane l is D[4 i + l / 16][l % 16].
template <int NB, int T>
__global__ void __launch_bounds__(256) k_gju(int ld, const int* __restrict__ nvec, const int* __restrict__ active,
                                            int c0, const C64* __restrict__ Aold_b, C64* __restrict__ Anew_b,
                                            const int* __restrict__ rowof_b, const int* __restrict__ posof_b) {
  constexpr int SUB = T / 32;
  const int b = blockIdx.z;
  const int n = nvec[b];
  if (!active[b] || c0 >= n) return;
  const int row0 = blockIdx.y * T, col0 = blockIdx.x * T;
  if (row0 >= n || col0 >= n) return;
  const int nbe = min(NB, n - c0);
  const size_t off = (size_t)b * ld * ld;
  const C64* Aold = Aold_b + off;
  C64* Anew = Anew_b + off;
  const int* rowof = rowof_b + (size_t)b * ld;
  const int* posof = posof_b + (size_t)b * ld;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = row0 + (w >> 1) * 16 * SUB, wc = col0 + (w & 1) * 16 * SUB;
  const int l16 = lane & 15, lq = lane >> 4;
  nk_d4 are[SUB][SUB], aim[SUB][SUB];
#pragma unroll
  for (int si = 0; si < SUB; ++si)
#pragma unroll
    for (int sj = 0; sj < SUB; ++sj) {
      are[si][sj] = nk_d4{0.0, 0.0, 0.0, 0.0};
      aim[si][sj] = nk_d4{0.0, 0.0, 0.0, 0.0};
    }
#pragma unroll
  for (int kk = 0; kk < NB / 4; ++kk) {
    const int t = kk * 4 + lq;
    const bool tin = t < nbe;
    const int src = tin ? rowof[c0 + t] : 0;
    C64 am[SUB], bm[SUB];
#pragma unroll
    for (int si = 0; si < SUB; ++si) {
      const int r = wr + si * 16 + l16;
      am[si] = (tin && r < n) ? Anew[(size_t)r * ld + c0 + t] : mk(0.0, 0.0);
    }
#pragma unroll
    for (int sj = 0; sj < SUB; ++sj) {
      const int c = wc + sj * 16 + l16;
      bm[sj] = (tin && c < n) ? Aold[(size_t)src * ld + c] : mk(0.0, 0.0);
    }
#pragma unroll
    for (int si = 0; si < SUB; ++si)
#pragma unroll
      for (int sj = 0; sj < SUB; ++sj) {
        are[si][sj] = __builtin_amdgcn_mfma_f64_16x16x4f64(am[si].re, bm[sj].re, are[si][sj], 0, 0, 0);
        are[si][sj] = __builtin_amdgcn_mfma_f64_16x16x4f64(-am[si].im, bm[sj].im, are[si][sj], 0, 0, 0);
        aim[si][sj] = __builtin_amdgcn_mfma_f64_16x16x4f64(am[si].re, bm[sj].im, aim[si][sj], 0, 0, 0);
        aim[si][sj] = __builtin_amdgcn_mfma_f64_16x16x4f64(am[si].im, bm[sj].re, aim[si][sj], 0, 0, 0);
      }
  }
#pragma unroll
  for (int si = 0; si < SUB; ++si)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wr + si * 16 + 4 * i + lq;
      if (r >= n) continue;
      const int p = posof[r];
      const bool keep = !(p >= c0 && p < c0 + nbe);
#pragma unroll
      for (int sj = 0; sj < SUB; ++sj) {
        const int c = wc + sj * 16 + l16;
        if (c >= n || (c >= c0 && c < c0 + nbe)) continue;
        const C64 base = keep ? Aold[(size_t)r * ld + c] : mk(0.0, 0.0);
        Anew[(size_t)r * ld + c] = base + mk(are[si][sj][i], aim[si][sj][i]);
      }
    }
}

__global__ void k_gjstart(int ld, int batch, const int* __restrict__ nvec, const int* __restrict__ active,
                          int* __restrict__ posof_b, double* __restrict__ logdet) {
  const int b = blockIdx.y;
  if (!active[b]) return;
  const int n = nvec[b];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    posof_b[(size_t)b * ld + i] = -1;
  if (blockIdx.x == 0 && threadIdx.x == 0) logdet[b] = 0.0;
}

// The host's stopping sums of every matrix (one workgroup each): the
// inversion step's |S_{n+1} - S_n|^2 and |S_{n+1}|^2 partials (k_gjcombine,
// nbl pairs) and the Newton-Schulz kernels' pairs (k_ns_gemm, ntile2 pairs),
// each thread adding a strided subset, then a fixed-order tree, so the sums do
// not depend on timing.  They go straight into host memory (out, four per
// matrix), where the host has left a sentinel bit pattern that it polls for
// being overwritten; partials a step did not write are summed too and
// ignored by the host.
__global__ void __launch_bounds__(256) k_rh_sums(int nbl, const double* __restrict__ part, int ntile2,
                                                 const double* __restrict__ nspart, double* __restrict__ out) {
  const int b = blockIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nbl; i += 256) {
    v[0] += part[((size_t)b * nbl + i) * 2 + 0];
    v[1] += part[((size_t)b * nbl + i) * 2 + 1];
  }
  for (int i = threadIdx.x; i < ntile2; i += 256) {
    v[2] += nspart[((size_t)b * ntile2 + i) * 2 + 0];
    v[3] += nspart[((size_t)b * ntile2 + i) * 2 + 1];
  }
  __shared__ double sh[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < 4; ++q) sh[q][threadIdx.x >> 6] = v[q];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 4; ++q) out[b * 4 + q] = (sh[q][0] + sh[q][1]) + (sh[q][2] + sh[q][3]);
}

// G0/G1: the ping-pong buffers; a matrix of order n ends its elimination in
// the buffer of its own last panel, (ceil(n / nb) - 1) % 2.
// S_{n+1}[posof[r]][rowof[c]] = (mu S_n[..][..] + X[r][c] / mu) / 2
__global__ void __launch_bounds__(256) k_gjcombine(int ld, int nb, const int* __restrict__ nvec,
                                                   const int* __restrict__ active, const C64* __restrict__ G0,
                                                   const C64* __restrict__ G1, C64* __restrict__ X_b,
                                                   const int* __restrict__ rowof_b, const int* __restrict__ posof_b,
                                                   const double* __restrict__ logdet, int scaling,
                                                   const double* __restrict__ mu_sched, int mu_steps, int step,
                                                   double* __restrict__ part) {
  const int b = blockIdx.y;
  const int n = nvec[b];
  double dsum = 0.0, nsum = 0.0;
  if (active[b]) {
    double mu = 1.0;
    if (scaling == NK_RH_DET || scaling == NK_RH_LEARNED) mu = exp(-logdet[b] / n);
    if (scaling == NK_RH_LEARNED && mu_sched && step < mu_steps) {  // learned correction of this step
      const double m = mu_sched[(size_t)b * mu_steps + step];
      if (m > 0.0) mu *= m;
    }
    const double imu = 1.0 / mu;
    const size_t off = (size_t)b * ld * ld;
    const int npan = (n + nb - 1) / nb;
    const C64* G = (((npan - 1) & 1) ? G1 : G0) + off;
    C64* X = X_b + off;
    const int* rowof = rowof_b + (size_t)b * ld;
    const int* posof = posof_b + (size_t)b * ld;
    const size_t nn = (size_t)n * n;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < nn; e += (size_t)gridDim.x * 256) {
      const int r = (int)(e / n), c = (int)(e % n);
      const size_t xi = (size_t)posof[r] * ld + rowof[c];
      const C64 xs = mu * X[xi];
      const C64 s = 0.5 * (xs + imu * G[(size_t)r * ld + c]);
      X[xi] = s;
      const C64 d = s - xs;
      dsum += norm2(d);
      nsum += norm2(s);
    }
  }
  __shared__ double sh[2][4];
  for (int o = 32; o > 0; o >>= 1) {
    dsum += __shfl_xor(dsum, o, 64);
    nsum += __shfl_xor(nsum, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = dsum;
    sh[1][threadIdx.x >> 6] = nsum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[((size_t)b * gridDim.x + blockIdx.x) * 2 + 0] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
    part[((size_t)b * gridDim.x + blockIdx.x) * 2 + 1] = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
  }
}


// ---------------------------------------------------------------------------
// Newton-Schulz tail of the iteration (an option of this library, not the
// paper's): once |I - S_n^2|_F < 1/2, X <- X (3 I - X^2) / 2 converges
// quadratically to the same sgn(S_n) = sgn(S_0) (with R = I - X^2 the next
// R is (3/4) R^2 + (1/4) R^3, so |R| falls monotonically below 1/2), and
// needs two matrix products per step instead of an inversion.
// k_ns_gemm: C = A B for n x n complex matrices, 32 x 32 output tile per
// 256-thread workgroup (2 x 2 waves of 16 x 16 matrix-core tiles), K in
// blocks of 16 staged through LDS with the next block's loads in flight
// during the current block's products.
//  MODE 0: C = 3 I - A B, partial sums of |I - A B|_F^2 (A = B = S);
//  MODE 1: C = (A B) / 2, partial sums of |C - A|_F^2 and |C|_F^2
//          (A = S, B = 3 I - S^2, so C is the next iterate).
// Partial sums: one pair per workgroup at part[(b * tiles^2 + tile) * 2].
template <int MODE>
__global__ void __launch_bounds__(256) k_ns_gemm(int ld, const int* __restrict__ nvec, const int* __restrict__ active,
                                                const C64* __restrict__ A_b, const C64* __restrict__ B_b,
                                                C64* __restrict__ C_b, double* __restrict__ part) {
  const int b = blockIdx.z;
  const int n = nvec[b];
  const int tile = blockIdx.y * gridDim.x + blockIdx.x;
  double s0 = 0.0, s1 = 0.0;
  __shared__ C64 sA[32][17];
  __shared__ C64 sB[16][33];
  __shared__ double sh[2][4];
  const bool live = active[b] && blockIdx.y * 32 < n && blockIdx.x * 32 < n;
  if (live) {
    const size_t off = (size_t)b * ld * ld;
    const C64* A = A_b + off;
    const C64* B = B_b + off;
    C64* C = C_b + off;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int row0 = blockIdx.y * 32, col0 = blockIdx.x * 32;
    const int l16 = lane & 15, lq = lane >> 4;
    const int wr = (w >> 1) * 16, wc = (w & 1) * 16;
    nk_d4 are = {0.0, 0.0, 0.0, 0.0}, aim = {0.0, 0.0, 0.0, 0.0};
    C64 ra[2], rb[2];
    auto load = [&](int k0) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int e = tid + 256 * q;
        const int ar = row0 + e / 16, ak = k0 + e % 16;
        ra[q] = (ar < n && ak < n) ? A[(size_t)ar * ld + ak] : mk(0.0, 0.0);
        const int bk = k0 + e / 32, bc = col0 + e % 32;
        rb[q] = (bk < n && bc < n) ? B[(size_t)bk * ld + bc] : mk(0.0, 0.0);
      }
    };
    load(0);
    for (int k0 = 0; k0 < n; k0 += 16) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int e = tid + 256 * q;
        sA[e / 16][e % 16] = ra[q];
        sB[e / 32][e % 32] = rb[q];
      }
      __syncthreads();
      if (k0 + 16 < n) load(k0 + 16);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const C64 am = sA[wr + l16][kk * 4 + lq];
        const C64 bm = sB[kk * 4 + lq][wc + l16];
        are = __builtin_amdgcn_mfma_f64_16x16x4f64(am.re, bm.re, are, 0, 0, 0);
        are = __builtin_amdgcn_mfma_f64_16x16x4f64(-am.im, bm.im, are, 0, 0, 0);
        aim = __builtin_amdgcn_mfma_f64_16x16x4f64(am.re, bm.im, aim, 0, 0, 0);
        aim = __builtin_amdgcn_mfma_f64_16x16x4f64(am.im, bm.re, aim, 0, 0, 0);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = row0 + wr + 4 * i + lq, c = col0 + wc + l16;
      if (r >= n || c >= n) continue;
      const C64 p = mk(are[i], aim[i]);
      if (MODE == 0) {
        const double dg = r == c ? 1.0 : 0.0;
        C[(size_t)r * ld + c] = mk(3.0 * dg - p.re, -p.im);
        s0 += norm2(mk(dg - p.re, -p.im));
      } else {
        const C64 g = 0.5 * p;
        C[(size_t)r * ld + c] = g;
        s0 += norm2(g - A[(size_t)r * ld + c]);
        s1 += norm2(g);
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o, 64);
    s1 += __shfl_xor(s1, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = s0;
    sh[1][threadIdx.x >> 6] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const size_t p = ((size_t)b * gridDim.x * gridDim.y + tile) * 2;
    part[p + 0] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
    part[p + 1] = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
  }
}

// S <- G for the matrices in the Newton-Schulz set
__global__ void k_ns_copy(int ld, const int* __restrict__ nvec, const int* __restrict__ active,
                          const C64* __restrict__ G_b, C64* __restrict__ S_b) {
  const int b = blockIdx.y;
  if (!active[b]) return;
  const int n = nvec[b];
  const size_t off = (size_t)b * ld * ld, nn = (size_t)n * n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = off + (e / n) * ld + (e % n);
    S_b[i] = G_b[i];
  }
}

// r_b = |S_b^2 - I|_F / sqrt(n_b) from the per-tile partial sums of
// |I - S^2|_F^2 that k_ns_gemm<0> leaves (tiles x tiles pairs per matrix),
// summed in tile order by one workgroup per matrix
__global__ void __launch_bounds__(256) k_rh_resid_sum(int tiles2, const int* __restrict__ nvec,
                                                      const double* __restrict__ part, double* __restrict__ out) {
  const int b = blockIdx.x;
  const int n = nvec[b];
  double acc = 0.0;
  for (int t = threadIdx.x; t < tiles2; t += 256) acc += part[((size_t)b * tiles2 + t) * 2];
  __shared__ double sh[4];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[b] = n > 0 ? sqrt(((sh[0] + sh[1]) + (sh[2] + sh[3])) / n) : 0.0;
}

// ---------------------------------------------------------------------------
// Small matrices (n <= 128): one 512-thread workgroup per matrix runs every
// Roberts-Higham iteration in a single launch, with the matrix being inverted
// in registers.  With nseg = floor(512 / n) row segments of rps = ceil(n / nseg)
// rows, thread tid owns column c = tid % n and rows r0 .. r0 + rps - 1 of
// segment tid / n (r0 = segment * rps); rps <= SQ.  Per pivot column t:
//   * the owners of column t copy it to LDS; every wave then finds the pivot
//     redundantly (largest unused row r_t, ties to the smaller row), so no
//     extra barrier is needed;
//   * the owner of (r_t, c) writes the scaled pivot row to LDS;
//   * every element updates from two LDS reads: the multiplier of its row
//     (a wave-wide broadcast) and the pivot-row value of its column.
// Rows are never moved: inv[pos(r)][r_c] is the element held at (r, c).
// LDS buffers are double-buffered by t, two barriers per pivot.  The
// iterates stay in the caller's global buffer and the stopping test runs in
// the kernel, so there is no host round trip per iteration.
constexpr int ST_RH = 512;  // threads: 128 columns x 4 row segments (256-register budget per lane)
constexpr int SMAX = 128;

__device__ __forceinline__ unsigned long long piv_key(double v, int r) {
  // larger |value| wins, then the smaller row index
  const float fv = (float)v;
  return ((unsigned long long)__float_as_uint(fv) << 32) | (unsigned)(0x7fffffff - r);
}

// the small kernel's 32-bit key: the float magnitude with its low eight
// mantissa bits replaced by 255 - r (r < 128, so never zero), and one
// unsigned maximum over the wave picks the largest magnitude to 15 mantissa
// bits, ties to the smaller row
__device__ __forceinline__ unsigned piv_key32(double v, int r) {
  return (__float_as_uint((float)v) & ~255u) | (unsigned)(255 - r);
}

template <int SQ>  // rows per thread, at least ceil(n / floor(512 / n)) (the host picks it)
__global__ void __launch_bounds__(ST_RH) k_rh_small(int ld, const int* __restrict__ nvec, C64* __restrict__ S_b,
                                                   int scaling, const double* __restrict__ mu_sched, int mu_steps,
                                                   int maxit, double tol, int* __restrict__ iters,
                                                   int* __restrict__ sing) {
  const int b = blockIdx.x;
  const int n = nvec[b];
  if (n <= 0) {
    if (threadIdx.x == 0) iters[b] = 0;
    return;
  }
  C64* S = S_b + (size_t)b * ld * ld;
  __shared__ C64 s_col[2][SMAX];
  __shared__ C64 s_row[2][SMAX];
  __shared__ int s_used[SMAX];
  __shared__ int s_rowof[SMAX];  // pivot row of column t
  __shared__ int s_pos[SMAX];    // column whose pivot row is r
  __shared__ double s_red[2][ST_RH / 64];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int nseg = ST_RH / n;
  const int rps = (n + nseg - 1) / nseg;  // <= SQ (checked by the host)
  const int c = tid % n;
  const int seg = tid / n;
  const int r0 = seg * rps;
  const int rend = min(n, r0 + rps);  // rows r0 .. rend - 1
  const bool colok = seg < nseg;
  C64 a[SQ];
  double prev = INFINITY;
  int it = 0, bad = 0;
  for (it = 1; it <= maxit; ++it) {
    // a per-iteration copy of the base pointer that the compiler cannot see
    // through: otherwise it hoists SQ 64-bit element addresses out of the
    // iteration loop and keeps them live through every pivot step
    C64* Sp = S;
    int base = r0 * ld + c;  // n <= 128 and ld <= 128: 32-bit offsets suffice
    asm volatile("" : "+s"(Sp), "+v"(base));
    const gp<C64> Si = as_global(Sp);
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
      C64 v = mk(0.0, 0.0);
      if (colok && r0 + q < rend) v = ldg(Si + (base + q * ld));
      a[q] = v;
      if ((q & 7) == 7) __builtin_amdgcn_sched_barrier(0);
    }
    for (int r = tid; r < n; r += ST_RH) s_used[r] = 0;
    // |det| as a running product of |pivot|^2 whose binary exponent is split
    // off after every step (no logarithm per pivot)
    double dm = 1.0;
    int de = 0;
    __syncthreads();
    for (int t = 0; t < n; ++t) {
      const int par = t & 1;
      if (colok && c == t) {
#pragma unroll
        for (int q = 0; q < SQ; ++q)
          if (r0 + q < rend) s_col[par][r0 + q] = a[q];
      }
      __syncthreads();
      unsigned key = 0;
      for (int r = lane; r < n; r += 64)
        if (!s_used[r]) {
          const C64 v = s_col[par][r];
          const unsigned kk = piv_key32(fabs(v.re) + fabs(v.im), r);
          key = kk > key ? kk : key;
        }
      key = wave_max_u32(key);
      // every unused row has a nonzero key, and one is unused while t < n; the
      // fallback only keeps the index in range should that ever not hold
      const int pr = key ? 255 - (int)(key & 255u) : t;
      const C64 pv = s_col[par][pr];
      if (!(fabs(pv.re) + fabs(pv.im) > 0.0)) bad = 1;
      const C64 d = crecip1(pv);
      if (scaling != NK_RH_NONE) {
        int ex;
        dm = frexp(dm * norm2(pv), &ex);
        de += ex;
      }
      if (colok && pr >= r0 && pr < rend) {
        C64 v = a[0];
#pragma unroll
        for (int q = 1; q < SQ; ++q)
          if (pr - r0 == q) v = a[q];
        s_row[par][c] = (c == t) ? d : cmul(v, d);
      }
      __syncthreads();
      if (tid == 0) {
        s_used[pr] = 1;
        s_rowof[t] = pr;
        s_pos[pr] = t;
      }
      const C64 rv = s_row[par][c];
      // column t keeps nothing of its old value (new entry -f d); every
      // other column subtracts f times the pivot row: one form for both
      const double keep = c == t ? 0.0 : 1.0;
      // rows past rend read stale LDS entries; their values are never used
#pragma unroll
      for (int q = 0; q < SQ; ++q) {
        const C64 f = s_col[par][min(r0 + q, SMAX - 1)];
        const double tre = fma(-f.im, rv.im, f.re * rv.re);
        const double tim = fma(f.re, rv.im, f.im * rv.re);
        a[q] = mk(fma(a[q].re, keep, -tre), fma(a[q].im, keep, -tim));
        if ((q & 7) == 7) __builtin_amdgcn_sched_barrier(0);  // bound the hoisted LDS reads
      }
      // the pivot row takes the scaled row itself (only its segment's threads)
      if (colok && pr >= r0 && pr < rend) {
        const int qs = pr - r0;
#pragma unroll
        for (int q = 0; q < SQ; ++q)
          if (q == qs) a[q] = rv;
      }
    }
    __syncthreads();
    // S_{n+1} = (mu S_n + (mu S_n)^{-1}) / 2, inv[pos(r)][rowof(c)] held at (r, c)
    const double logdet = scaling != NK_RH_NONE ? 0.5 * (log(dm) + de * 0.69314718055994530942) : 0.0;
    double mu = 1.0;
    if (scaling == NK_RH_DET) mu = exp(-logdet / n);
    if (scaling == NK_RH_LEARNED) {  // determinant scaling times the learned correction of this step
      const double m = (mu_sched && it - 1 < mu_steps) ? mu_sched[(size_t)b * mu_steps + (it - 1)] : -1.0;
      mu = exp(-logdet / n) * (m > 0.0 ? m : 1.0);
    }
    const double imu = 1.0 / mu;
    double dsum = 0.0, nsum = 0.0;
    if (colok) {
      const int j = s_rowof[c];
#pragma unroll
      for (int q = 0; q < SQ; ++q) {
        if (r0 + q < rend) {
          const int xi = s_pos[r0 + q] * ld + j;
          const C64 xs = mu * S[xi];
          const C64 sn = 0.5 * (xs + imu * a[q]);
          S[xi] = sn;
          dsum += norm2(sn - xs);
          nsum += norm2(sn);
        }
        if ((q & 7) == 7) __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      dsum += __shfl_xor(dsum, o, 64);
      nsum += __shfl_xor(nsum, o, 64);
    }
    if (lane == 0) {
      s_red[0][wid] = dsum;
      s_red[1][wid] = nsum;
    }
    __syncthreads();
    dsum = 0.0;
    nsum = 0.0;
#pragma unroll
    for (int w = 0; w < ST_RH / 64; ++w) {
      dsum += s_red[0][w];
      nsum += s_red[1][w];
    }
    const double change = sqrt(dsum / nsum);
    __syncthreads();
    if (bad || !(change > tol) || (change < 1e-6 && change > 0.5 * prev)) break;
    prev = change;
  }
  if (tid == 0) {
    iters[b] = it > maxit ? maxit : it;
    if (bad) sing[b] = 1;
    else if (it > maxit) sing[b] = 2;  // the cap ended the iteration before the stopping test held
  }
}

// ---------------------------------------------------------------------------
namespace {
std::mutex g_rh_mu;
DevBuf g_G0, g_G1, g_int, g_dbl, g_sched, g_nsp;
// pinned staging of the large path: flag uploads and the stopping sums
HostBuf g_pin, g_pinr;
// the Newton-Schulz tail of the large path (nk_rh_newton_schulz); on by default
int g_ns_tail = 1;
}  // namespace

template <int NB, int RM, int PTH, int T>
static void launch_inverse(int batch, int ld, int maxn, const int* nvec, const int* act, const C64* S, C64* G0,
                           C64* G1, int* rowof, int* posof, double* logdet, int* sing, hipStream_t st) {
  const C64* cur = S;
  int which = 0;
  const int tiles = (maxn + T - 1) / T;
  hipLaunchKernelGGL(k_gjstart, dim3((maxn + 255) / 256, batch), dim3(256), 0, st, ld, batch, nvec, act, posof,
                     logdet);
  for (int c0 = 0; c0 < maxn; c0 += NB) {
    C64* nxt = which ? G1 : G0;
    hipLaunchKernelGGL((k_gjp<NB, RM, PTH>), dim3(batch), dim3(PTH), 0, st, ld, nvec, act, c0, cur, nxt, rowof,
                       posof, logdet, sing);
    hipLaunchKernelGGL((k_gju<NB, T>), dim3(tiles, tiles, batch), dim3(UT), 0, st, ld, nvec, act, c0, cur, nxt,
                       rowof, posof);
    cur = nxt;
    which ^= 1;
  }
}

// The launch shapes of the blocked inverse: panel threads x rows per thread
// (which must cover ld) and the update tile.  The panel width is not among
// the choices: it sets the grouping of the update sums, 16 up to ld = 1024,
// 8 up to 2048 and 4 above, fixed by ld alone.
struct GJShape {
  int nb, rm, pth, tile;
};
// every instantiated shape (the panel keeps rm x nb complex values per
// thread in registers, so rm x nb x 4 VGPRs must fit beside the rest at
// pth / 256 waves per SIMD: at most 64 at 1024 threads, 128 at 512)
#define NK_GJ_SHAPES(X)                                                                                      \
  X(16, 1, 256, 32) X(16, 1, 256, 64) X(16, 1, 512, 32) X(16, 1, 512, 64) X(16, 1, 1024, 32)                \
  X(16, 1, 1024, 64) X(16, 2, 256, 32) X(16, 2, 256, 64) X(16, 2, 512, 32) X(16, 2, 512, 64)                \
  X(8, 2, 1024, 32) X(8, 2, 1024, 64) X(8, 4, 512, 32) X(8, 4, 512, 64)                                     \
  X(4, 4, 1024, 32) X(4, 4, 1024, 64)
#define NK_GJ_ENTRY(NB, RM, PTH, T) {NB, RM, PTH, T},
constexpr GJShape kGJShapes[] = {NK_GJ_SHAPES(NK_GJ_ENTRY)};
#undef NK_GJ_ENTRY

static int gj_nb(int ld) { return ld <= PT ? 16 : ld <= 2 * PT ? 8 : 4; }

static bool gj_feasible(const GJShape& sh, int ld) {
  for (const GJShape& k : kGJShapes)
    if (k.nb == sh.nb && k.rm == sh.rm && k.pth == sh.pth && k.tile == sh.tile)
      return sh.nb == gj_nb(ld) && sh.pth * sh.rm >= ld;
  return false;
}

// one blocked inverse with a shape that gj_feasible accepts for ld
static void launch_inverse_shape(const GJShape& sh, int batch, int ld, int maxn, const int* nvec, const int* act,
                                 const C64* S, C64* G0, C64* G1, int* rowof, int* posof, double* logdet, int* sing,
                                 hipStream_t st) {
#define NK_GJ_CALL(NB, RM, PTH, T)                                                                            \
  if (sh.nb == NB && sh.rm == RM && sh.pth == PTH && sh.tile == T)                                            \
    return launch_inverse<NB, RM, PTH, T>(batch, ld, maxn, nvec, act, S, G0, G1, rowof, posof, logdet, sing, st);
  NK_GJ_SHAPES(NK_GJ_CALL)
#undef NK_GJ_CALL
}

// autotuner state: the chosen shape per (size class, batch class), and an
// optional forced shape (nk_rh_tile_force)
std::map<int, GJShape> g_gj_choice;
GJShape g_gj_force{0, 0, 0, 0};

static int gj_key(int maxn, int batch) {
  const int bc = batch <= 1 ? 0 : batch <= 4 ? 1 : batch <= 16 ? 2 : 3;
  return ((maxn + 63) / 64) * 4 + bc;
}

// the shape for this batch: forced, cached, or found by timing one inverse of
// the current iterate with every feasible shape (the results are discarded;
// every shape computes the same bits)
static int gj_choose(int batch, int ld, int maxn, const int* nvec, const int* act, const C64* S, C64* G0, C64* G1,
                     int* rowof, int* posof, double* logdet, int* sing, hipStream_t st, GJShape* out) {
  if (g_gj_force.pth) {
    const GJShape f{gj_nb(ld), g_gj_force.rm, g_gj_force.pth, g_gj_force.tile};
    if (gj_feasible(f, ld)) {
      *out = f;
      return NK_OK;
    }
  }
  const int key = gj_key(maxn, batch);
  auto it = g_gj_choice.find(key);
  if (it != g_gj_choice.end() && gj_feasible(it->second, ld)) {
    *out = it->second;
    return NK_OK;
  }
  hipEvent_t e0, e1;
  NK_HIP(hipEventCreate(&e0));
  NK_HIP(hipEventCreate(&e1));
  float best = INFINITY;
  GJShape pick{0, 0, 0, 0};
  for (const GJShape& sh : kGJShapes) {
    if (!gj_feasible(sh, ld)) continue;
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {  // the first run of a shape warms it up
      NK_HIP(hipEventRecord(e0, st));
      launch_inverse_shape(sh, batch, ld, maxn, nvec, act, S, G0, G1, rowof, posof, logdet, sing, st);
      NK_HIP(hipEventRecord(e1, st));
      NK_HIP(hipEventSynchronize(e1));
      NK_HIP(hipEventElapsedTime(&ms, e0, e1));
    }
    if (ms < best) {
      best = ms;
      pick = sh;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  NK_HIP(hipGetLastError());
  g_gj_choice[key] = pick;
  *out = pick;
  return NK_OK;
}

// the warning for a batch: a singular iterate (state 1) or the iteration cap
// reached before the stopping test held (state 2) in any matrix
static int rh_outcome(int batch, const int* state, int maxit) {
  for (int b = 0; b < batch; ++b)
    if (state[b] == 1) {
      set_error("Roberts-Higham: singular iterate in matrix %d", b);
      return NK_WARN_NOTCONV;
    }
  for (int b = 0; b < batch; ++b)
    if (state[b] == 2) {
      set_error("Roberts-Higham: matrix %d did not converge in %d iterations", b, maxit);
      return NK_WARN_NOTCONV;
    }
  return NK_OK;
}

int rh_newton_schulz(int enable) {
  std::lock_guard<std::mutex> lock(g_rh_mu);
  const int old = g_ns_tail;
  g_ns_tail = enable ? 1 : 0;
  return old;
}

int rh_tile_force(int rm, int pth, int tile) {
  std::lock_guard<std::mutex> lock(g_rh_mu);
  if (rm == 0 && pth == 0 && tile == 0) {
    g_gj_force = GJShape{0, 0, 0, 0};
    return NK_OK;
  }
  for (const GJShape& k : kGJShapes)
    if (k.rm == rm && k.pth == pth && k.tile == tile) {
      g_gj_force = GJShape{0, rm, pth, tile};  // nb follows ld at use
      return NK_OK;
    }
  set_error("no blocked-inverse shape with %d rows per thread, %d panel threads and tile %d", rm, pth, tile);
  return NK_EINVAL;
}

int rh_tile_choice(int maxn, int batch, int* nb, int* rm, int* pth, int* tile) {
  std::lock_guard<std::mutex> lock(g_rh_mu);
  auto it = g_gj_choice.find(gj_key(maxn, batch));
  if (it == g_gj_choice.end()) {
    *nb = *rm = *pth = *tile = 0;
    return 0;
  }
  *nb = it->second.nb;
  *rm = it->second.rm;
  *pth = it->second.pth;
  *tile = it->second.tile;
  return 1;
}

// |S^2 - I|_F / sqrt(n) of every matrix of the batch into resid_host: one
// product S S on the matrix cores (k_ns_gemm<0>, which leaves 3 I - S^2 in the
// scratch buffer G0 and the partial sums of |I - S^2|_F^2), then the sums,
// written by k_rh_resid_sum straight into pinned host memory
static int rh_residuals(int batch, int maxn, int ld, const int* nvec, const C64* S, double* resid_host,
                        hipStream_t st) {
  const int ntile = (maxn + 31) / 32;
  const size_t nsp = (size_t)batch * ntile * ntile * 2;
  if (g_nsp.ensure(nsp * sizeof(double) + (size_t)batch * sizeof(int))) return NK_ENOMEM;
  if (g_pinr.ensure((size_t)batch * (sizeof(double) + sizeof(int)))) return NK_ENOMEM;
  double* part = g_nsp.as<double>();
  int* all = reinterpret_cast<int*>(part + nsp);
  int* ones = reinterpret_cast<int*>(g_pinr.host<double>() + batch);
  std::fill(ones, ones + batch, 1);
  NK_HIP(hipMemcpyAsync(all, ones, batch * sizeof(int), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_ns_gemm<0>, dim3(ntile, ntile, batch), dim3(256), 0, st, ld, nvec, all, S, S, g_G0.as<C64>(),
                     part);
  hipLaunchKernelGGL(k_rh_resid_sum, dim3(batch), dim3(256), 0, st, ntile * ntile, nvec, part, g_pinr.dev<double>());
  NK_HIP(hipGetLastError());
  NK_HIP(hipStreamSynchronize(st));
  std::copy(g_pinr.host<double>(), g_pinr.host<double>() + batch, resid_host);
  return NK_OK;
}

int rh_sign_batched(int batch, int ld, const int* n_host, C64* S, int scaling, int maxit, double tol,
                    int* iters_host, double* resid_host, hipStream_t st) {
  std::lock_guard<std::mutex> lock(g_rh_mu);
  if (batch <= 0 || ld <= 0) return NK_OK;
  if (ld > 4 * PT) {
    set_error("Roberts-Higham: matrix size %d exceeds %d", ld, 4 * PT);
    return NK_EINVAL;
  }
  const size_t mb = (size_t)batch * ld * ld * sizeof(C64);
  const int nbl = 64;
  if (g_G0.ensure(mb) || g_G1.ensure(mb) || g_int.ensure((size_t)batch * (2 * ld + 4) * sizeof(int)) ||
      g_dbl.ensure((size_t)batch * (2 * nbl + 4) * sizeof(double)))
    return NK_ENOMEM;
  int* nvec = g_int.as<int>();
  int* act = nvec + batch;
  int* sing = act + batch;
  int* rowof = sing + batch;
  int* posof = rowof + (size_t)batch * ld;
  double* logdet = g_dbl.as<double>();
  double* resid = logdet + batch;
  double* part = resid + batch;

  // Pinned, device-mapped staging (the previous call ended with a stream
  // synchronisation, so none of it is still in use): seven int arrays (the
  // orders, zeros, the initial active set, the inversion and Newton-Schulz
  // flags of the large path, the returned iteration counts and states) and
  // four stopping sums per matrix, which k_rh_sums writes into host memory.
  // Each flag array is uploaded only when its content changes and rewritten
  // only once later work of the stream has been seen to finish (so its last
  // upload has been consumed), and every host decision waits for one small
  // kernel's results instead of copies through pageable memory and a stream
  // synchronisation.
  const size_t pin_ints = (7 * (size_t)batch + 1) & ~(size_t)1;  // keeps the sums 8-byte aligned
  if (g_pin.ensure(pin_ints * sizeof(int) + 4 * (size_t)batch * sizeof(double))) return NK_ENOMEM;
  int* pin_n = g_pin.host<int>();
  int* pin_zero = pin_n + batch;
  int* pin_act0 = pin_zero + batch;
  int* pin_gj = pin_act0 + batch;
  int* pin_ns = pin_gj + batch;
  int* pin_iters = pin_ns + batch;
  int* pin_state = pin_iters + batch;
  const double* sums_h = reinterpret_cast<const double*>(g_pin.host<int>() + pin_ints);
  double* sums_d = reinterpret_cast<double*>(g_pin.dev<int>() + pin_ints);

  int maxn = 0;
  std::vector<int> act_h(batch);
  for (int b = 0; b < batch; ++b) maxn = std::max(maxn, n_host[b]);
  std::copy(n_host, n_host + batch, pin_n);
  std::fill(pin_zero, pin_zero + batch, 0);
  NK_HIP(hipMemcpyAsync(nvec, pin_n, batch * sizeof(int), hipMemcpyHostToDevice, st));
  // learned scaling: the installed model's factors for the first steps of
  // each matrix, predicted from S_0 (without a model: determinant scaling)
  const int mu_steps = NK_MLP_STEPS;
  const double* mdev = nullptr;
  if (scaling == NK_RH_LEARNED) {
    if (g_sched.ensure((size_t)batch * mu_steps * sizeof(double))) return NK_ENOMEM;
    int have = 0;
    if (int e = mlp_schedule(batch, ld, nvec, S, g_sched.as<double>(), &have, st)) return e;
    if (have) mdev = g_sched.as<double>();
  }
  if (maxn <= SMAX) {
    NK_HIP(hipMemcpyAsync(sing, pin_zero, batch * sizeof(int), hipMemcpyHostToDevice, st));
    int rps = 0;  // largest rows-per-thread over the batch
    for (int b = 0; b < batch; ++b)
      if (n_host[b] > 0) rps = std::max(rps, (n_host[b] + ST_RH / n_host[b] - 1) / (ST_RH / n_host[b]));
    // the smallest rows-per-thread bound that covers the batch: rows past a
    // thread's own are computed and discarded, so a tight bound halves the
    // per-pivot work each time it halves
    if (rps <= 2)
      hipLaunchKernelGGL(k_rh_small<2>, dim3(batch), dim3(ST_RH), 0, st, ld, nvec, S, scaling, mdev, mu_steps, maxit,
                         tol, act, sing);
    else if (rps <= 4)
      hipLaunchKernelGGL(k_rh_small<4>, dim3(batch), dim3(ST_RH), 0, st, ld, nvec, S, scaling, mdev, mu_steps, maxit,
                         tol, act, sing);
    else if (rps <= 8)
      hipLaunchKernelGGL(k_rh_small<8>, dim3(batch), dim3(ST_RH), 0, st, ld, nvec, S, scaling, mdev, mu_steps, maxit,
                         tol, act, sing);
    else if (rps <= 16)
      hipLaunchKernelGGL(k_rh_small<16>, dim3(batch), dim3(ST_RH), 0, st, ld, nvec, S, scaling, mdev, mu_steps, maxit,
                         tol, act, sing);
    else
      hipLaunchKernelGGL(k_rh_small<32>, dim3(batch), dim3(ST_RH), 0, st, ld, nvec, S, scaling, mdev, mu_steps, maxit,
                         tol, act, sing);
    NK_HIP(hipGetLastError());
    NK_HIP(hipMemcpyAsync(pin_iters, act, batch * sizeof(int), hipMemcpyDeviceToHost, st));
    NK_HIP(hipMemcpyAsync(pin_state, sing, batch * sizeof(int), hipMemcpyDeviceToHost, st));
    if (resid_host)
      if (int e = rh_residuals(batch, maxn, ld, nvec, S, resid_host, st)) return e;
    NK_HIP(hipStreamSynchronize(st));
    std::copy(pin_iters, pin_iters + batch, iters_host);
    return rh_outcome(batch, pin_state, maxit);
  }
  maxn = 0;
  for (int b = 0; b < batch; ++b) {
    maxn = std::max(maxn, n_host[b]);
    act_h[b] = n_host[b] > 0 ? 1 : 0;
    iters_host[b] = 0;
  }
  std::copy(act_h.begin(), act_h.end(), pin_act0);
  NK_HIP(hipMemcpyAsync(act, pin_act0, batch * sizeof(int), hipMemcpyHostToDevice, st));
  // Newton-Schulz tail: workspace and per-matrix state (0: inversion steps,
  // 1: Newton-Schulz steps, entered once |I - S^2|_F < 1/2 and kept)
  const int ntile = (maxn + 31) / 32;
  const int ntile2 = ntile * ntile;
  const size_t nsp = (size_t)batch * ntile2 * 2;
  if (g_nsp.ensure(nsp * sizeof(double) + (size_t)batch * sizeof(int))) return NK_ENOMEM;
  double* nspart = g_nsp.as<double>();
  int* act_ns = reinterpret_cast<int*>(nspart + nsp);
  std::vector<int> ns_h(batch, 0), try_h(batch, 0), gj_h(batch, 0);
  // the device content of act and act_ns as last uploaded (-1: unknown)
  std::vector<int> dev_act(act_h), dev_ns(batch, -1);
  const int ns_on = g_ns_tail;
  GJShape shape;
  if (int e = gj_choose(batch, ld, maxn, nvec, act, S, g_G0.as<C64>(), g_G1.as<C64>(), rowof, posof, logdet, sing, st,
                        &shape))
    return e;
  NK_HIP(hipMemcpyAsync(sing, pin_zero, batch * sizeof(int), hipMemcpyHostToDevice, st));
  std::vector<double> prev(batch, INFINITY);
  // a flag array to the device, only when it differs from its last upload;
  // the staging slot is rewritten only here, after the stopping sums of a
  // later point of the stream (or a synchronisation) have been seen, so its
  // previous upload has been consumed
  auto upload = [&](int* dev, int* pin, const std::vector<int>& v, std::vector<int>& last) -> int {
    if (v == last) return NK_OK;
    std::copy(v.begin(), v.end(), pin);
    NK_HIP(hipMemcpyAsync(dev, pin, batch * sizeof(int), hipMemcpyHostToDevice, st));
    last = v;
    return NK_OK;
  };
  // the stopping sums of this point of the stream, in host memory: the host
  // fills them with a sentinel bit pattern (a NaN no arithmetic produces),
  // launches k_rh_sums and polls for up to 2 ms until every value is
  // overwritten (an iteration's kernels are usually done by then); otherwise
  // it waits on the stream, which also reports any error of the queued work.
  // Every value is one aligned 8-byte store.  Before each fill the previous
  // sums have all arrived, so no earlier write can land on a sentinel.
  constexpr uint64_t kSentinel = 0x7FF4D15EA5E0F00Dull;
  volatile uint64_t* sums_bits = reinterpret_cast<volatile uint64_t*>(const_cast<double*>(sums_h));
  auto sums = [&]() -> int {
    for (int i = 0; i < 4 * batch; ++i) sums_bits[i] = kSentinel;
    hipLaunchKernelGGL(k_rh_sums, dim3(batch), dim3(256), 0, st, nbl, (const double*)part, ntile2,
                       (const double*)nspart, sums_d);
    NK_HIP(hipGetLastError());
    const auto t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < 4 * batch;) {
      if (sums_bits[i] != kSentinel) {
        ++i;
        continue;
      }
      if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) {
        NK_HIP(hipStreamSynchronize(st));
        break;
      }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return NK_OK;
  };
  // the step at which a matrix may try the Newton-Schulz test: once its
  // relative change has fallen below this (earlier tests would only fail)
  const double ns_try = 0.05;
  for (int it = 1; it <= maxit; ++it) {
    bool any = false;
    for (int b = 0; b < batch; ++b) any = any || act_h[b];
    if (!any) break;
    // 1. the Newton-Schulz test (and its first product) for matrices in the
    //    tail or close enough to try it: T = 3 I - S^2, |I - S^2|_F
    bool anytry = false;
    for (int b = 0; b < batch; ++b) {
      try_h[b] = (ns_on && act_h[b] && (ns_h[b] || prev[b] < ns_try)) ? 1 : 0;
      anytry = anytry || try_h[b];
    }
    if (anytry) {
      if (int e = upload(act_ns, pin_ns, try_h, dev_ns)) return e;
      hipLaunchKernelGGL(k_ns_gemm<0>, dim3(ntile, ntile, batch), dim3(256), 0, st, ld, nvec, act_ns, S, S,
                         g_G0.as<C64>(), nspart);
      NK_HIP(hipGetLastError());
      // only a matrix not yet in the tail waits for its test: inside it
      // |I - S^2|_F only falls (see above), so the product is all it needs
      bool wait = false;
      for (int b = 0; b < batch; ++b) wait = wait || (try_h[b] && !ns_h[b]);
      if (wait) {
        if (int e = sums()) return e;
        for (int b = 0; b < batch; ++b)
          if (try_h[b] && !ns_h[b]) ns_h[b] = std::sqrt(sums_h[b * 4 + 2]) < 0.5 ? 1 : 0;
      }
    }
    bool anyns = false, anygj = false;
    for (int b = 0; b < batch; ++b) {
      const int nsb = act_h[b] && ns_h[b];
      try_h[b] = nsb;
      gj_h[b] = act_h[b] && !nsb;
      anyns = anyns || nsb;
      anygj = anygj || gj_h[b];
    }
    // 2. Newton-Schulz step: G1 = S (3 I - S^2) / 2, then S <- G1
    if (anyns) {
      if (int e = upload(act_ns, pin_ns, try_h, dev_ns)) return e;
      hipLaunchKernelGGL(k_ns_gemm<1>, dim3(ntile, ntile, batch), dim3(256), 0, st, ld, nvec, act_ns, S,
                         g_G0.as<C64>(), g_G1.as<C64>(), nspart);
      hipLaunchKernelGGL(k_ns_copy, dim3(64, batch), dim3(256), 0, st, ld, nvec, act_ns, g_G1.as<C64>(), S);
      NK_HIP(hipGetLastError());
    }
    // 3. inversion step: S <- (mu S + (mu S)^{-1}) / 2 (the learned factor of
    //    step it - 1 read from the device schedule)
    if (anygj) {
      if (int e = upload(act, pin_gj, gj_h, dev_act)) return e;
      const int nbw = gj_nb(ld);
      launch_inverse_shape(shape, batch, ld, maxn, nvec, act, S, g_G0.as<C64>(), g_G1.as<C64>(), rowof, posof, logdet,
                           sing, st);
      const int rs = scaling == NK_RH_LEARNED ? NK_RH_LEARNED : (scaling == NK_RH_DET ? NK_RH_DET : NK_RH_NONE);
      hipLaunchKernelGGL(k_gjcombine, dim3(nbl, batch), dim3(256), 0, st, ld, nbw, nvec, act, g_G0.as<C64>(),
                         g_G1.as<C64>(), S, rowof, posof, logdet, rs, mdev, mu_steps, it - 1, part);
      NK_HIP(hipGetLastError());
    }
    if (int e = sums()) return e;
    for (int b = 0; b < batch; ++b) {
      if (!act_h[b]) continue;
      const double d = ns_h[b] ? sums_h[b * 4 + 2] : sums_h[b * 4 + 0];
      const double nn = ns_h[b] ? sums_h[b * 4 + 3] : sums_h[b * 4 + 1];
      const double change = std::sqrt(d / nn);
      iters_host[b] = it;
      if (!(change > tol) || (change < 1e-6 && change > 0.5 * prev[b])) act_h[b] = 0;
      prev[b] = change;
    }
  }
  NK_HIP(hipMemcpyAsync(pin_state, sing, batch * sizeof(int), hipMemcpyDeviceToHost, st));
  if (resid_host)
    if (int e = rh_residuals(batch, maxn, ld, nvec, S, resid_host, st)) return e;
  NK_HIP(hipStreamSynchronize(st));
  for (int b = 0; b < batch; ++b)
    if (act_h[b] && !pin_state[b]) pin_state[b] = 2;  // still active after maxit iterations
  return rh_outcome(batch, pin_state, maxit);
}

}  // namespace nk
