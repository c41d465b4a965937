// Roberts-Higham iteration S_{n+1} = (S_n + S_n^{-1}) / 2 (Eq. (4)) for a
// batch of dense complex matrices of uneven sizes, on gfx950.
//
// The inverse is an out-of-place blocked Gauss-Jordan elimination with
// partial pivoting.  For each panel of NB columns:
//  * k_gj_panel (one 1024-thread workgroup per matrix) eliminates the panel
//    columns in registers: pivot search over the rows not yet used, row
//    bookkeeping in LDS (the rows themselves are not moved), and writes the
//    transformed panel M in pivot order plus the panel's row permutation;
//  * k_gj_update applies the rank-NB update to every other column,
//      new[pos][j] = (pos in panel ? 0 : old[src(pos)][j]) + sum_t M[pos][t] old[src(c0 + t)][j],
//    reading the previous buffer and writing the other one (ping-pong), so
//    no workgroup ever reads a row another one is writing.
// The panel's thread count (and so rows per thread) and the update's tile
// are chosen per matrix-size class by timing every feasible pair once (the
// autotuner below); none of them changes the arithmetic: the pivot is the
// largest candidate with ties to the smaller position whatever the thread
// count, and every element sums its panel terms in the same order whatever
// the tile, so the choice never changes a bit of the result.
// k_rh_combine undoes the accumulated row permutation as a column
// permutation of the inverse, forms the average (optionally with a positive
// scale mu, which leaves the limit unchanged) and emits partial sums of
// |S_{n+1} - S_n|_F^2 and |S_{n+1}|_F^2 for the host's stopping test.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

#include "nk_internal.h"

namespace nk {

constexpr int PT = 1024;  // largest panel thread count
constexpr int UT = 256;   // update threads (16 x 16), each (T / 16)^2 elements of a T x T tile

__device__ __forceinline__ double cabs1(C64 a) { return fabs(a.re) + fabs(a.im); }

__device__ __forceinline__ C64 cinv(C64 a) {
  // 1 / a, scaled to avoid overflow in |a|^2
  const double s = fmax(fabs(a.re), fabs(a.im));
  const double ar = a.re / s, ai = a.im / s;
  const double d = (ar * ar + ai * ai) * s;
  return mk(ar / d, -ai / d);
}

template <int NB, int RM, int PTH>
__global__ void __launch_bounds__(PTH) k_gj_panel(int ld, const int* __restrict__ nvec, const int* __restrict__ active,
                                                 int c0, const C64* __restrict__ Aold_b, C64* __restrict__ Anew_b,
                                                 int* __restrict__ p2r_b, int* __restrict__ perm_b,
                                                 double* __restrict__ logdet, int* __restrict__ sing) {
  const int b = blockIdx.x;
  const int n = nvec[b];
  if (!active[b] || c0 >= n) return;
  const int nbe = min(NB, n - c0);
  const size_t off = (size_t)b * ld * ld;
  const C64* Aold = Aold_b + off;
  C64* Anew = Anew_b + off;
  int* p2r = p2r_b + (size_t)b * ld;
  int* perm = perm_b + (size_t)b * ld;

  __shared__ int s_p2r[PTH * RM];
  __shared__ int s_r2p[PTH * RM];
  __shared__ C64 s_prow[NB];
  __shared__ double s_val[PTH / 64];
  __shared__ int s_pos[PTH / 64];
  __shared__ double s_ld;
  __shared__ int s_sing;

  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  C64 a[RM][NB];
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    const int r = tid + m * PTH;
#pragma unroll
    for (int t = 0; t < NB; ++t) a[m][t] = (r < n && t < nbe) ? Aold[(size_t)r * ld + c0 + t] : mk(0.0, 0.0);
  }
  for (int r = tid; r < n; r += PTH) {
    s_p2r[r] = r;
    s_r2p[r] = r;
  }
  if (tid == 0) {
    s_ld = 0.0;
    s_sing = 0;
  }
  __syncthreads();

#pragma unroll
  for (int t = 0; t < NB; ++t) {
    if (t < nbe) {
      const int c = c0 + t;
      double best = -1.0;
      int bpos = 0x7fffffff;
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        const int r = tid + m * PTH;
        if (r < n) {
          const int pos = s_r2p[r];
          double v = cabs1(a[m][t]);
          if (!(v >= 0.0)) v = 0.0;  // a NaN entry counts as a zero pivot, so some row is always chosen
          if (pos >= c && (v > best || (v == best && pos < bpos))) {
            best = v;
            bpos = pos;
          }
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(best, o, 64);
        const int op = __shfl_xor(bpos, o, 64);
        if (ov > best || (ov == best && op < bpos)) {
          best = ov;
          bpos = op;
        }
      }
      if (lane == 0) {
        s_val[wid] = best;
        s_pos[wid] = bpos;
      }
      __syncthreads();
      best = s_val[0];
      bpos = s_pos[0];
#pragma unroll
      for (int w = 1; w < PTH / 64; ++w) {
        const double ov = s_val[w];
        const int op = s_pos[w];
        if (ov > best || (ov == best && op < bpos)) {
          best = ov;
          bpos = op;
        }
      }
      const int p = bpos < n ? bpos : c;  // (position c is always a candidate)
      const int pr = s_p2r[p];
      const int rc = s_p2r[c];
      if ((pr & (PTH - 1)) == tid) {
#pragma unroll
        for (int m = 0; m < RM; ++m) {
          if (m == pr / PTH) {
            const C64 piv = a[m][t];
            // a zero pivot flags the matrix as singular; the elimination
            // goes on with a zero multiplier instead of 1/0, so no NaN
            // spreads through the rest of the panel
            const bool nz = best > 0.0;
            if (!nz) s_sing = 1;
            const C64 d = nz ? cinv(piv) : mk(0.0, 0.0);
            if (nz) s_ld += log(sqrt(piv.re * piv.re + piv.im * piv.im));
#pragma unroll
            for (int u = 0; u < NB; ++u) s_prow[u] = (u == t) ? d : cmul(a[m][u], d);
          }
        }
      }
      __syncthreads();
      if (tid == 0) {
        s_p2r[c] = pr;
        s_p2r[p] = rc;
        s_r2p[pr] = c;
        s_r2p[rc] = p;
      }
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        const int r = tid + m * PTH;
        if (r < n) {
          if (r == pr) {
#pragma unroll
            for (int u = 0; u < NB; ++u) a[m][u] = s_prow[u];
          } else {
            const C64 f = a[m][t];
#pragma unroll
            for (int u = 0; u < NB; ++u) {
              const C64 base = (u == t) ? mk(0.0, 0.0) : a[m][u];
              a[m][u] = base - cmul(f, s_prow[u]);
            }
          }
        }
      }
      __syncthreads();
    }
  }
  // M in pivot order, the panel's position -> source-row map, the running permutation
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    const int r = tid + m * PTH;
    if (r < n) {
      const int pos = s_r2p[r];
#pragma unroll
      for (int t = 0; t < NB; ++t)
        if (t < nbe) Anew[(size_t)pos * ld + c0 + t] = a[m][t];
    }
  }
  int pv[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    const int pos = tid + m * PTH;
    pv[m] = pos < n ? perm[s_p2r[pos]] : 0;
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    const int pos = tid + m * PTH;
    if (pos < n) {
      perm[pos] = pv[m];
      p2r[pos] = s_p2r[pos];
    }
  }
  if (tid == 0) {
    logdet[b] += s_ld;
    if (s_sing) sing[b] = 1;
  }
}

template <int NB, int T>
__global__ void __launch_bounds__(UT) k_gj_update(int ld, const int* __restrict__ nvec, const int* __restrict__ active,
                                                  int c0, const C64* __restrict__ Aold_b, C64* __restrict__ Anew_b,
                                                  const int* __restrict__ p2r_b) {
  const int b = blockIdx.z;
  const int n = nvec[b];
  if (!active[b] || c0 >= n) return;
  constexpr int E = T / 16;  // rows and columns per thread
  const int row0 = blockIdx.y * T, col0 = blockIdx.x * T;
  if (row0 >= n || col0 >= n) return;
  const int nbe = min(NB, n - c0);
  const size_t off = (size_t)b * ld * ld;
  const C64* Aold = Aold_b + off;
  C64* Anew = Anew_b + off;
  const int* p2r = p2r_b + (size_t)b * ld;
  __shared__ C64 sM[T][NB + 1];
  __shared__ C64 sR[NB][T + 1];
  __shared__ int sP[T];
  const int tid = threadIdx.x;
  for (int e = tid; e < T * NB; e += UT) {
    const int i = e / NB, t = e % NB;
    const int pos = row0 + i;
    sM[i][t] = (pos < n && t < nbe) ? Anew[(size_t)pos * ld + c0 + t] : mk(0.0, 0.0);
  }
  for (int e = tid; e < T * NB; e += UT) {
    const int t = e / T, j = e % T;
    const int col = col0 + j;
    sR[t][j] = (t < nbe && col < n) ? Aold[(size_t)p2r[c0 + t] * ld + col] : mk(0.0, 0.0);
  }
  if (tid < T) sP[tid] = (row0 + tid < n) ? p2r[row0 + tid] : 0;
  __syncthreads();
  const int tx = tid & 15, ty = tid >> 4;
#pragma unroll
  for (int ii = 0; ii < E; ++ii) {
    const int i = ty * E + ii;
    const int pos = row0 + i;
    if (pos >= n) continue;
    const bool inpanel = pos >= c0 && pos < c0 + nbe;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int j = tx + 16 * q;
      const int col = col0 + j;
      if (col >= n || (col >= c0 && col < c0 + nbe)) continue;
      C64 acc = inpanel ? mk(0.0, 0.0) : Aold[(size_t)sP[i] * ld + col];
#pragma unroll
      for (int t = 0; t < NB; ++t) acc = acc + cmul(sM[i][t], sR[t][j]);
      Anew[(size_t)pos * ld + col] = acc;
    }
  }
}

__global__ void k_rh_start(int ld, int batch, const int* __restrict__ nvec, const int* __restrict__ active,
                           int* __restrict__ perm_b, double* __restrict__ logdet) {
  const int b = blockIdx.y;
  if (!active[b]) return;
  const int n = nvec[b];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    perm_b[(size_t)b * ld + i] = i;
  if (blockIdx.x == 0 && threadIdx.x == 0) logdet[b] = 0.0;
}

// G0/G1: the ping-pong buffers; a matrix of order n ends its elimination in
// the buffer of its own last panel, (ceil(n / nb) - 1) % 2.
__global__ void __launch_bounds__(256) k_rh_combine(int ld, int nb, const int* __restrict__ nvec,
                                                    const int* __restrict__ active, const C64* __restrict__ G0,
                                                    const C64* __restrict__ G1,
                                                    C64* __restrict__ X_b, const int* __restrict__ perm_b,
                                                    const double* __restrict__ logdet, int scaling,
                                                    const double* __restrict__ mu_in, double* __restrict__ part) {
  const int b = blockIdx.y;
  const int n = nvec[b];
  double dsum = 0.0, nsum = 0.0;
  if (active[b]) {
    double mu = 1.0;
    if (scaling == NK_RH_DET || scaling == NK_RH_LEARNED) mu = exp(-logdet[b] / n);
    if (scaling == NK_RH_LEARNED && mu_in && mu_in[b] > 0.0) mu *= mu_in[b];  // learned correction
    const double imu = 1.0 / mu;
    const size_t off = (size_t)b * ld * ld;
    const int npan = (n + nb - 1) / nb;
    const C64* G = (((npan - 1) & 1) ? G1 : G0) + off;
    C64* X = X_b + off;
    const int* perm = perm_b + (size_t)b * ld;
    const size_t nn = (size_t)n * n;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < nn; e += (size_t)gridDim.x * 256) {
      const int i = (int)(e / n), p = (int)(e % n);
      const size_t xi = (size_t)i * ld + perm[p];
      const C64 xs = mu * X[xi];
      const C64 s = 0.5 * (xs + imu * G[(size_t)i * ld + p]);
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

// r_b = |S (S e_1) - e_1| per matrix (one workgroup per matrix)
__global__ void __launch_bounds__(256) k_rh_resid(int ld, const int* __restrict__ nvec, const C64* __restrict__ S_b,
                                                  double* __restrict__ out) {
  const int b = blockIdx.x;
  const int n = nvec[b];
  const C64* S = S_b + (size_t)b * ld * ld;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    C64 t = mk(0.0, 0.0);
    for (int j = 0; j < n; ++j) t = t + cmul(S[(size_t)i * ld + j], S[(size_t)j * ld]);
    if (i == 0) t.re -= 1.0;
    acc += norm2(t);
  }
  __shared__ double sh[4];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[b] = sqrt((sh[0] + sh[1]) + (sh[2] + sh[3]));
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

template <int SQ>  // rows per thread; n <= 4 SQ
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
      key = __reduce_max_sync(~0ull, key);
      // every unused row has a nonzero key, and one is unused while t < n; the
      // fallback only keeps the index in range should that ever not hold
      const int pr = key ? 255 - (int)(key & 255u) : t;
      const C64 pv = s_col[par][pr];
      if (!(fabs(pv.re) + fabs(pv.im) > 0.0)) bad = 1;
      const C64 d = cinv(pv);
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
DevBuf g_G0, g_G1, g_int, g_dbl, g_mu, g_sched;
}  // namespace

template <int NB, int RM, int PTH, int T>
static void launch_inverse(int batch, int ld, int maxn, const int* nvec, const int* act, const C64* S, C64* G0,
                           C64* G1, int* p2r, int* perm, double* logdet, int* sing, hipStream_t st) {
  const C64* cur = S;
  int which = 0;
  const int tiles = (maxn + T - 1) / T;
  for (int c0 = 0; c0 < maxn; c0 += NB) {
    C64* nxt = which ? G1 : G0;
    hipLaunchKernelGGL((k_gj_panel<NB, RM, PTH>), dim3(batch), dim3(PTH), 0, st, ld, nvec, act, c0, cur, nxt, p2r,
                       perm, logdet, sing);
    hipLaunchKernelGGL((k_gj_update<NB, T>), dim3(tiles, tiles, batch), dim3(UT), 0, st, ld, nvec, act, c0, cur, nxt,
                       p2r);
    cur = nxt;
    which ^= 1;
  }
}

// The launch shapes of the blocked inverse: panel threads x rows per thread
// (which must cover ld) and the update tile.  The panel width is not among
// the choices: it sets the grouping of the update sums, 16 up to ld = 1024
// and 8 above, fixed by ld alone.
struct GJShape {
  int nb, rm, pth, tile;
};
// every instantiated shape (the panel keeps rm x nb complex values per
// thread in registers, so rm x nb x 4 VGPRs must fit beside the rest at
// pth / 256 waves per SIMD; 4 rows of 16 would live in scratch memory)
#define NK_GJ_SHAPES(X)                                                                                      \
  X(16, 1, 256, 32) X(16, 1, 256, 64) X(16, 1, 512, 32) X(16, 1, 512, 64) X(16, 1, 1024, 32)                \
  X(16, 1, 1024, 64) X(16, 2, 256, 32) X(16, 2, 256, 64) X(16, 2, 512, 32) X(16, 2, 512, 64)                \
  X(8, 2, 1024, 32) X(8, 2, 1024, 64) X(8, 4, 512, 32)                                                      \
  X(8, 4, 512, 64) X(8, 4, 1024, 32) X(8, 4, 1024, 64)
#define NK_GJ_ENTRY(NB, RM, PTH, T) {NB, RM, PTH, T},
constexpr GJShape kGJShapes[] = {NK_GJ_SHAPES(NK_GJ_ENTRY)};
#undef NK_GJ_ENTRY

static int gj_nb(int ld) { return ld <= PT ? 16 : 8; }

static bool gj_feasible(const GJShape& sh, int ld) {
  for (const GJShape& k : kGJShapes)
    if (k.nb == sh.nb && k.rm == sh.rm && k.pth == sh.pth && k.tile == sh.tile)
      return sh.nb == gj_nb(ld) && sh.pth * sh.rm >= ld;
  return false;
}

// one blocked inverse with a shape that gj_feasible accepts for ld
static void launch_inverse_shape(const GJShape& sh, int batch, int ld, int maxn, const int* nvec, const int* act,
                                 const C64* S, C64* G0, C64* G1, int* p2r, int* perm, double* logdet, int* sing,
                                 hipStream_t st) {
#define NK_GJ_CALL(NB, RM, PTH, T)                                                                            \
  if (sh.nb == NB && sh.rm == RM && sh.pth == PTH && sh.tile == T)                                            \
    return launch_inverse<NB, RM, PTH, T>(batch, ld, maxn, nvec, act, S, G0, G1, p2r, perm, logdet, sing, st);
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
                     int* p2r, int* perm, double* logdet, int* sing, hipStream_t st, GJShape* out) {
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
      hipLaunchKernelGGL(k_rh_start, dim3((maxn + 255) / 256, batch), dim3(256), 0, st, ld, batch, nvec, act, perm,
                         logdet);
      NK_HIP(hipEventRecord(e0, st));
      launch_inverse_shape(sh, batch, ld, maxn, nvec, act, S, G0, G1, p2r, perm, logdet, sing, st);
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
      g_dbl.ensure((size_t)batch * (2 * nbl + 4) * sizeof(double)) || g_mu.ensure((size_t)batch * sizeof(double)))
    return NK_ENOMEM;
  int* nvec = g_int.as<int>();
  int* act = nvec + batch;
  int* sing = act + batch;
  int* p2r = sing + batch;
  int* perm = p2r + (size_t)batch * ld;
  double* logdet = g_dbl.as<double>();
  double* resid = logdet + batch;
  double* part = resid + batch;
  double* mu_dev = g_mu.as<double>();

  int maxn = 0;
  std::vector<int> act_h(batch), zeros(batch, 0);
  for (int b = 0; b < batch; ++b) maxn = std::max(maxn, n_host[b]);
  NK_HIP(hipMemcpyAsync(nvec, n_host, batch * sizeof(int), hipMemcpyHostToDevice, st));
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
    NK_HIP(hipMemcpyAsync(sing, zeros.data(), batch * sizeof(int), hipMemcpyHostToDevice, st));
    int rps = 0;  // largest rows-per-thread over the batch
    for (int b = 0; b < batch; ++b)
      if (n_host[b] > 0) rps = std::max(rps, (n_host[b] + ST_RH / n_host[b] - 1) / (ST_RH / n_host[b]));
    if (rps <= 16)
      hipLaunchKernelGGL(k_rh_small<16>, dim3(batch), dim3(ST_RH), 0, st, ld, nvec, S, scaling, mdev, mu_steps, maxit,
                         tol, act, sing);
    else
      hipLaunchKernelGGL(k_rh_small<32>, dim3(batch), dim3(ST_RH), 0, st, ld, nvec, S, scaling, mdev, mu_steps, maxit,
                         tol, act, sing);
    NK_HIP(hipGetLastError());
    std::vector<int> sing_h(batch);
    NK_HIP(hipMemcpyAsync(iters_host, act, batch * sizeof(int), hipMemcpyDeviceToHost, st));
    NK_HIP(hipMemcpyAsync(sing_h.data(), sing, batch * sizeof(int), hipMemcpyDeviceToHost, st));
    if (resid_host) {
      hipLaunchKernelGGL(k_rh_resid, dim3(batch), dim3(256), 0, st, ld, nvec, S, resid);
      NK_HIP(hipMemcpyAsync(resid_host, resid, batch * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    NK_HIP(hipStreamSynchronize(st));
    return rh_outcome(batch, sing_h.data(), maxit);
  }
  maxn = 0;
  for (int b = 0; b < batch; ++b) {
    maxn = std::max(maxn, n_host[b]);
    act_h[b] = n_host[b] > 0 ? 1 : 0;
    iters_host[b] = 0;
  }
  NK_HIP(hipMemcpyAsync(act, act_h.data(), batch * sizeof(int), hipMemcpyHostToDevice, st));
  GJShape shape;
  if (int e = gj_choose(batch, ld, maxn, nvec, act, S, g_G0.as<C64>(), g_G1.as<C64>(), p2r, perm, logdet, sing, st,
                        &shape))
    return e;
  NK_HIP(hipMemcpyAsync(sing, zeros.data(), batch * sizeof(int), hipMemcpyHostToDevice, st));
  std::vector<double> prev(batch, INFINITY), part_h((size_t)batch * nbl * 2), mu_h(batch, 1.0);
  std::vector<double> sched_h;
  if (mdev) {
    sched_h.resize((size_t)batch * mu_steps);
    NK_HIP(hipMemcpyAsync(sched_h.data(), mdev, sched_h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    NK_HIP(hipStreamSynchronize(st));
  }
  for (int it = 1; it <= maxit; ++it) {
    bool any = false;
    for (int b = 0; b < batch; ++b) any = any || act_h[b];
    if (!any) break;
    NK_HIP(hipMemcpyAsync(act, act_h.data(), batch * sizeof(int), hipMemcpyHostToDevice, st));
    if (scaling == NK_RH_LEARNED) {
      for (int b = 0; b < batch; ++b)
        mu_h[b] = (mdev && it - 1 < mu_steps) ? sched_h[(size_t)b * mu_steps + (it - 1)] : -1.0;
      NK_HIP(hipMemcpyAsync(mu_dev, mu_h.data(), batch * sizeof(double), hipMemcpyHostToDevice, st));
    }
    hipLaunchKernelGGL(k_rh_start, dim3((maxn + 255) / 256, batch), dim3(256), 0, st, ld, batch, nvec, act, perm,
                       logdet);
    const int nbw = gj_nb(ld);
    launch_inverse_shape(shape, batch, ld, maxn, nvec, act, S, g_G0.as<C64>(), g_G1.as<C64>(), p2r, perm, logdet,
                         sing, st);
    const int rs = scaling == NK_RH_LEARNED ? NK_RH_LEARNED : (scaling == NK_RH_DET ? NK_RH_DET : NK_RH_NONE);
    hipLaunchKernelGGL(k_rh_combine, dim3(nbl, batch), dim3(256), 0, st, ld, nbw, nvec, act, g_G0.as<C64>(),
                       g_G1.as<C64>(), S, perm, logdet, rs, mu_dev, part);
    NK_HIP(hipGetLastError());
    NK_HIP(hipMemcpyAsync(part_h.data(), part, part_h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    NK_HIP(hipStreamSynchronize(st));
    for (int b = 0; b < batch; ++b) {
      if (!act_h[b]) continue;
      double d = 0.0, nn = 0.0;
      for (int i = 0; i < nbl; ++i) {
        d += part_h[((size_t)b * nbl + i) * 2 + 0];
        nn += part_h[((size_t)b * nbl + i) * 2 + 1];
      }
      const double change = std::sqrt(d / nn);
      iters_host[b] = it;
      if (!(change > tol) || (change < 1e-6 && change > 0.5 * prev[b])) act_h[b] = 0;
      prev[b] = change;
    }
  }
  std::vector<int> sing_h(batch);
  NK_HIP(hipMemcpyAsync(sing_h.data(), sing, batch * sizeof(int), hipMemcpyDeviceToHost, st));
  if (resid_host) {
    hipLaunchKernelGGL(k_rh_resid, dim3(batch), dim3(256), 0, st, ld, nvec, S, resid);
    NK_HIP(hipMemcpyAsync(resid_host, resid, batch * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  NK_HIP(hipStreamSynchronize(st));
  for (int b = 0; b < batch; ++b)
    if (act_h[b] && !sing_h[b]) sing_h[b] = 2;  // still active after maxit iterations
  return rh_outcome(batch, sing_h.data(), maxit);
}

}  // namespace nk
