// The small problem of the sign approximation on gfx950: the k-vector z with
// sgn(A) x ~ ||x|| V_k z.
//
//  ell == 0 (non-nested, Eqs. (3)-(4)): z = sgn(H_k) e_1 by Roberts-Higham on
//  the dense k x k Ritz matrix.
//  ell  > 0 (nested, Sec. 3, Eqs. (5)-(6)): B = H_k + H_k^{-1}; an inner
//  Krylov space K_l(B, e_1) (Lanczos for Hermitian H_k, two-sided Lanczos
//  otherwise, full re-(bi)orthogonalisation); z = V_l sgn(H_l) e_1.
//
// H_k^{-1} comes from one LU factorisation of the tridiagonal H_k with
// partial pivoting (U has two super-diagonals), after which k threads solve
// H x = e_j for every column j at once and write B densely; the inner
// iteration then only needs dense mat-vecs with B (and B^dag), which spread
// over the whole GPU, instead of k-long sequential solves inside its loop.
#include <algorithm>
#include <cmath>
#include <vector>

#include "hostbuf.h"
#include "nk_internal.h"

namespace nk {

constexpr int ST = 256;

__device__ __forceinline__ double cabs1s(C64 a) { return fabs(a.re) + fabs(a.im); }
// 1 / b = conj(b) / |b|^2 with b first scaled by a power of two (exact) so
// that |b|^2 neither overflows nor underflows: one division on the
// recurrence's critical path instead of cdiv's four
__device__ __forceinline__ C64 crecip(C64 b) {
  int e;
  (void)frexp(fmax(fabs(b.re), fabs(b.im)), &e);
  const double br = ldexp(b.re, -e), bi = ldexp(b.im, -e);
  const double q = 1.0 / (br * br + bi * bi);
  return mk(ldexp(br * q, -e), ldexp(-bi * q, -e));
}
__device__ __forceinline__ C64 cdiv(C64 a, C64 b) {
  const double s = fmax(fabs(b.re), fabs(b.im));
  const double br = b.re / s, bi = b.im / s;
  const double d = (br * br + bi * bi) * s;
  return mk((a.re * br + a.im * bi) / d, (a.im * br - a.re * bi) / d);
}

// LU with partial pivoting of the tridiagonal H (diag alpha, super beta,
// sub delta).  Row i of U holds 1/U0i[i], U1[i], U2[i] on columns i, i+1, i+2;
// Lm[i] is the multiplier that eliminates column i of the row below the
// pivot row; Sw[i] says whether rows i and i+1 were exchanged.  The
// elimination is sequential (one thread); the coefficients are first staged
// in LDS by the whole block so the loop does not wait on global memory.
constexpr int TRI_LDS_MAX = 1365;  // 3 k complex in LDS (<= 64 KB of dynamic LDS)

// the sequential elimination, with the coefficients read through al/be/de
// (LDS or global: one instantiation each, so every access has its own
// address space)
template <class P>
__device__ __forceinline__ void tri_lu_seq(int k, P al, P be, P de, C64* __restrict__ Lm, int* __restrict__ Sw,
                                           C64* __restrict__ U0i, C64* __restrict__ U1, C64* __restrict__ U2,
                                           int* __restrict__ sing) {
  const C64 z = mk(0.0, 0.0);
  C64 a0 = ldg(al), a1 = k > 1 ? ldg(be) : z, a2 = z;
  int bad = 0;
  for (int i = 0; i + 1 < k; ++i) {
    const C64 b0 = ldg(de + i), b1 = ldg(al + i + 1), b2 = (i + 2 < k) ? ldg(be + i + 1) : z;
    const bool sw = cabs1s(a0) < cabs1s(b0);
    const C64 p0 = sw ? b0 : a0, p1 = sw ? b1 : a1, p2 = sw ? b2 : a2;
    const C64 o0 = sw ? a0 : b0, o1 = sw ? a1 : b1, o2 = sw ? a2 : b2;
    if (!(cabs1s(p0) > 0.0)) bad = 1;
    const C64 inv = crecip(p0);
    const C64 m = cmul(o0, inv);
    U0i[i] = inv;
    U1[i] = p1;
    U2[i] = p2;
    Lm[i] = m;
    Sw[i] = sw ? 1 : 0;
    a0 = o1 - cmul(m, p1);
    a1 = o2 - cmul(m, p2);
    a2 = z;
  }
  if (!(cabs1s(a0) > 0.0)) bad = 1;
  U0i[k - 1] = crecip(a0);
  U1[k - 1] = z;
  U2[k - 1] = z;
  if (k >= 2) U2[k - 2] = z;
  *sing = bad;
}

__global__ void __launch_bounds__(256) k_tri_lu(int k, const C64* __restrict__ alpha, const C64* __restrict__ beta,
                                                const C64* __restrict__ delta, C64* __restrict__ Lm,
                                                int* __restrict__ Sw, C64* __restrict__ U0i, C64* __restrict__ U1,
                                                C64* __restrict__ U2, int* __restrict__ sing) {
  extern __shared__ C64 sm[];
  const bool lds = k <= TRI_LDS_MAX;
  if (lds) {
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
      sm[i] = alpha[i];
      sm[k + i] = i + 1 < k ? beta[i] : mk(0.0, 0.0);
      sm[2 * k + i] = i + 1 < k ? delta[i] : mk(0.0, 0.0);
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  if (lds)
    tri_lu_seq(k, (const C64*)sm, (const C64*)sm + k, (const C64*)sm + 2 * k, Lm, Sw, U0i, U1, U2, sing);
  else
    tri_lu_seq(k, as_global(alpha), as_global(beta), as_global(delta), Lm, Sw, U0i, U1, U2, sing);
}

// column j of H^{-1} (solve H x = e_j), then B = H + H^{-1}; B row-major k x k.
// The factors are staged in LDS when they fit.  The forward sweep of e_j is
// zero before row j - 1, so it starts there.  The backward sweep reads eight
// rows of the forward result ahead of the recurrence (rows below the one
// being written, so the reads never see a row of this sweep), which keeps
// eight loads in flight instead of one.
struct TriF {
  C64 lm, u0i, u1, u2;
};
constexpr int TRI_INV_LDS_MAX = 960;  // k x (64 + 4) B in LDS (<= 64 KB of dynamic LDS)

template <bool LDS>
__device__ __forceinline__ void tri_inv_col(int j, int k, const TriF* sf, const int* ssw, gp<const C64> Lm,
                                            gp<const int> Sw, gp<const C64> U0i, gp<const C64> U1,
                                            gp<const C64> U2, gp<C64> B) {
  const C64 z = mk(0.0, 0.0);
  const int i0 = j > 0 ? j - 1 : 0;
  for (int i = 0; i < i0; ++i) stg(B + (size_t)i * k + j, z);
  C64 fc = (j == 0) ? mk(1.0, 0.0) : z;
  for (int i = i0; i + 1 < k; ++i) {
    const C64 fn = (i + 1 == j) ? mk(1.0, 0.0) : z;
    const int sw = LDS ? ssw[i] : Sw[i];
    const C64 piv = sw ? fn : fc, oth = sw ? fc : fn;
    stg(B + (size_t)i * k + j, piv);
    fc = oth - cmul(LDS ? sf[i].lm : ldg(Lm + i), piv);
  }
  stg(B + (size_t)(k - 1) * k + j, fc);
  C64 x1 = z, x2 = z;
  auto step = [&](int i, C64 y) {
    const C64 u1 = LDS ? sf[i].u1 : ldg(U1 + i), u2 = LDS ? sf[i].u2 : ldg(U2 + i), u0 = LDS ? sf[i].u0i : ldg(U0i + i);
    const C64 xi = cmul(y - cmul(u1, x1) - cmul(u2, x2), u0);
    stg(B + (size_t)i * k + j, xi);
    x2 = x1;
    x1 = xi;
  };
  int i = k - 1;
  for (; i >= 7; i -= 8) {
    C64 y[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) y[u] = ldg(B + (size_t)(i - u) * k + j);
#pragma unroll
    for (int u = 0; u < 8; ++u) step(i - u, y[u]);
  }
  for (; i >= 0; --i) step(i, ldg(B + (size_t)i * k + j));
}

__global__ void __launch_bounds__(64) k_tri_inv(int k, const C64* __restrict__ Lm, const int* __restrict__ Sw,
                                                const C64* __restrict__ U0i, const C64* __restrict__ U1,
                                                const C64* __restrict__ U2, const C64* __restrict__ alpha,
                                                const C64* __restrict__ beta, const C64* __restrict__ delta,
                                                C64* __restrict__ B) {
  extern __shared__ TriF sf[];
  int* ssw = reinterpret_cast<int*>(sf + (k <= TRI_INV_LDS_MAX ? k : 0));
  const bool lds = k <= TRI_INV_LDS_MAX;
  if (lds) {
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
      sf[i].lm = Lm[i];
      sf[i].u0i = U0i[i];
      sf[i].u1 = U1[i];
      sf[i].u2 = U2[i];
      ssw[i] = Sw[i];
    }
    __syncthreads();
  }
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  if (lds)
    tri_inv_col<true>(j, k, sf, ssw, as_global(Lm), as_global(Sw), as_global(U0i), as_global(U1), as_global(U2),
                      as_global(B));
  else
    tri_inv_col<false>(j, k, sf, ssw, as_global(Lm), as_global(Sw), as_global(U0i), as_global(U1), as_global(U2),
                       as_global(B));
  B[(size_t)j * k + j] = B[(size_t)j * k + j] + alpha[j];
  if (j > 0) B[(size_t)(j - 1) * k + j] = B[(size_t)(j - 1) * k + j] + beta[j - 1];
  if (j + 1 < k) B[(size_t)(j + 1) * k + j] = B[(size_t)(j + 1) * k + j] + delta[j];
}

// BH = B^dag (tiled transpose through LDS)
__global__ void k_adjoint(int k, const C64* __restrict__ B, C64* __restrict__ BH) {
  __shared__ C64 t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int yy = threadIdx.y; yy < 32; yy += 8) {
    const int r = by + yy, c = bx + threadIdx.x;
    if (r < k && c < k) t[yy][threadIdx.x] = B[(size_t)r * k + c];
  }
  __syncthreads();
  for (int yy = threadIdx.y; yy < 32; yy += 8) {
    const int r = bx + yy, c = by + threadIdx.x;
    if (r < k && c < k) BH[(size_t)r * k + c] = conj(t[threadIdx.x][yy]);
  }
}

// dense tridiagonal H (ld = k), row-major
__global__ void k_tri_dense(int k, const C64* __restrict__ alpha, const C64* __restrict__ beta,
                            const C64* __restrict__ delta, C64* __restrict__ H) {
  const size_t nn = (size_t)k * k;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / k), j = (int)(e % k);
    C64 v = mk(0.0, 0.0);
    if (i == j) v = alpha[i];
    else if (j == i + 1) v = beta[i];
    else if (i == j + 1) v = delta[j];
    H[e] = v;
  }
}

// ---------------------------------------------------------------------------
// inner Krylov on dense B: three launches per step.
//  k_in_gemv : normalise the previous raw vectors (from partial sums), store
//              v_i / w_i, u = B v_i - beta v_{i-1}, q = B^dag w_i - delta w_{i-1}
//              (one wave per row), and the partial first-pass projections
//              W^dag u, V^dag q over the block's GR rows;
//  k_in_sub  : reduce the partial projections, subtract (u -= V c, q -= W d;
//              eight lanes per row), then emit either the partial projections
//              of the second Gram-Schmidt pass or the partial sums of
//              s = q^dag u, |u|^2, |q|^2 for the next normalisation.
// V, W column-major (column j at j*k).  Hermitian: one side, W = V, q = u.
// Arnoldi: the one-sided form on a general B, with every projection
// coefficient kept (column i of the Hessenberg H_l, both passes summed).
constexpr int GR = 16;  // rows per k_in_gemv block (one wave each, 1024 threads)
constexpr int LMAX = 512;  // largest inner size (LDS of k_in_sub)
constexpr int SR = 32;  // rows per k_in_sub block (eight lanes each)

struct Inner {
  int k, herm, lmax;
  const C64* B;
  const C64* BH;
  C64* V;
  C64* W;
  C64* uraw[2];  // ping-pong raw vectors (u side)
  C64* qraw[2];  // (q side)
  C64* part1;    // [2][nb1][lmax] partial projections from k_in_gemv
  C64* part2;    // [2][nb2][lmax] second-pass partial projections
  double* part3; // [4][nb2] normalisation partial sums
  int nb1, nb2;
  C64* a;
  C64* b;
  C64* d;
  int* flags;
  C64* hcol;     // [lmax][lmax] Arnoldi: column i of H_l at i * lmax (both passes summed)
  int arnoldi;   // 1: one-sided recurrence on a general B, every coefficient kept
};

// the descriptor with its buffers seen as global memory (see as_global)
struct InnerG {
  int k, herm, lmax, nb1, nb2;
  gp<const C64> B, BH;
  gp<C64> V, W, u0, u1, q0, q1, part1, part2, a, b, d;  // u0/u1, q0/q1: the raw ping-pong vectors
  gp<double> part3;
  gp<int> flags;
  gp<C64> hcol;
  int arnoldi;
};

__device__ __forceinline__ InnerG inner_view(const Inner& s) {
  InnerG g;
  g.k = s.k;
  g.herm = s.herm;
  g.lmax = s.lmax;
  g.nb1 = s.nb1;
  g.nb2 = s.nb2;
  g.B = as_global(s.B);
  g.BH = as_global(s.BH);
  g.V = as_global(s.V);
  g.W = as_global(s.W);
  g.u0 = as_global(s.uraw[0]);
  g.u1 = as_global(s.uraw[1]);
  g.q0 = as_global(s.qraw[0]);
  g.q1 = as_global(s.qraw[1]);
  g.part1 = as_global(s.part1);
  g.part2 = as_global(s.part2);
  g.part3 = as_global(s.part3);
  g.a = as_global(s.a);
  g.b = as_global(s.b);
  g.d = as_global(s.d);
  g.flags = as_global(s.flags);
  g.hcol = as_global(s.hcol);
  g.arnoldi = s.arnoldi;
  return g;
}

// The descriptor of this block's problem: a kernel argument (read straight
// from the kernel-argument segment, one round trip less) for a single
// problem, entry blockIdx.z of a device array for a batch.
template <bool BATCH>
__device__ __forceinline__ const Inner& inner_desc(const Inner& s0, const Inner* SS) {
  if constexpr (BATCH)
    return SS[blockIdx.z];
  else
    return s0;
}

// c ? a : b for two fields of a local descriptor.  A plain select of two
// fields lets the compiler turn it into one load through a selected address,
// which keeps the whole descriptor in scratch memory; passing both values
// through an empty asm first leaves a select of registers.
template <class T>
__device__ __forceinline__ T pick(bool c, T a, T b) {
  asm volatile("" : "+s"(a), "+s"(b));
  return c ? a : b;
}

// raw vector h (0/1) of the u side (q = 0) or the q side (q = 1)
__device__ __forceinline__ gp<C64> rawv(const InnerG& g, int q, int h) {
  return pick(q != 0, pick(h != 0, g.q1, g.q0), pick(h != 0, g.u1, g.u0));
}

template <int NTH>
__device__ __forceinline__ void bsum(double (&v)[4]) {
  __shared__ double sh[4][NTH / 64];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < 4; ++q) sh[q][threadIdx.x >> 6] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NTH / 64; ++w) t += sh[q][w];
    v[q] = t;
  }
}

// bsum when only the first wave holds nonzero terms (nb <= 64 partial sums,
// thread t holding partial t): that wave alone reduces and shares the sums,
// which equal bsum's (the other waves would add zeros)
template <int NTH>
__device__ __forceinline__ void bsum_first(double (&v)[4], int nb) {
  if (nb > 64) {
    bsum<NTH>(v);
    return;
  }
  __shared__ double sh1[4];
  if (threadIdx.x < 64) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
    if (threadIdx.x == 0)
#pragma unroll
      for (int q = 0; q < 4; ++q) sh1[q] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = sh1[q];
}

// Every inner kernel serves a batch of independent problems: problem
// blockIdx.z is SS[blockIdx.z]; the grid is sized for the largest, and a
// workgroup beyond its own problem's size or steps returns at once.
// Everything a block loads except the normalisation scale is known at launch
// (the row of B, the previous raw vector, the old basis entry and the
// projection columns), so it is all issued before the partial sums of the
// previous step are reduced: one memory round trip instead of four.  Each
// wave multiplies its own row's new entry into the projection columns and
// leaves the products in LDS; they are summed over the block's rows in row
// order, as a single thread summing them would.
constexpr int GP = 2;  // projection columns per lane loaded at launch (j < 128)

template <bool BATCH>
__global__ void __launch_bounds__(GR * 64) k_in_gemv(const Inner s0, const Inner* __restrict__ SS, int i) {
  extern __shared__ C64 s_p[];  // [GR][i + 1] per-row projection products
  const Inner& S = inner_desc<BATCH>(s0, SS);
  const InnerG s = inner_view(S);
  // a batch launch covers the largest problem; a single problem is launched
  // for exactly its own steps and blocks
  if (BATCH && (i >= s.lmax || (int)blockIdx.x >= s.nb1)) return;
  const int k = s.k;
  const int side = blockIdx.y;  // 0: u = B v, 1: q = B^dag w
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = blockIdx.x * GR + wave;
  const bool live = r < k;
  const int rs = live ? r : 0;  // rows past k load row 0 and discard it
  // the side-dependent pointers come straight from the descriptor: selected
  // copies of the local view would keep that view in scratch memory
  const int h = i & 1;
  C64* const r0 = side ? S.qraw[0] : S.uraw[0];
  C64* const r1 = side ? S.qraw[1] : S.uraw[1];
  gp<const C64> src = as_global((const C64*)(h ? r1 : r0));
  gp<C64> dst = as_global(h ? r0 : r1);
  gp<const C64> M = as_global(side ? S.BH : S.B);
  gp<C64> basis = as_global(side ? S.W : S.V);
  const bool other = !s.herm;
  gp<const C64> proj = as_global((const C64*)(s.herm ? S.V : (side ? S.V : S.W)));
  gp<const C64> osrc = as_global((const C64*)(side ? (h ? S.uraw[1] : S.uraw[0]) : (h ? S.qraw[1] : S.qraw[0])));
  // loads issued at launch: eight columns of the row and of the raw vector
  // per lane (clamped to column 0 past the end), this row's raw entries, the
  // old basis entry and up to GP projection columns per lane
  C64 mv[8], xv[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int c = lane + 64 * u, cc = c < k ? c : 0;
    mv[u] = ldg(M + (size_t)rs * k + cc);
    xv[u] = ldg(src + cc);
  }
  const C64 xr_raw = ldg(src + rs);
  const C64 xo_raw = ldg(osrc + rs);
  const C64 vold = ldg(basis + (size_t)(i > 0 ? i - 1 : 0) * k + rs);
  C64 pj[GP];
#pragma unroll
  for (int m = 0; m < GP; ++m) {
    const int j = lane + 64 * m;
    pj[m] = ldg(proj + (size_t)(j < i ? j : 0) * k + rs);
  }
  // the previous step's normalisation partial sums (i > 0)
  double v[4] = {0, 0, 0, 0};
  if (i > 0)
    for (int bb = threadIdx.x; bb < s.nb2; bb += GR * 64)
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] += s.part3[q * s.nb2 + bb];
  // a breakdown at an earlier step ends the iteration; the flag is read only
  // now so that its latency overlaps the loads above (all in bounds)
  if (s.flags[0]) return;
  C64 scal = mk(1.0, 0.0), sub = mk(0.0, 0.0);
  C64 scal_o = mk(1.0, 0.0);  // scale of the other side's new column
  if (i > 0) {
    bsum_first<GR * 64>(v, s.nb2);
    const C64 sd = s.herm ? mk(v[2], 0.0) : mk(v[0], v[1]);
    const double sabs = sqrt(norm2(sd));
    if (!(sabs > 1e-14 * sqrt(v[2] * (s.herm ? v[2] : v[3])))) {
      if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) s.flags[0] = i;
      return;
    }
    const double delta = sqrt(sabs);
    const C64 beta = (1.0 / delta) * sd;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
      stg(s.b + (i - 1), beta);
      stg(s.d + (i - 1), mk(delta, 0.0));
    }
    const C64 sv = mk(1.0 / delta, 0.0), sw = (1.0 / norm2(beta)) * beta;  // v = u / delta, w = q / conj(beta)
    scal = side ? sw : sv;
    scal_o = side ? sv : sw;
    sub = side ? mk(delta, 0.0) : beta;
  }
  // u_r = (B v_i)_r - sub * v_{i-1, r}: the batch loaded at launch, then
  // (k > 512) the rest of the row eight columns per lane at a time
  C64 ac[4] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
  auto madd = [&](int c0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = c0 + 64 * u;
      if (c < k) {
        const C64 x = (i > 0) ? cmul(scal, xv[u]) : mk(c == 0 ? 1.0 : 0.0, 0.0);
        ac[u & 3] = ac[u & 3] + cmul(mv[u], x);
      }
    }
  };
  madd(lane);
  for (int c0 = lane + 8 * 64; c0 < k; c0 += 8 * 64) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = c0 + 64 * u, cc = c < k ? c : 0;
      mv[u] = ldg(M + (size_t)rs * k + cc);
      xv[u] = ldg(src + cc);
    }
    madd(c0);
  }
  C64 acc = (ac[0] + ac[1]) + (ac[2] + ac[3]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    acc.re += __shfl_xor(acc.re, o, 64);
    acc.im += __shfl_xor(acc.im, o, 64);
  }
  const C64 xr = (i > 0) ? cmul(scal, xr_raw) : mk(r == 0 ? 1.0 : 0.0, 0.0);  // v_i (or w_i) at row r
  if (i > 0) acc = acc - cmul(sub, vold);
  if (live && lane == 0) {
    stg(basis + (size_t)i * k + r, xr);
    stg(dst + r, acc);
  }
  // this row's terms of the first-pass projections W^dag u (V^dag q): column
  // i of the other basis is being written by the other side's blocks in this
  // launch, so its entry is formed here from the raw vector (Hermitian: it
  // is this row's own new entry)
  const int ncol = i + 1;
  for (int m0 = 0; m0 * 64 < ncol; m0 += GP) {
#pragma unroll
    for (int m = 0; m < GP; ++m) {
      const int j = lane + 64 * (m0 + m);
      if (j < ncol) {
        C64 pv;
        if (j == i) pv = other ? ((i > 0) ? cmul(scal_o, xo_raw) : mk(r == 0 ? 1.0 : 0.0, 0.0)) : xr;
        else pv = (m0 == 0) ? pj[m] : ldg(proj + (size_t)j * k + rs);
        s_p[wave * ncol + j] = cmulc(pv, acc);
      }
    }
  }
  __syncthreads();
  gp<C64> out = s.part1 + ((size_t)side * s.nb1 + blockIdx.x) * s.lmax;
  for (int j = threadIdx.x; j < ncol; j += GR * 64) {
    C64 t = mk(0.0, 0.0);
#pragma unroll
    for (int w = 0; w < GR; ++w)
      if (blockIdx.x * GR + w < k) t = t + s_p[w * ncol + j];
    stg(out + j, t);
  }
}

// dynamic LDS of k_in_gemv at step i: GR x (i + 1) products (128 KB at the
// largest inner size)
static size_t gemv_lds(int i) { return (size_t)GR * (i + 1) * sizeof(C64); }

// pass 1 (last == 0): reduce part1, subtract, emit part2;
// pass 2 (last == 1): reduce part2, subtract, emit the normalisation sums.
// Every phase issues its loads in one batch per thread: the partial-sum and
// projection phases give each (side, column) four consecutive lanes that
// split the terms and meet by shuffles; the subtraction handles both sides
// in the same batch.
constexpr int TPJ = 4;  // lanes per (side, column) in the reduction phases

template <bool BATCH>
__global__ void __launch_bounds__(ST) k_in_sub(const Inner s0, const Inner* __restrict__ SS, int i, int last) {
  const InnerG s = inner_view(inner_desc<BATCH>(s0, SS));
  if (BATCH && (i >= s.lmax || (last && i + 1 >= s.lmax) || (int)blockIdx.x >= s.nb2)) return;
  const int k = s.k;
  const int sides = s.herm ? 1 : 2;
  __shared__ C64 s_c[2][LMAX];
  __shared__ C64 s_u[2][SR];
  gp<const C64> pin = pick(last != 0, s.part2, s.part1);
  const int nbin = pick(last != 0, s.nb2, s.nb1);
  const int ncol = i + 1;
  const int l4 = threadIdx.x & (TPJ - 1);
  // reduce the partial projections: item = (side, j), TPJ lanes each
  for (int it0 = 0; it0 < sides * ncol; it0 += ST / TPJ) {
    const int item = it0 + (int)threadIdx.x / TPJ;
    const bool ok = item < sides * ncol;
    const int side = ok ? item / ncol : 0, j = ok ? item % ncol : 0;
    gp<const C64> pp = pin + (size_t)side * nbin * s.lmax + j;
    C64 t0 = mk(0.0, 0.0), t1 = t0;
    for (int bb0 = l4; bb0 < nbin; bb0 += 8 * TPJ) {
      C64 pv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int bb = bb0 + u * TPJ;
        pv[u] = ldg(pp + (size_t)(bb < nbin ? bb : 0) * s.lmax);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (bb0 + u * TPJ < nbin) {
          if (u & 1)
            t1 = t1 + pv[u];
          else
            t0 = t0 + pv[u];
        }
    }
    C64 t = t0 + t1;
#pragma unroll
    for (int o = 1; o < TPJ; o <<= 1) {
      t.re += __shfl_xor(t.re, o, 64);
      t.im += __shfl_xor(t.im, o, 64);
    }
    if (ok && l4 == 0) s_c[side][j] = t;
  }
  // a breakdown flagged at this or an earlier step ends the iteration; the
  // flag is read only now so that its latency overlaps the loads above (all
  // in bounds)
  if (s.flags[0]) return;
  __syncthreads();
  if (!last && blockIdx.x == 0 && threadIdx.x == 0) stg(s.a + i, s.herm ? mk(s_c[0][i].re, 0.0) : s_c[0][i]);
  if (s.arnoldi && blockIdx.x == 0)  // column i of H_l: the first pass stores, the second adds
    for (int j = threadIdx.x; j <= i; j += ST) {
      gp<C64> h = s.hcol + (size_t)i * s.lmax + j;
      stg(h, last ? ldg(h) + s_c[0][j] : s_c[0][j]);
    }
  // u -= V c, q -= W d: eight lanes per row, columns jl, jl + 8, ... of both
  // sides in one batch of loads
  const int rl = threadIdx.x >> 3, jl = threadIdx.x & 7;
  const int r = blockIdx.x * SR + rl;
  gp<C64> u = rawv(s, 0, (i + 1) & 1);
  gp<C64> q = rawv(s, 1, (i + 1) & 1);
  C64 acc[2][2] = {{mk(0.0, 0.0), mk(0.0, 0.0)}, {mk(0.0, 0.0), mk(0.0, 0.0)}};
  if (r < k) {
    for (int j0 = jl; j0 <= i; j0 += 8 * 8) {
      C64 bv[2][8];
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        gp<const C64> basis = side ? s.W : s.V;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const int j = j0 + 8 * m;
          bv[side][m] = (side < sides) ? ldg(basis + (size_t)(j <= i ? j : 0) * k + r) : mk(0.0, 0.0);
        }
      }
#pragma unroll
      for (int side = 0; side < 2; ++side)
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const int j = j0 + 8 * m;
          if (side < sides && j <= i) acc[side][m & 1] = acc[side][m & 1] + cmul(bv[side][m], s_c[side][j]);
        }
    }
  }
  for (int side = 0; side < sides; ++side) {
    C64 a = acc[side][0] + acc[side][1];
#pragma unroll
    for (int o = 4; o > 0; o >>= 1) {
      a.re += __shfl_xor(a.re, o, 64);
      a.im += __shfl_xor(a.im, o, 64);
    }
    if (jl == 0) {
      C64 nv = mk(0.0, 0.0);
      if (r < k) {
        gp<C64> x = side ? q : u;
        nv = ldg(x + r) - a;
        stg(x + r, nv);
      }
      s_u[side][rl] = nv;
    }
  }
  __syncthreads();
  if (!last) {
    // second-pass partial projections over this block's rows: item = (side, j)
    const int nr = min(SR, k - blockIdx.x * SR);  // rows of this block (s_u is zero past them)
    for (int it0 = 0; it0 < sides * ncol; it0 += ST / TPJ) {
      const int item = it0 + (int)threadIdx.x / TPJ;
      const bool ok = item < sides * ncol;
      const int side = ok ? item / ncol : 0, j = ok ? item % ncol : 0;
      gp<const C64> proj = pick(s.herm || side, s.V, s.W);
      gp<const C64> pj = proj + (size_t)j * k + blockIdx.x * SR;
      C64 t0 = mk(0.0, 0.0), t1 = t0;
      for (int w0 = l4; w0 < nr; w0 += 8 * TPJ) {
        C64 pv[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const int w = w0 + m * TPJ;
          pv[m] = ldg(pj + (w < nr ? w : 0));
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const int w = w0 + m * TPJ;
          if (w < nr) {
            if (m & 1)
              t1 = t1 + cmulc(pv[m], s_u[side][w]);
            else
              t0 = t0 + cmulc(pv[m], s_u[side][w]);
          }
        }
      }
      C64 t = t0 + t1;
#pragma unroll
      for (int o = 1; o < TPJ; o <<= 1) {
        t.re += __shfl_xor(t.re, o, 64);
        t.im += __shfl_xor(t.im, o, 64);
      }
      if (ok && l4 == 0) stg(s.part2 + ((size_t)side * s.nb2 + blockIdx.x) * s.lmax + j, t);
    }
    return;
  }
  double v[4] = {0, 0, 0, 0};
  if (threadIdx.x < SR) {
    const C64 un = s_u[0][threadIdx.x];
    const C64 qn = s.herm ? un : s_u[1][threadIdx.x];
    const C64 t = cmulc(qn, un);
    v[0] = t.re;
    v[1] = t.im;
    v[2] = norm2(un);
    v[3] = norm2(qn);
  }
  bsum<ST>(v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) s.part3[qq * s.nb2 + blockIdx.x] = v[qq];
}

// dense upper Hessenberg H_l (ld = l, row-major) of the Arnoldi option.
// The recurrence subtracts b[c - 1] v_{c-1} from B v_c before it projects
// (the Lanczos form), so the stored coefficient of v_{c-1} lacks b[c - 1]:
// H[r][c] = hcol[c * lmax + r] (+ b[r] for r = c - 1) for r <= c,
// H[c + 1][c] = |u_c| = d[c], else 0
__global__ void k_hess_dense(int l, int lmax, const C64* __restrict__ hcol, const C64* __restrict__ b,
                             const C64* __restrict__ d, C64* __restrict__ H) {
  const size_t nn = (size_t)l * l;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / l), c = (int)(e % l);
    C64 v = mk(0.0, 0.0);
    if (r <= c) v = hcol[(size_t)c * lmax + r];
    if (r + 1 == c) v = v + b[r];
    if (r == c + 1) v = d[c];
    H[e] = v;
  }
}

// z = V y (k rows, l columns)
__global__ void k_in_lift(int k, int l, const C64* __restrict__ V, const C64* __restrict__ S, int lds,
                          C64* __restrict__ z) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= k) return;
  C64 acc = mk(0.0, 0.0);
  for (int j = 0; j < l; ++j) acc = acc + cmul(V[(size_t)j * k + r], S[(size_t)j * lds]);
  z[r] = acc;
}

// z = column 0 of S (ld = k)
__global__ void k_col0(int k, const C64* __restrict__ S, C64* __restrict__ z) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < k) z[r] = S[(size_t)r * k];
}

// ---------------------------------------------------------------------------
namespace {
DevBuf g_small, g_batch;
HostBuf g_small_pin;  // pinned readback of the inner iteration's flags
}

// device pointers of the tridiagonal factorisation of H_k
struct TriWork {
  C64 *Lm, *U0i, *U1, *U2;
  int* Sw;
};

// workspace of one inner problem of order k with ell steps, carved from base
// (base == nullptr: only the size); fills s and tw
static size_t inner_layout(int k, int ell, int hermitian, char* base, Inner* s, TriWork* tw) {
  const int nb1 = (k + GR - 1) / GR, nb2 = (k + SR - 1) / SR;
  const size_t kk = (size_t)k * k;
  size_t bytes = 0;
  auto take = [&](size_t b) {
    size_t o = bytes;
    bytes += (b + 255) & ~(size_t)255;
    return o;
  };
  const size_t oB = take(kk * sizeof(C64));
  const size_t oBH = take(hermitian ? 0 : kk * sizeof(C64));
  const size_t oV = take((size_t)k * ell * sizeof(C64));
  const size_t oW = take(hermitian ? 0 : (size_t)k * ell * sizeof(C64));
  const size_t oR = take((size_t)4 * k * sizeof(C64));
  const size_t oF = take((size_t)5 * k * sizeof(C64) + (size_t)k * sizeof(int));
  const size_t oC = take((size_t)3 * ell * sizeof(C64));
  const size_t oP1 = take((size_t)2 * nb1 * ell * sizeof(C64));
  const size_t oP2 = take((size_t)2 * nb2 * ell * sizeof(C64));
  const size_t oP3 = take((size_t)4 * nb2 * sizeof(double));
  const size_t oHc = take((size_t)ell * ell * sizeof(C64));
  const size_t oI = take(8 * sizeof(int));
  if (!base) return bytes;
  s->k = k;
  s->herm = hermitian;
  s->lmax = ell;
  s->B = (C64*)(base + oB);
  s->BH = hermitian ? s->B : (C64*)(base + oBH);
  s->V = (C64*)(base + oV);
  s->W = hermitian ? s->V : (C64*)(base + oW);
  C64* R = (C64*)(base + oR);
  s->uraw[0] = R;
  s->uraw[1] = R + k;
  s->qraw[0] = R + 2 * k;
  s->qraw[1] = R + 3 * k;
  C64* F = (C64*)(base + oF);
  tw->Lm = F;
  tw->U0i = F + k;
  tw->U1 = F + 2 * k;
  tw->U2 = F + 3 * k;
  tw->Sw = (int*)(F + 5 * k);
  C64* Cc = (C64*)(base + oC);
  s->a = Cc;
  s->b = Cc + ell;
  s->d = Cc + 2 * ell;
  s->part1 = (C64*)(base + oP1);
  s->part2 = (C64*)(base + oP2);
  s->part3 = (double*)(base + oP3);
  s->nb1 = nb1;
  s->nb2 = nb2;
  s->flags = (int*)(base + oI);
  s->hcol = (C64*)(base + oHc);
  s->arnoldi = 0;
  return bytes;
}

// B = H_k + H_k^{-1} (and B^dag) of one problem; clears its flags and b
static int inner_prepare(int k, int hermitian, const C64* alpha, const C64* beta, const C64* delta, const Inner& s,
                         const TriWork& tw, hipStream_t st) {
  NK_HIP(hipMemsetAsync(s.flags, 0, 8 * sizeof(int), st));
  NK_HIP(hipMemsetAsync(s.b, 0, 2 * s.lmax * sizeof(C64), st));
  const size_t lds_lu = k <= TRI_LDS_MAX ? (size_t)3 * k * sizeof(C64) : 0;
  const size_t lds_inv = k <= TRI_INV_LDS_MAX ? (size_t)k * (sizeof(TriF) + sizeof(int)) : 0;
  hipLaunchKernelGGL(k_tri_lu, dim3(1), dim3(256), lds_lu, st, k, alpha, beta, delta, tw.Lm, tw.Sw, tw.U0i, tw.U1,
                     tw.U2, s.flags + 1);
  hipLaunchKernelGGL(k_tri_inv, dim3((k + 63) / 64), dim3(64), lds_inv, st, k, tw.Lm, tw.Sw, tw.U0i, tw.U1, tw.U2,
                     alpha, beta, delta, (C64*)s.B);
  if (!hermitian)
    hipLaunchKernelGGL(k_adjoint, dim3((k + 31) / 32, (k + 31) / 32), dim3(32, 8), 0, st, k, s.B, (C64*)s.BH);
  NK_HIP(hipGetLastError());
  return NK_OK;
}

int small_sign_dev(int k, int ell, int hermitian, const C64* alpha, const C64* beta, const C64* delta,
                   int rh_scaling, int rh_maxit, double rh_tol, C64* z, SmallOut* out, hipStream_t st, int inner) {
  if (k <= 0) return NK_EINVAL;
  if (ell > k) ell = k;
  // Arnoldi runs the one-sided (Lanczos-form) recurrence on the general B and
  // keeps every coefficient; its H_l is upper Hessenberg
  const int arnoldi = inner == NK_INNER_ARNOLDI && ell > 0;
  const int oneside = hermitian || arnoldi;
  if (arnoldi && out && (out->hl_host || out->inner_only)) {
    set_error("the tridiagonal H_l export is for the outer level's family only");
    return NK_EINVAL;
  }
  if (ell <= 0) {
    // non-nested: RH on dense H_k
    if (g_small.ensure((size_t)k * k * sizeof(C64))) return NK_ENOMEM;
    C64* H = g_small.as<C64>();
    hipLaunchKernelGGL(k_tri_dense, dim3(1024), dim3(256), 0, st, k, alpha, beta, delta, H);
    NK_HIP(hipGetLastError());
    int it = 0;
    double res = 0;
    int e = rh_sign_batched(1, k, &k, H, rh_scaling, rh_maxit, rh_tol, &it, &res, st);
    if (e < 0) return e;
    hipLaunchKernelGGL(k_col0, dim3((k + 255) / 256), dim3(256), 0, st, k, H, z);
    NK_HIP(hipGetLastError());
    if (out) {
      out->rh_iters = it;
      out->ell_used = 0;
      out->rh_residual = res;
    }
    return e;
  }
  // nested
  if (ell > LMAX) {
    set_error("inner Krylov size %d exceeds %d", ell, LMAX);
    return NK_EINVAL;
  }
  const size_t lay = inner_layout(k, ell, oneside, nullptr, nullptr, nullptr);
  const size_t oS = (lay + 255) & ~(size_t)255;
  const size_t oD = oS + (((size_t)ell * ell * sizeof(C64) + 255) & ~(size_t)255);
  if (g_small.ensure(oD) || g_small_pin.ensure(2 * sizeof(int))) return NK_ENOMEM;
  char* base = g_small.as<char>();
  Inner s;
  TriWork tw;
  inner_layout(k, ell, oneside, base, &s, &tw);
  s.arnoldi = arnoldi;
  C64* Hl = (C64*)(base + oS);
  if (int e = inner_prepare(k, oneside, alpha, beta, delta, s, tw, st)) return e;
  const int sides = oneside ? 1 : 2;
  for (int i = 0; i < ell; ++i) {
    hipLaunchKernelGGL(k_in_gemv<false>, dim3(s.nb1, sides, 1), dim3(GR * 64), gemv_lds(i), st, s, nullptr, i);
    hipLaunchKernelGGL(k_in_sub<false>, dim3(s.nb2, 1, 1), dim3(ST), 0, st, s, nullptr, i, 0);
    if (i + 1 < ell) hipLaunchKernelGGL(k_in_sub<false>, dim3(s.nb2, 1, 1), dim3(ST), 0, st, s, nullptr, i, 1);
  }
  NK_HIP(hipGetLastError());
  int* fl = g_small_pin.host<int>();
  NK_HIP(hipMemcpyAsync(fl, s.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  NK_HIP(hipStreamSynchronize(st));
  if (fl[1]) {
    set_error("nested small problem: H_k is singular");
    return NK_WARN_NOTCONV;
  }
  const int lu = fl[0] ? fl[0] : ell;
  if (out && out->hl_host) {
    NK_HIP(hipMemcpyAsync(out->hl_host, s.a, lu * sizeof(C64), hipMemcpyDeviceToHost, st));
    NK_HIP(hipMemcpyAsync(out->hl_host + lu, s.b, lu * sizeof(C64), hipMemcpyDeviceToHost, st));
    NK_HIP(hipMemcpyAsync(out->hl_host + 2 * lu, s.d, lu * sizeof(C64), hipMemcpyDeviceToHost, st));
    NK_HIP(hipStreamSynchronize(st));
  }
  if (out && out->vl_dev)
    NK_HIP(hipMemcpyAsync(out->vl_dev, s.V, (size_t)k * lu * sizeof(C64), hipMemcpyDeviceToDevice, st));
  if (out && out->inner_only) {
    out->ell_used = lu;
    return fl[0] ? NK_WARN_BREAKDOWN : NK_OK;
  }
  if (arnoldi)
    hipLaunchKernelGGL(k_hess_dense, dim3(256), dim3(256), 0, st, lu, ell, s.hcol, s.b, s.d, Hl);
  else
    hipLaunchKernelGGL(k_tri_dense, dim3(256), dim3(256), 0, st, lu, s.a, s.b, s.d, Hl);
  NK_HIP(hipGetLastError());
  int it = 0;
  double res = 0;
  int e = rh_sign_batched(1, lu, &lu, Hl, rh_scaling, rh_maxit, rh_tol, &it, &res, st);
  if (e < 0) return e;
  hipLaunchKernelGGL(k_in_lift, dim3((k + 255) / 256), dim3(256), 0, st, k, lu, s.V, Hl, lu, z);
  NK_HIP(hipGetLastError());
  if (out) {
    out->rh_iters = it;
    out->ell_used = lu;
    out->rh_residual = res;
  }
  return e ? e : (fl[0] ? NK_WARN_BREAKDOWN : NK_OK);
}

// The inner projections of r problems at once: one launch per kernel and
// step serves all of them (grid z = problem).  Problem s has order k[s] and
// ell[s] steps; its H_ell (diagonal, super-, sub-diagonal) goes to
// hl_host + s * 3 * ldh (rows of ldh) and its basis V_ell (column j at
// j * k[s]) to vl_dev + s * vl_stride; ell_used[s] < ell[s] after an
// invariant subspace or a breakdown.
int small_inner_batch(int r, const int* k, const int* ell, int hermitian, const C64* const* alpha,
                      const C64* const* beta, const C64* const* delta, C64* hl_host, int ldh, C64* vl_dev,
                      size_t vl_stride, int* ell_used, hipStream_t st) {
  std::vector<size_t> off(r + 1, 0);
  for (int s = 0; s < r; ++s) {
    if (ell[s] < 1 || ell[s] > LMAX || ell[s] > k[s] || ell[s] > ldh) {
      set_error("inner problem %d: ell = %d outside [1, min(k = %d, %d)]", s, ell[s], k[s], LMAX);
      return NK_EINVAL;
    }
    off[s + 1] = off[s] + ((inner_layout(k[s], ell[s], hermitian, nullptr, nullptr, nullptr) + 255) & ~(size_t)255);
  }
  if (g_batch.ensure(off[r] + (size_t)r * sizeof(Inner) + 256)) return NK_ENOMEM;
  char* base = g_batch.as<char>();
  std::vector<Inner> S(r);
  std::vector<TriWork> tw(r);
  int lmax = 0, nb1 = 0, nb2 = 0;
  for (int s = 0; s < r; ++s) {
    inner_layout(k[s], ell[s], hermitian, base + off[s], &S[s], &tw[s]);
    if (int e = inner_prepare(k[s], hermitian, alpha[s], beta[s], delta[s], S[s], tw[s], st)) return e;
    lmax = std::max(lmax, ell[s]);
    nb1 = std::max(nb1, S[s].nb1);
    nb2 = std::max(nb2, S[s].nb2);
  }
  Inner* sdev = (Inner*)(base + off[r]);
  NK_HIP(hipMemcpyAsync(sdev, S.data(), r * sizeof(Inner), hipMemcpyHostToDevice, st));
  const int sides = hermitian ? 1 : 2;
  for (int i = 0; i < lmax; ++i) {
    hipLaunchKernelGGL(k_in_gemv<true>, dim3(nb1, sides, r), dim3(GR * 64), gemv_lds(i), st, Inner{}, sdev, i);
    hipLaunchKernelGGL(k_in_sub<true>, dim3(nb2, 1, r), dim3(ST), 0, st, Inner{}, sdev, i, 0);
    if (i + 1 < lmax) hipLaunchKernelGGL(k_in_sub<true>, dim3(nb2, 1, r), dim3(ST), 0, st, Inner{}, sdev, i, 1);
  }
  NK_HIP(hipGetLastError());
  std::vector<int> fl((size_t)2 * r);
  for (int s = 0; s < r; ++s) NK_HIP(hipMemcpyAsync(&fl[2 * s], S[s].flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  NK_HIP(hipStreamSynchronize(st));
  int warn = NK_OK;
  for (int s = 0; s < r; ++s) {
    if (fl[2 * s + 1]) {
      set_error("nested small problem %d: H_k is singular", s);
      return NK_WARN_NOTCONV;
    }
    const int lu = fl[2 * s] ? fl[2 * s] : ell[s];
    if (fl[2 * s]) warn = NK_WARN_BREAKDOWN;
    ell_used[s] = lu;
    C64* h = hl_host + (size_t)s * 3 * ldh;
    NK_HIP(hipMemcpyAsync(h, S[s].a, lu * sizeof(C64), hipMemcpyDeviceToHost, st));
    NK_HIP(hipMemcpyAsync(h + ldh, S[s].b, lu * sizeof(C64), hipMemcpyDeviceToHost, st));
    NK_HIP(hipMemcpyAsync(h + 2 * ldh, S[s].d, lu * sizeof(C64), hipMemcpyDeviceToHost, st));
    NK_HIP(hipMemcpyAsync(vl_dev + (size_t)s * vl_stride, S[s].V, (size_t)k[s] * lu * sizeof(C64),
                          hipMemcpyDeviceToDevice, st));
  }
  NK_HIP(hipStreamSynchronize(st));
  return warn;
}

}  // namespace nk
