// Internal declarations of the nested-Krylov sign-function library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "nk.h"

namespace nk {

// ---------------------------------------------------------------------------
// complex numbers in registers and memory (8- or 16-byte aligned pairs)
template <class R>
struct __align__(2 * sizeof(R)) Cx {
  R re, im;
};

template <class R>
__host__ __device__ __forceinline__ Cx<R> mk(R a, R b) {
  Cx<R> z;
  z.re = a;
  z.im = b;
  return z;
}
template <class R>
__host__ __device__ __forceinline__ Cx<R> operator+(Cx<R> a, Cx<R> b) { return mk(a.re + b.re, a.im + b.im); }
template <class R>
__host__ __device__ __forceinline__ Cx<R> operator-(Cx<R> a, Cx<R> b) { return mk(a.re - b.re, a.im - b.im); }
template <class R>
__host__ __device__ __forceinline__ Cx<R> operator*(R s, Cx<R> a) { return mk(s * a.re, s * a.im); }
template <class R>
__host__ __device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// conj(a) * b
template <class R>
__host__ __device__ __forceinline__ Cx<R> cmulc(Cx<R> a, Cx<R> b) {
  return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <class R>
__host__ __device__ __forceinline__ Cx<R> conj(Cx<R> a) { return mk(a.re, -a.im); }
template <class R>
__host__ __device__ __forceinline__ R norm2(Cx<R> a) { return a.re * a.re + a.im * a.im; }

using C64 = Cx<double>;

// A pointer read from memory (a descriptor in a buffer) or chosen between an
// LDS and a global array is generic to the compiler, which then emits flat
// instructions that wait on both the vector-memory and the LDS counters;
// device buffers are global memory, and this view says so.
template <class T>
using gp = T __attribute__((address_space(1)))*;
template <class T>
__device__ __forceinline__ gp<T> as_global(T* p) {
  return (gp<T>)p;
}
// complex loads and stores through such a view (struct copies need generic
// objects; the two halves become one 16-byte access)
__device__ __forceinline__ Cx<double> ldg(gp<const Cx<double>> p) { return mk<double>(p->re, p->im); }
__device__ __forceinline__ Cx<double> ldg(gp<Cx<double>> p) { return mk<double>(p->re, p->im); }
__device__ __forceinline__ Cx<double> ldg(const Cx<double>* p) { return *p; }  // any other space
__device__ __forceinline__ void stg(gp<Cx<double>> p, Cx<double> v) {
  p->re = v.re;
  p->im = v.im;
}
using C32 = Cx<float>;

template <class R>
__host__ __device__ __forceinline__ Cx<double> widen(Cx<R> a) { return mk<double>((double)a.re, (double)a.im); }
template <class R>
__host__ __device__ __forceinline__ Cx<R> narrow(Cx<double> a) { return mk<R>((R)a.re, (R)a.im); }

// ---------------------------------------------------------------------------
// lattice geometry: dims {Lx, Ly, Lz, Lt}.
// Canonical (API) site order: ((t Lz + z) Ly + y) Lx + x.
// Device site order is tiled: the lattice is cut into tiles of b0 x b1 x b2 x b3
// sites (16 x 4 x 4 x 4 where the extents allow; b0 else 8, 4 or 2, the
// others else 2) and
//   site = tile * TS + local,  local = ((tl b2 + zl) b1 + yl) b0 + xl,
//   tile = ((TT n2 + TZ) n1 + TY) n0 + TX,
// so that one workgroup's sites form a compact hypercube whose neighbours
// mostly lie in the same tile (and in cache).
struct Geom {
  int L[4];
  int stride[4];  // canonical strides 1, Lx, Lx Ly, Lx Ly Lz
  int V;
  int b[4];       // tile extent per direction
  int lb[4];      // log2 b
  int lstr[4];    // local strides within a tile
  int nt[4];      // tiles per direction
  int tstr[4];    // site offset between neighbouring tiles in each direction
  int lts;        // log2 of the tile size TS
};

void geom_init(Geom& g, const int dims[4]);

// device index of the site with coordinates (x, y, z, t)
__host__ __device__ __forceinline__ int tiled_index(const Geom& g, int x, int y, int z, int t) {
  const int c[4] = {x, y, z, t};
  int tile = 0, loc = 0;
#pragma unroll
  for (int d = 3; d >= 0; --d) {
    tile = tile * g.nt[d] + (c[d] >> g.lb[d]);
    loc = (loc << g.lb[d]) | (c[d] & (g.b[d] - 1));
  }
  return (tile << g.lts) + loc;
}

// device spinor layout (tiled site order; only pack/unpack see the canonical
// order).  FP64: component c = spin*3 + colour is a contiguous array of V
// complex numbers, field[c * V + site].  FP32: components 2p and 2p + 1 of a
// site sit side by side, field[(p * V + site) * 2 + (c & 1)], so that one
// 16-byte load fetches two components (one 16-byte FP64 component per load
// already fills a lane's widest load).  Krylov vectors live in these layouts.
// Device link layout: FP64 U[(nu * 9 + a * 3 + b) * V + site]; FP32 entries
// in pairs like the spinors, U[((nu * 5 + e / 2) * V + site) * 2 + (e & 1)]
// (the pair of entry 8 has an unused second half); BF16 storage keeps the 6
// complex entries of rows 0, 1 as packed words, words 0-3 of link (nu, site)
// at [(nu * V + site) * 4 + w] and words 4-5 at [16 V + (nu * V + site) * 2 + w - 4].
template <class R>
struct SpinorIndex;
template <>
struct SpinorIndex<double> {
  __host__ __device__ static size_t at(int V, int c, int s) { return (size_t)c * V + s; }
  __host__ __device__ static size_t to64(int, size_t i) { return i; }
};
template <>
struct SpinorIndex<float> {
  __host__ __device__ static size_t at(int V, int c, int s) { return ((size_t)(c >> 1) * V + s) * 2 + (c & 1); }
  // the FP64-layout index of element i of an FP32 vector
  __host__ __device__ static size_t to64(int V, size_t i) {
    const size_t ps = i >> 1;
    return (size_t)(2 * (int)(ps / V) + (int)(i & 1)) * V + (ps % V);
  }
};
// index of component c of device site s in a vector of precision R
template <class R>
__host__ __device__ __forceinline__ size_t sidx(int V, int c, int s) {
  return SpinorIndex<R>::at(V, c, s);
}
// index in a vector of precision R of element i of an FP64 vector, and back
template <class R>
__host__ __device__ __forceinline__ size_t sidx_of64(int V, size_t i) {
  return SpinorIndex<R>::at(V, (int)(i / V), (int)(i % V));
}
template <class R>
__host__ __device__ __forceinline__ size_t sidx_to64(int V, size_t i) {
  return SpinorIndex<R>::to64(V, i);
}

// ---------------------------------------------------------------------------
// error state
void set_error(const char* fmt, ...);
int hip_fail(hipError_t e, const char* what, const char* file, int line);

#define NK_HIP(call)                                                  \
  do {                                                                \
    hipError_t _e = (call);                                           \
    if (_e != hipSuccess) return ::nk::hip_fail(_e, #call, __FILE__, __LINE__); \
  } while (0)

// ---------------------------------------------------------------------------
// simple growable device buffer
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int ensure(size_t need);
  void release();
  template <class T>
  T* as() const { return reinterpret_cast<T*>(p); }
};

// A function-local workspace, released when it goes out of scope (hipFree
// waits for the device, so no kernel still reads it).  File-scope buffers and
// the handle's buffers are plain DevBufs: the handle releases its own in its
// destructor, and file-scope ones live until the process ends.
struct ScopedBuf : DevBuf {
  ScopedBuf() = default;
  ScopedBuf(const ScopedBuf&) = delete;
  ScopedBuf& operator=(const ScopedBuf&) = delete;
  ~ScopedBuf() { release(); }
};

}  // namespace nk

// the opaque handle
struct nk_lattice {
  nk::Geom g;
  int device = 0;
  bool have_gauge = false;
  nk::DevBuf U64, U32, Ubf;  // gauge field in the three storage formats
  // workspaces of the outer recurrence
  nk::DevBuf vk;       // outer basis V_k (unnormalised columns)
  nk::DevBuf work;     // p, q, W ring, scratch vectors
  nk::DevBuf coef;     // alpha, beta, delta, scales, flags
  nk::DevBuf part;     // per-workgroup partial sums
  nk::DevBuf canon;    // canonical-layout staging for host calls
  nk::DevBuf lift;     // lift coefficients
  nk::DevBuf tmp;      // device-layout temporaries of the stand-alone operator calls
  nk::DevBuf bvec;     // multi-source path: per-source vectors (basis, W ring, p, q, x, y)
  nk::DevBuf bsmall;   // multi-source path: coefficients, partial sums, small problems
  nk::DevBuf defl;     // deflation: partial sums, projections, projected sources
  nk::DevBuf ovl;      // overlap operator and solver: CG vectors, sign temporaries
  nk::DevBuf eig;      // eigensolver: four blocks of p vectors, partial sums, p x p matrices
  // multi-source path: sweeps captured as HIP graphs, keyed by their launch arguments
  struct Graph {
    std::vector<char> key;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<Graph> graphs;
  hipStream_t cap_stream = nullptr;  // private stream the sweeps are captured on
  // autotuned direction groups of the outer-recurrence stencil kernel,
  // [hermitian][precision]; 0 = not tuned yet
  int k1_groups[2][3] = {{0, 0, 0}, {0, 0, 0}};
  // sources per workgroup of the lockstep stencil kernel (1, 2 or 4), per
  // direction-group count (index 0: two groups, 1: four); 0 = not tuned yet
  int blk_group[2] = {0, 0};
  nk::DevBuf tunebuf;  // scratch coefficients of the autotuner
  // optional per-launch timing of the outer-recurrence kernels
  std::vector<hipEvent_t> evpool;
  std::vector<int> evkind;  // kind of each recorded (start, stop) pair: 0 = K1, 1 = K2
  size_t evnext = 0;
  ~nk_lattice();
};

namespace nk {

// ----- launchers implemented in the .hip files ------------------------------
// deflation.hip: bit i set = eigenvalue i has negative real part
struct DeflSigns {
  uint64_t w[NK_DEFL_MAX / 64];
};
int defl_partials(size_t n);
// c[i] = a_i^dag x for the m columns a_i (each n entries, one after another);
// part holds m * defl_partials(n) partial sums
int defl_dots(const C64* a, int m, size_t n, const C64* x, C64* part, C64* c, hipStream_t st);
// overlap.hip: y = Dov x (dagger = 0) or Dov^dag x, p->nrhs sources, tmp as
// large as x; CGNR for Dov y = b (one source)
// eig.hip: the m eigenpairs of gamma5 Dw(0) smallest in modulus (block of p,
// Chebyshev degree `degree`), starting from the p vectors v0
// the m eigenpairs of gamma5 Dw(mu) nearest the imaginary axis, right and
// left vectors with L^dag R = I (lam: 2 m doubles, re/im)
int eig_critical(nk_lattice* lat, double m_w, double mu, int m, int p, int degree, double tol, int maxit,
                 const C64* v0, double* lam, C64* r_out, C64* l_out, int* passes, double* resid, hipStream_t st);
int eig_hermitian(nk_lattice* lat, double m_w, int m, int p, int degree, double tol, int maxit, const C64* v0,
                  double* lam, C64* r_out, int* passes, double* resid, hipStream_t st);
// d.m > 0: the sign applications are deflated with (d.lam, d.R, d.L)
struct OvDefl {
  int m = 0;
  const double* lam = nullptr;
  const void* R = nullptr;
  const void* L = nullptr;
};
int overlap_apply(nk_lattice* lat, const nk_sign_params* p, int dagger, const OvDefl& d, const C64* x, C64* y,
                  C64* tmp, nk_sign_info* info, hipStream_t st);
int overlap_solve(nk_lattice* lat, const nk_sign_params* p, const OvDefl& d, double tol, int maxit, const C64* b,
                  C64* y, int* iters, double* resid, hipStream_t st);
// mode 0: out = x - R c; mode 1: out += R sgn(Lambda) c
int defl_combine(const C64* r, int m, size_t n, const C64* c, const DeflSigns& neg, int mode, const C64* x, C64* out,
                 hipStream_t st);

// layout.hip
int pack_gauge(nk_lattice* lat, const C64* canon, hipStream_t st);
template <class R>
int pack_spinor(const Geom& g, const C64* canon, Cx<R>* dev, hipStream_t st);
template <class R>
int unpack_spinor(const Geom& g, const Cx<R>* dev, C64* canon, hipStream_t st);

// wilson.hip
int apply_dw_dev(nk_lattice* lat, double m_w, double mu, int g5, const C64* x, C64* y, hipStream_t st);
int apply_pair_dev(nk_lattice* lat, double m_w, double mu, const C64* v, const C64* w, C64* av, C64* adw,
                   hipStream_t st);

// krylov.hip -- outer basis; coefficient arrays stay on the device
struct Coefs {
  C64* alpha;  // [k]
  C64* beta;   // [k]  beta[j]  = H[j][j+1]
  C64* delta;  // [k]  delta[j] = H[j+1][j]
  double* sv;  // [k+1] v_j = sv[j] * vt_j
  C64* sw;     // [k+1] w_j = sw[j] * wt_j
  int* flags;  // [4]: 0 = breakdown step (0 = none)
};
struct BasisPlan {
  int prec;       // NK_PREC_*
  int hermitian;  // Lanczos (1) or 2sL (0)
  double m_w, mu;
  int k;
  int store;      // 1: keep every column in V_k; 0: ring of 3 columns (two-pass sweeps)
  int profile;    // bracket every K1 / K2 launch with HIP events
};
size_t basis_vector_bytes(const Geom& g, int prec);
int basis_run(nk_lattice* lat, const BasisPlan& bp, const C64* x_canon, int j0, int j1, Coefs c, void* vk,
              hipStream_t st, int* breakdown_out);
// sum the recorded kernel durations (after a synchronisation) and reset the record
// a (start, stop) event of the handle's pool for profiled launches, and the
// summed durations of the recorded pairs by kind (0 = stencil step, 1 = update)
int prof_event(nk_lattice* lat, hipEvent_t* ev);
int prof_collect(nk_lattice* lat, double* t_k1, double* t_k2, int* n_k1, int* n_k2);
int lift_run(nk_lattice* lat, const BasisPlan& bp, int kused, const C64* z, double xnorm_dummy, Coefs c,
             const void* vk, C64* y_canon, hipStream_t st);
int two_pass_lift(nk_lattice* lat, const BasisPlan& bp, const C64* x_canon, int kused, const C64* z, Coefs c,
                  C64* y_canon, hipStream_t st);

int lift_columns(int n, int kused, const C64* vk, size_t colstride, const C64* z, const double* sv, C64* lc, C64* y,
                 hipStream_t st);

// block.hip -- many sources in lockstep (two-sided Lanczos, FP64); returns 1
// when the request is not one the block path covers (the caller then runs
// the sources one after another)
int block_sign(nk_lattice* lat, const nk_sign_params* p, const C64* x_canon, C64* y_canon, nk_sign_info* info,
               hipStream_t st);

// small.hip -- the small problem on the device
struct SmallOut {
  int rh_iters = 0;
  int ell_used = 0;
  double rh_residual = 0;
  C64* hl_host = nullptr;  // if set: receives H_ell's diagonal, super- and sub-diagonal (3 x ell, host)
  C64* vl_dev = nullptr;   // if set: receives the inner basis V_ell (device, column j at j * k)
  bool inner_only = false; // stop after the inner projection (no Roberts-Higham, no lift)
};
int small_sign_dev(int k, int ell, int hermitian, const C64* alpha, const C64* beta, const C64* delta,
                   int rh_scaling, int rh_maxit, double rh_tol, C64* z, SmallOut* out, hipStream_t st,
                   int inner = NK_INNER_SAME);

// the inner projections of r problems at once (see small.hip)
int small_inner_batch(int r, const int* k, const int* ell, int hermitian, const C64* const* alpha,
                      const C64* const* beta, const C64* const* delta, C64* hl_host, int ldh, C64* vl_dev,
                      size_t vl_stride, int* ell_used, hipStream_t st);

// rh.hip -- batched Roberts-Higham on dense matrices (S on the device, row-major,
// matrix b at b * ld * ld)
// the blocked inverse's launch shape: force one for every later call (all
// zero: back to the autotuner), or read the autotuner's choice for a size and
// batch class (returns 0 before it has chosen)
int rh_tile_force(int rm, int pth, int tile);
// the Newton-Schulz tail of the large path on (1) or off (0); returns the previous setting
int rh_newton_schulz(int enable);
int rh_tile_choice(int maxn, int batch, int* nb, int* rm, int* pth, int* tile);
int rh_sign_batched(int batch, int ld, const int* n_host, C64* S, int scaling, int maxit, double tol,
                    int* iters_host, double* resid_host, hipStream_t st);

// mlp.hip -- learned Roberts-Higham scaling (device pointers)
int mlp_features(int batch, int ld, const int* nvec_dev, const C64* S, float* feat, hipStream_t st);
int mlp_forward(int batch, const float* P, const float* feat, float* y, float* act, hipStream_t st);
int mlp_spectral_loss(int batch, const int* off, const C64* lam, const float* y, float gscale, float* loss,
                      float* dy, hipStream_t st);
int mlp_backward(int batch, const float* P, const float* feat, const float* act, const float* dy, float* delta,
                 float* grad, hipStream_t st);
int mlp_adam(int n, float* p, const float* g, float* m, float* v, int t, float lr, float b1, float b2, float eps,
             hipStream_t st);
int mlp_model_set(const float* params_host);
// [batch][NK_MLP_STEPS] FP64 factors (-1 = fall back) from the installed model; *have = 0 without one
int mlp_schedule(int batch, int ld, const int* nvec_dev, const C64* S, double* mu_dev, int* have, hipStream_t st);

}  // namespace nk
