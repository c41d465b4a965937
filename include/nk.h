/*
 * nk.h -- C ABI of the nested-Krylov sign-function library for MI355X (gfx950).
 *
 * The library computes y ~ sgn(A) x for A = gamma5 Dw(mu), the Wilson-Dirac
 * operator with the Hasenfratz-Karsch chemical potential (Bloch & Heybrock,
 * "A nested Krylov subspace method for the overlap operator", Sec. 1, Eq. (1)).
 * The approximation is the Krylov/Ritz one of Sec. 2, Eq. (3): Lanczos at
 * mu = 0 and two-sided Lanczos otherwise, and either the non-nested small
 * problem sgn(H_k) e_1 by the Roberts-Higham iteration (Eq. (4)) or the nested
 * one of Sec. 3, Eq. (5), with the preconditioning step H_k -> H_k + H_k^{-1}
 * (Eq. (6)).
 *
 * Conventions (the paper leaves them open; these are fixed here):
 *   dims = {Lx, Ly, Lz, Lt}, every L >= 2 and even; Lt is the temporal
 *   direction (antiperiodic, carries mu); x, y, z are periodic.
 *   A "canonical" spinor field is complex128, interleaved (re, im), indexed
 *   [t][z][y][x][spin 4][colour 3]; n = 12 V complex entries, V = Lx Ly Lz Lt.
 *   A canonical gauge field is complex128 [t][z][y][x][nu 4][3][3] with
 *   U[..][nu][a][b] the SU(3) link from x to x + nu (nu = 0..3 = x, y, z, t).
 *   gamma matrices: chiral Euclidean basis, gamma5 = diag(1, 1, -1, -1).
 *   Dw(mu) psi(x) = (4 + m_w) psi(x) - 1/2 sum_nu [ e^{+mu d_{nu t}} (1 - gamma_nu)
 *       U_nu(x) psi(x + nu) + e^{-mu d_{nu t}} (1 + gamma_nu) U_nu(x - nu)^dag psi(x - nu) ].
 *
 * Ownership: callers own every buffer they pass.  The library copies what it
 * needs and keeps no user pointer after a call returns.  It owns its device
 * workspaces: a handle's (Krylov bases etc.) are sized on first use and freed
 * by nk_lattice_destroy; the process-wide ones of the small problem, the
 * Roberts-Higham iteration and the learned model grow to the largest problem
 * seen and are kept until the process ends.
 *
 * Threads: calls on one handle must be serialised.  So must, across all
 * handles, every call that reaches the process-wide workspaces:
 * nk_sign_apply[_device], nk_sign_apply_deflated_device,
 * nk_overlap_apply_device, nk_overlap_solve_device (these three apply the
 * sign), nk_small_sign, nk_inner_matrix, nk_rh_sign, nk_rh_model_set and the
 * learned-scaling kernels.  nk_rh_tile_force and
 * nk_rh_tile_choice are thread-safe.
 *
 * Errors: every entry point returns 0 (NK_OK) on success, a negative code on
 * failure (outputs unspecified) or a positive warning (outputs valid).
 * nk_last_error() returns a thread-local message for the last failure.
 *
 * "_device" variants take device pointers and a HIP stream (NULL = the
 * default stream); they enqueue their work on that stream.  Host-pointer
 * variants are synchronous.
 */
#ifndef NK_H
#define NK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nk_lattice nk_lattice;
typedef struct ihipStream_t* nk_stream_t; /* a hipStream_t */

/* return codes */
#define NK_OK 0
#define NK_EINVAL (-1)      /* bad argument (dims, pointer, k, ell, nrhs, ...) */
#define NK_ENOGAUGE (-2)    /* no gauge field set on the handle */
#define NK_ENOMEM (-3)      /* device allocation failed (two_pass OFF and V_k does not fit) */
#define NK_EHIP (-4)        /* a HIP runtime call failed */
#define NK_WARN_NOTCONV 1   /* est > tol at k, or Roberts-Higham hit its iteration cap */
#define NK_WARN_BREAKDOWN 2 /* two-sided Lanczos broke down; result uses the steps before it */

/* precision of the outer Krylov recurrence (the small problem is always FP64) */
#define NK_PREC_FP64 0
#define NK_PREC_FP32 1           /* FP32 spinors and links, FP64 dots and coefficients */
#define NK_PREC_FP32_BF16LINKS 2 /* as FP32 with links stored in BF16 (12 reals), SU(3) rebuilt in FP32 */

/* Roberts-Higham scaling */
#define NK_RH_NONE 0    /* the paper's unscaled iteration, Eq. (4) */
#define NK_RH_DET 1     /* mu_n = |det S_n|^{-1/n} */
#define NK_RH_LEARNED 2 /* mu_n = |det S_n|^{-1/n} exp(y_n): determinant scaling times a correction
                          predicted for the first NK_MLP_STEPS steps by the model installed with
                          nk_rh_model_set (y = 0 later, for an implausible prediction and when no
                          model is installed) */

/* the learned-scaling network: NK_MLP_IN features -> 3 x NK_MLP_HIDDEN (tanh)
 * -> NK_MLP_STEPS values y_n.  Flat FP32 parameters, in this order:
 * W1[H][IN], b1[H], W2[H][H], b2[H], W3[H][H], b3[H], W4[STEPS][H], b4[STEPS]
 * (NK_MLP_NTRAIN trainable values), then the feature standardisation
 * mean[IN], inv_std[IN] (NK_MLP_NPARAMS in total). */
#define NK_MLP_IN 16
#define NK_MLP_HIDDEN 64
#define NK_MLP_STEPS 4
#define NK_MLP_NTRAIN 9668
#define NK_MLP_NPARAMS 9700

/* inner basis of the nested method */
#define NK_INNER_SAME 0
#define NK_INNER_ARNOLDI 1

/* two-pass lift */
#define NK_TWO_PASS_AUTO 0 /* store V_k when it fits in device memory, else two passes */
#define NK_TWO_PASS_ON 1   /* never store V_k: rebuild the basis in a second pass */
#define NK_TWO_PASS_OFF 2  /* always store V_k (NK_ENOMEM if it does not fit) */

typedef struct nk_sign_params {
  double m_w;          /* Wilson mass, -2 < m_w < 0 (Sec. 1) */
  double mu;           /* chemical potential; mu == 0 selects Hermitian Lanczos */
  int32_t k;           /* outer Krylov size (maximum when tol > 0) */
  int32_t ell;         /* inner Krylov size; 0 = non-nested method */
  double tol;          /* stop early when est < tol (0 = always run k steps) */
  int32_t nrhs;        /* number of sources (each its own Krylov space) */
  int32_t precision;   /* NK_PREC_* */
  int32_t rh_scaling;  /* NK_RH_* */
  int32_t two_pass;    /* NK_TWO_PASS_* */
  int32_t est_delay;   /* d of the estimate est = |z(k) - [z(k-d); 0]| / |z(k)|; 0 = no estimate */
  int32_t check_every; /* steps between early-stop checks when tol > 0 */
  int32_t rh_maxit;    /* Roberts-Higham iteration cap */
  double rh_tol;       /* Roberts-Higham stop: |S_{n+1} - S_n|_F <= rh_tol |S_{n+1}|_F */
  const int32_t* ell_per_rhs; /* optional host array [nrhs] of per-source ell (NULL = ell for all) */
  int32_t profile;     /* n > 0: time the two outer-recurrence kernels of every n-th step with HIP
                        * events bound to those launches on the caller's stream (0 = off;
                        * negative = NK_EINVAL) */
  int32_t block;       /* 1: run the nrhs sources in lockstep (two-sided Lanczos, FP64, tol = 0):
                        * four launches per step for all sources, batched small problems;
                        * 2: the same with each sweep of the basis replayed from a HIP graph
                        * captured on first use and cached on the handle; other cases, and 0,
                        * run the sources one after another */
  int32_t inner;       /* basis of the nested method's inner space K_l(B, e_1) (Sec. 3, which
                        * leaves it open): NK_INNER_SAME, the outer level's family with full
                        * re-(bi)orthogonalisation (Lanczos at mu = 0, two-sided Lanczos
                        * otherwise), or NK_INNER_ARNOLDI (orthonormal basis, Hessenberg H_l);
                        * lockstep runs (block > 0) take NK_INNER_SAME only */
} nk_sign_params;

typedef struct nk_sign_info {
  int32_t k_used;         /* outer steps actually taken */
  int32_t ell_used;       /* inner steps (0 for the non-nested method) */
  int32_t rh_iters;       /* Roberts-Higham iterations on the small matrix */
  int32_t breakdown_step; /* 2sL step of a serious breakdown, 0 = none */
  int32_t two_pass;       /* 1 if the lift rebuilt the basis */
  int32_t pad;
  double est;             /* convergence estimate (NaN if not computed) */
  double rh_residual;     /* |S^2 - I|_F / sqrt(n) of the final Roberts-Higham iterate S of order n (0 when S^2 = I) */
  double t_basis_ms, t_small_ms, t_lift_ms;
  /* with params.profile: summed durations and launch counts of the two
   * outer-recurrence kernels (K1: stencil step, K2: update step); with
   * params.block = 1 each launch covers all sources of a lockstep range
   * (block = 2 replays graphs, which carry no events) */
  double t_stencil_ms, t_update_ms;
  int32_t n_stencil, n_update;
} nk_sign_info;

/* Fill *p with defaults: m_w = -1, mu = 0, k = 100, ell = 0, tol = 0, nrhs = 1,
 * FP64, unscaled RH, two_pass AUTO, est_delay = 0, check_every = 50,
 * rh_maxit = 100, rh_tol = 1e-13, ell_per_rhs = NULL, profile = 0, block = 0,
 * inner = NK_INNER_SAME. */
void nk_sign_params_default(nk_sign_params* p);

/* Create a lattice context on the current HIP device: the four-dimensional
 * lattice on which the Wilson-Dirac operator of Sec. 1 (the Dw inside
 * Eq. (1)) acts.  dims = {Lx, Ly, Lz, Lt}, each >= 2 and even.  NK_EINVAL on
 * bad dims or out == NULL. */
int nk_lattice_create(const int32_t dims[4], nk_lattice** out);

/* Free the context and all its device memory.  NULL-safe. */
int nk_lattice_destroy(nk_lattice* lat);

/* Set the gauge field, the SU(3) link variables U_nu(x) that the hopping
 * terms of Dw (Sec. 1) multiply, from a host array in canonical layout
 * (4 V 9 complex128).  Copied to the device in the library's own layout;
 * the caller keeps U. */
int nk_gauge_set(nk_lattice* lat, const double* U);

/* As nk_gauge_set (the links of Sec. 1), from a device pointer (canonical
 * layout), on `stream`. */
int nk_gauge_set_device(nk_lattice* lat, const void* dU, nk_stream_t stream);

/* y = Dw(mu) x (gamma5 == 0) or y = gamma5 Dw(mu) x (gamma5 != 0) for nrhs
 * canonical vectors stored one after another (x, y: nrhs * 12 V complex128).
 * The operator of Sec. 1; host pointers, synchronous.  x and y must not alias. */
int nk_apply_dw(nk_lattice* lat, double m_w, double mu, int32_t gamma5,
                const double* x, double* y, int32_t nrhs);

/* Device-pointer variant of nk_apply_dw, asynchronous on `stream`. */
int nk_apply_dw_device(nk_lattice* lat, double m_w, double mu, int32_t gamma5,
                       const void* x, void* y, int32_t nrhs, nk_stream_t stream);

/* The fused pair used by two-sided Lanczos (Sec. 2): av = A(mu) v and
 * adw = A(mu)^dag w = A(-mu) w for A = gamma5 Dw, one link load for both.
 * Canonical device vectors (12 V complex128 each); asynchronous on `stream`. */
int nk_apply_pair_device(nk_lattice* lat, double m_w, double mu,
                         const void* v, const void* w, void* av, void* adw,
                         nk_stream_t stream);

/* The library's own FP64 device layout of a spinor field ("packed"): 12 V
 * complex128 per vector, component-major, sites in the handle's tile order.
 * The operator of Sec. 1 is applied there without a layout change, so a caller
 * that applies it many times (an outer solver) packs once, applies as often as
 * it needs and unpacks once.  The layout is a permutation of the canonical one,
 * so sums, norms and inner products are the same in both (up to summation
 * order); a packed vector is only meaningful on a handle of the same
 * dimensions.  All four are asynchronous on `stream`; the caller owns every
 * buffer.  NK_EINVAL on NULL pointers, nrhs < 1 or aliasing input and output;
 * the two applications return NK_ENOGAUGE before nk_gauge_set. */

/* canonical -> packed for nrhs vectors stored one after another */
int nk_spinor_pack_device(nk_lattice* lat, const void* x, void* xp, int32_t nrhs, nk_stream_t stream);

/* packed -> canonical for nrhs vectors stored one after another */
int nk_spinor_unpack_device(nk_lattice* lat, const void* xp, void* x, int32_t nrhs, nk_stream_t stream);

/* yp = [gamma5] Dw(mu) xp on packed vectors: one stencil launch, no scratch
 * memory.  Bit-identical to nk_apply_dw_device on the same vector. */
int nk_apply_dw_packed_device(nk_lattice* lat, double m_w, double mu, int32_t gamma5,
                              const void* xp, void* yp, nk_stream_t stream);

/* The fused pair (avp = A(mu) vp, adwp = A(-mu) wp, A = gamma5 Dw) on packed
 * vectors: one stencil launch.  Bit-identical to nk_apply_pair_device.
 * Neither output may alias an input or the other output. */
int nk_apply_pair_packed_device(nk_lattice* lat, double m_w, double mu,
                                const void* vp, const void* wp, void* avp, void* adwp,
                                nk_stream_t stream);

/* The outer Krylov basis only (Sec. 2): k steps of Lanczos (mu == 0) or
 * two-sided Lanczos from x (canonical device vector), in p->precision.
 * Writes the tridiagonal Ritz matrix H_k to host arrays: alpha[2k] (complex
 * diagonal), beta[2k] (complex, beta[j] = H[j][j+1]), delta[2k] (complex,
 * delta[j] = H[j+1][j]); entries past k_used are zero.  info may be NULL. */
int nk_krylov_basis_device(nk_lattice* lat, const nk_sign_params* p, const void* x,
                           double* alpha, double* beta, double* delta,
                           nk_sign_info* info, nk_stream_t stream);

/* The small problem on the device, from a host tridiagonal H_k (layout as
 * above): z = sgn(H_k) e_1 (ell == 0, Eqs. (3)-(4)) or z = V_l sgn(H_l) e_1
 * with the inner space K_l(H_k + H_k^{-1}, e_1) (Sec. 3, Eqs. (5)-(6)).
 * hermitian != 0 selects inner Lanczos, else inner two-sided Lanczos.
 * z: host complex128[k].  info may be NULL.  Synchronous. */
int nk_small_sign(int32_t k, int32_t ell, int32_t hermitian,
                  const double* alpha, const double* beta, const double* delta,
                  const nk_sign_params* p, double* z, nk_sign_info* info);

/* Roberts-Higham sign of `batch` dense complex matrices (Eq. (4)) on the
 * device.  S: host complex128, matrix b at offset b * ld * ld, row-major,
 * leading dimension ld, size n[b] <= ld.  On return S holds sgn(S) and
 * iters[b] the iteration counts.  scaling = NK_RH_*.  Synchronous. */
int nk_rh_sign(int32_t batch, int32_t ld, const int32_t* n, double* S,
               int32_t scaling, int32_t maxit, double tol, int32_t* iters);

/* The inner projection of Sec. 3: from a host tridiagonal H_k (layout as
 * above), ell steps of Lanczos (hermitian != 0) or two-sided Lanczos on
 * B = H_k + H_k^{-1} from e_1 (Eq. (6)), with full re-(bi)orthogonalisation.
 * Writes the tridiagonal H_ell to host a[2 ell], b[2 ell], d[2 ell] (same
 * layout as H_k) and its order to *ell_used (smaller than ell after an
 * invariant subspace or a breakdown).  Synchronous. */
int nk_inner_matrix(int32_t k, int32_t ell, int32_t hermitian,
                    const double* alpha, const double* beta, const double* delta,
                    double* a, double* b, double* d, int32_t* ell_used);

/* --- learned Roberts-Higham scaling (an extension of Eq. (4)) -------------
 * sgn(mu S) = sgn(S) for mu > 0 (the argument of Eq. (7) holds for mu z), so
 * the factors change only the iteration count.  Training is label-free: for
 * a diagonalisable S_0 each eigenvalue follows z <- (mu z + 1/(mu z)) / 2 and
 * log|det S_n| = sum log|z|, and the loss is the smooth maximum over
 * eigenvalues of log |z_T - sgn Re lambda| after NK_MLP_STEPS steps.
 * All pointers below are device pointers (FP32 unless stated); every call
 * is asynchronous on `stream`. */

/* Install (host params[NK_MLP_NPARAMS]) or remove (NULL) the model used by
 * NK_RH_LEARNED; process-wide, copied to the current device. */
int nk_rh_model_set(const float* params);

/* NK_MLP_IN features of each dense matrix: S device complex128 [batch][ld][ld]
 * row-major, orders n (host int32[batch], n[b] <= ld); feat [batch][NK_MLP_IN]. */
int nk_rh_features_device(int32_t batch, int32_t ld, const int32_t* n, const void* S, float* feat,
                          nk_stream_t stream);

/* Forward pass: y [batch][NK_MLP_STEPS]; act [batch][3][NK_MLP_HIDDEN]
 * keeps the hidden activations for the backward pass (may be NULL). */
int nk_mlp_forward_device(int32_t batch, const float* params, const float* feat, float* y, float* act,
                          nk_stream_t stream);

/* Spectral loss per sample and its gradient times gscale:
 * eigenvalues of sample b are lam[off[b] .. off[b+1]) (device complex128;
 * off device int32[batch + 1], at most 1024 per sample); loss [batch];
 * dy [batch][NK_MLP_STEPS] = gscale * dloss_b / dy_b. */
int nk_rh_spectral_loss_device(int32_t batch, const int32_t* off, const void* lam, const float* y,
                               float gscale, float* loss, float* dy, nk_stream_t stream);

/* Backward pass: grad [NK_MLP_NTRAIN] = sum_b d<dy_b, y_b>/dparams, summed
 * over the batch in a fixed order; delta is workspace [batch][3][NK_MLP_HIDDEN]. */
int nk_mlp_backward_device(int32_t batch, const float* params, const float* feat, const float* act,
                           const float* dy, float* delta, float* grad, nk_stream_t stream);

/* One Adam step on params[0 .. n) (n <= NK_MLP_NTRAIN normally) with moment
 * buffers m, v; t counts steps from 1. */
int nk_adam_step_device(int32_t n, float* params, const float* grad, float* m, float* v, int32_t t,
                        float lr, float beta1, float beta2, float eps, nk_stream_t stream);

/* y ~ sgn(gamma5 Dw(mu)) x (Eqs. (3)-(6)), nrhs canonical host vectors.
 * Synchronous.  NK_WARN_* on a valid but unconverged/broken-down result.
 * info may be NULL (for nrhs > 1 it describes the last source). */
int nk_sign_apply(nk_lattice* lat, const nk_sign_params* p, const double* x, double* y,
                  nk_sign_info* info);

/* Device-pointer variant; it synchronises `stream` before returning (the
 * early-stop checks and the small problem need host decisions). */
int nk_sign_apply_device(nk_lattice* lat, const nk_sign_params* p, const void* x, void* y,
                         nk_sign_info* info, nk_stream_t stream);

/* Largest number of deflated eigenpairs nk_sign_apply_deflated_device takes. */
#define NK_DEFL_MAX 1024

/* y ~ sgn(gamma5 Dw(mu)) x with m critical eigenvalues treated exactly
 * (deflation, Sec. 2): with right eigenvectors R = [r_1 .. r_m]
 * (A r_i = lambda_i r_i), left eigenvectors L = [l_1 .. l_m]
 * (l_i^dag A = lambda_i l_i^dag) and L^dag R = I,
 *   y = R sgn(Lambda) (L^dag x) + [Krylov approximation of sgn(A)] (x - R L^dag x),
 * where the Krylov part is exactly what nk_sign_apply_device computes with the
 * same parameters (nested for ell > 0, non-nested for ell = 0), applied to the
 * projected source.  sgn(lambda) = sgn(Re lambda).  At mu = 0 (Hermitian A)
 * pass L = R with orthonormal columns.
 *   lam  host, 2 m doubles: the eigenvalues, (re, im) interleaved; only the
 *        sign of the real part is used, and a zero or non-finite entry is
 *        NK_EINVAL;
 *   R, L device complex128, m canonical vectors each, one after another
 *        (column i at offset i * 12 V); the library does not check that they
 *        are eigenvectors or that L^dag R = I: the result is exact only when
 *        they are;
 *   x, y device complex128, p->nrhs canonical vectors; the same eigenpairs
 *        serve every source.  y must not overlap x, R or L.
 * 0 <= m <= NK_DEFL_MAX; m = 0 is nk_sign_apply_device.  A source whose
 * projection is exactly zero (x in the span of R) gets only the exact part,
 * and runs no Krylov iteration.  Workspace (p->nrhs projected sources and the
 * projections) is kept in the handle.  Synchronises `stream` before
 * returning; info as for nk_sign_apply_device (zeroed if no source needed the
 * Krylov part). */
int nk_sign_apply_deflated_device(nk_lattice* lat, const nk_sign_params* p, int32_t m, const double* lam,
                                  const void* R, const void* L, const void* x, void* y, nk_sign_info* info,
                                  nk_stream_t stream);

/* The critical eigenpairs that deflation treats exactly (Sec. 2), for the
 * Hermitian case mu = 0: the m eigenvalues of H = gamma5 Dw(0) (mass m_w)
 * smallest in modulus, with orthonormal eigenvectors, to pass to
 * nk_sign_apply_deflated_device as lam, R and L = R.  The paper takes them
 * as given; this library computes them by Chebyshev-filtered subspace
 * iteration on H^2 with a block of p vectors (m <= p <= 128; a few more than
 * m speed convergence) and filter degree `degree`, starting from the p
 * canonical device vectors V0 (for example Gaussian; not modified), with
 * Rayleigh-Ritz on H^2 after each filter pass.
 *   lam     host, m doubles, ascending in modulus;
 *   R       device, m canonical vectors, one after another;
 *   *passes filter passes used, *resid the largest |H r_i - lam_i r_i|.
 * Stops when *resid <= tol * (|4 + m_w| + 8) (a bound on |H|) or after maxit
 * passes (NK_WARN_NOTCONV, the current Ritz pairs returned).  The
 * eigenvalues of H^2 just above the block limit the speed: the smaller the
 * gap, the more passes.  NK_EINVAL for bad sizes or R overlapping V0, or if
 * the block loses rank; NK_ENOGAUGE without a gauge field.  Workspace (four
 * blocks of p vectors) is kept in the handle.  Synchronises `stream`. */
int nk_eig_hermitian_device(nk_lattice* lat, double m_w, int32_t m, int32_t p, int32_t degree, double tol,
                            int32_t maxit, const void* V0, double* lam, void* R, int32_t* passes, double* resid,
                            nk_stream_t stream);

/* The critical eigenpairs that deflation treats exactly (Sec. 2) for any mu:
 * the m eigenvalues of A = gamma5 Dw(mu) (mass m_w) nearest the imaginary
 * axis (smallest |Re lambda|), with right eigenvectors R (A r_i = lambda_i
 * r_i, unit norm) and left eigenvectors L (l_i^dag A = lambda_i l_i^dag)
 * scaled so that L^dag R = I, to pass to nk_sign_apply_deflated_device as
 * lam, R and L.  The paper takes them as given; this library computes them
 * by two-sided Chebyshev-filtered subspace iteration: right and left blocks
 * of p vectors (m <= p <= 128) filtered by the degree-`degree` Chebyshev
 * polynomial in A^2 and (A^dag)^2 = A(-mu)^2, which amplifies the part of the
 * spectrum with the smallest Re lambda^2 (the eigenvalues near the
 * imaginary axis, while the imaginary parts of the others stay small), then
 * two-sided Rayleigh-Ritz.  Both blocks start from the p canonical device
 * vectors V0 (not modified).
 *   lam     host, 2 m doubles: the eigenvalues (re, im), ascending |Re|;
 *   R, L    device, m canonical vectors each, one after another;
 *   *passes filter passes used, *resid the largest relative residual
 *           |A r_i - lambda_i r_i| or |A^dag l_i - conj(lambda_i) l_i| / |l_i|.
 * Stops when *resid <= tol * (|4 + m_w| + 6 + 2 cosh mu) (a bound on |A|) or
 * after maxit passes (NK_WARN_NOTCONV, the current Ritz pairs returned).
 * At mu = 0 it finds what nk_eig_hermitian_device finds, with L = R.
 * NK_EINVAL for bad sizes, overlapping V0, R and L, or if the blocks lose
 * rank; NK_ENOGAUGE without a gauge field.  Workspace (six blocks of p
 * vectors) is kept in the handle.  Synchronises `stream`. */
int nk_eig_critical_device(nk_lattice* lat, double m_w, double mu, int32_t m, int32_t p, int32_t degree, double tol,
                           int32_t maxit, const void* V0, double* lam, void* R, void* L, int32_t* passes,
                           double* resid, nk_stream_t stream);

/* The overlap operator (Sec. 1, Eq. (1)) on p->nrhs canonical device vectors:
 *   dagger = 0: y = Dov(mu) x = x + gamma5 sgn(gamma5 Dw(mu)) x;
 *   dagger = 1: y = Dov(mu)^dag x = x + sgn(gamma5 Dw(-mu)) gamma5 x
 * (sgn(A)^dag = sgn(A^dag) and A^dag = gamma5 Dw(-mu)), with the sign
 * computed by nk_sign_apply_device with the parameters p (nested for
 * ell > 0), so the same errors and warnings apply, a zero source included.
 * m > 0 deflates the sign (Sec. 2) with the m eigenpairs (lam, R, L) of A, as
 * nk_sign_apply_deflated_device takes them; for Dov^dag the library uses the
 * eigenpairs of A^dag that these give: eigenvalues conj(lam), right
 * eigenvectors L, left eigenvectors R.  m = 0: lam, R, L may be NULL.
 * gamma5 = diag(1, 1, -1, -1) on the spin index.  y must not overlap x, R
 * or L; one temporary of the size of x is kept in the handle.  Synchronises
 * `stream` before returning; info describes the sign application. */
int nk_overlap_apply_device(nk_lattice* lat, const nk_sign_params* p, int32_t dagger, int32_t m, const double* lam,
                            const void* R, const void* L, const void* x, void* y, nk_sign_info* info,
                            nk_stream_t stream);

/* Solve Dov(mu) y = b for one canonical device vector b (p->nrhs must be 1)
 * by the conjugate-gradient method on the normal equations
 * Dov^dag Dov y = Dov^dag b (CGNR), from y = 0, with Dov and Dov^dag applied
 * as nk_overlap_apply_device does (two sign applications per iteration,
 * deflated with the m eigenpairs (lam, R, L) when m > 0).
 * Stops when the recursively updated residual |b - Dov y| <= tol |b| or after
 * maxit iterations (NK_WARN_NOTCONV, y the last iterate).  The attainable
 * residual is bounded by the sign's own accuracy at (k, ell).  b = 0 gives
 * y = 0 with *iters = 0.  Writes the iterations and the final relative
 * residual to *iters, *resid.  Returns the largest warning of the sign
 * applications or NK_WARN_NOTCONV; tol <= 0, maxit < 1, nrhs != 1 or b and y
 * overlapping are NK_EINVAL.  Workspace (five vectors) is kept in the handle;
 * synchronises `stream` before returning. */
int nk_overlap_solve_device(nk_lattice* lat, const nk_sign_params* p, int32_t m, const double* lam, const void* R,
                            const void* L, double tol, int32_t maxit, const void* b, void* y, int32_t* iters,
                            double* resid, nk_stream_t stream);

/* Launch shape of the blocked Gauss-Jordan inverse inside Roberts-Higham for
 * matrices of order > 128 (Eq. (4)): panel threads (256, 512 or 1024) x rows
 * per thread (1, 2 or 4; their product must cover the order) and the update
 * tile (32 or 64).  The library's autotuner times every feasible shape once
 * per class of matrix order (multiples of 64) and batch size (1, 2-4, 5-16,
 * more) and keeps the fastest; no shape changes a bit of the result.
 * nk_rh_tile_force fixes one shape for every later call where it is feasible
 * (0, 0, 0: back to the autotuner); NK_EINVAL for a shape that does not
 * exist.  nk_rh_tile_choice writes {panel width, rows per thread, panel
 * threads, tile} chosen for order n and batch size `batch` and returns 1, or
 * writes zeros and returns 0 before the autotuner has chosen; NK_EINVAL for
 * n < 1, batch < 1 or a NULL shape.  Both are process-wide and thread-safe. */
int nk_rh_tile_force(int32_t rows_per_thread, int32_t panel_threads, int32_t update_tile);

/* The Newton-Schulz tail of the Roberts-Higham iteration for orders > 128
 * (an option of this library, not part of Eq. (4)): once an iterate S
 * satisfies |I - S^2|_F < 1/2, the remaining steps are S <- S (3 I - S^2) / 2
 * (two matrix products on the FP64 matrix cores instead of an inversion),
 * which converges quadratically to the same limit sgn(S_0); the stopping
 * test is the same.  Tried for a matrix once its relative change per step has
 * fallen below 0.05.  Process-wide; enable != 0 turns it on (the default),
 * 0 off (every step an inversion, as Eq. (4)).  Returns the previous
 * setting.  Thread-safe. */
int nk_rh_newton_schulz(int32_t enable);
int nk_rh_tile_choice(int32_t n, int32_t batch, int32_t shape[4]);

/* Sources per workgroup (1, 2 or 4) of the lockstep stencil kernel
 * (params.block > 0): with 2 or 4, the lanes of one site carry that many
 * sources and share each link load.  The library times the three once per
 * handle on the first lockstep run and keeps the fastest (a larger group only
 * when more than 5% faster).  set = 1, 2 or 4 fixes the choice on this handle
 * for later runs; set = 0 changes nothing.  Returns the choice before the
 * call (0 before the first lockstep run); NK_EINVAL for a NULL handle or
 * another set.  The group changes the order of the partial sums of w^dag A v,
 * so results differ between group sizes by rounding. */
int nk_block_group(nk_lattice* lat, int32_t set);

/* Direction groups (2 or 4) of the outer-recurrence stencil kernel that the
 * autotuner chose on this handle for the given precision and recurrence
 * (hermitian != 0: Lanczos), 0 before the first basis run; NK_EINVAL for a
 * NULL handle or an unknown precision.  The autotuner times both kernels once
 * per handle on the first outer-basis run and keeps the faster. */
int nk_stencil_groups(nk_lattice* lat, int32_t precision, int32_t hermitian);

/* A measurement helper, not part of the method: the bandwidth this
 * library's own streaming code reaches, the ceiling against which the
 * stencil and the recurrences are read.  Over n complex128 entries, 16 bytes
 * per lane per access with four accesses in flight per lane, `blocks`
 * workgroups of 256 threads (grid-stride):
 *   kind 0: read a once, c[0 .. blocks) = per-workgroup partial sums of |a_i|^2;
 *   kind 1: c = a (copy);
 *   kind 2: c = a + b / 2 (triad).
 * Device pointers, asynchronous on `stream`; b is read by kind 2 only.
 * NK_EINVAL for an unknown kind, n < 1, blocks < 1 or a missing pointer. */
int nk_stream_device(int32_t kind, int64_t n, const void* a, const void* b, void* c, int32_t blocks,
                     nk_stream_t stream);

/* Largest lattice (sites) that nk_apply_dw_noalloc_device takes: 16^4. */
#define NK_NOALLOC_MAX_SITES 65536

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * y = [gamma5] Dw(mu) x as nk_apply_dw_device, bit for bit, on nrhs canonical
 * device vectors, asynchronous on `stream`, with the two layout temporaries
 * (the packed source and the packed result) in a fixed device array of
 * 2 x 12 x NK_NOALLOC_MAX_SITES complex128 (24 MiB) that each device holds
 * from its first use until the process ends.  The call allocates and frees
 * nothing.  Lattices of more than NK_NOALLOC_MAX_SITES sites are NK_EINVAL;
 * other errors as nk_apply_dw_device.  Every call on one device shares that
 * device's array, so calls that overlap on one device (on different streams,
 * or from different threads) race and must be serialised by the caller. */
int nk_apply_dw_noalloc_device(nk_lattice* lat, double m_w, double mu, int32_t gamma5, const void* x, void* y,
                               int32_t nrhs, nk_stream_t stream);

/* Thread-local message for the last failure ("" if none). */
const char* nk_last_error(void);

/* Library version string. */
const char* nk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NK_H */
