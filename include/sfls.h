/*
 * sfls.h -- C ABI of the MI355X (gfx950) superfast line-spectral-estimation
 * library.
 *
 * The method is T. L. Hansen, B. H. Fleury, B. D. Rao, "Superfast Line
 * Spectral Estimation", IEEE Trans. Signal Process., 2018 (complete-data
 * case, Phi = I, M = N).  Given y in C^N the estimator returns the model order
 * K, frequencies theta_k in [0,1), amplitudes alpha_k and the noise variance
 * beta (Sec. II-A problem statement; alpha = gamma .* q, Sec. II-B footnote).
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - psi(theta)_n = exp(j 2 pi n theta), n = 0..N-1 (0-indexed form of Sec. II-A).
 *  - Complex data are interleaved (re, im) pairs: "c128" = 2 doubles per
 *    element, "c64" = 2 floats per element.
 *  - Ragged batches: instance b occupies elements [off[b], off[b] + n[b]) of
 *    every flat per-sample array.  n[] and off[] (and every other array whose
 *    description says "host") are HOST arrays read synchronously; all data
 *    arrays are DEVICE pointers on the context's device.
 *  - All work is enqueued on `stream` (a hipStream_t, NULL = the legacy
 *    default stream) and is asynchronous: outputs are valid once the stream
 *    has been synchronised.  The caller owns every buffer it passes; the
 *    library owns its workspace (kept in the context, grown on demand).
 *  - Argument errors are detected on the host before anything is enqueued
 *    and return SFLS_EINVAL with a message retrievable by sfls_last_error().
 *    Numerical failures are reported per instance through `status` arrays.
 *  - A context is not thread-safe; use one context per host thread.  Calls
 *    on one context must not overlap (they share its workspace).
 */
#ifndef SFLS_H
#define SFLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SFLS_OK = 0,
    SFLS_NOTCONV = 1,     /* per instance: iteration cap reached, estimate returned */
    SFLS_EINVAL = -1,     /* bad argument (host-side check) */
    SFLS_ENOMEM = -2,     /* device allocation failed */
    SFLS_EDEVICE = -3,    /* HIP runtime error */
    SFLS_ENOTPD = -4,     /* per instance: Toeplitz matrix not positive definite */
    SFLS_ECAPACITY = -5,  /* per instance: more components wanted than kcap */
    SFLS_EUNSUPPORTED = -6, /* size outside what this build handles */
    SFLS_EAGAIN = -7      /* server: no free slot or device memory for the request now */
} sfls_status;

typedef enum { SFLS_FP64 = 0, SFLS_MIXED = 1 } sfls_precision; /* MIXED: FP32 grid FFTs */
typedef enum { SFLS_C64 = 0, SFLS_C128 = 1 } sfls_dtype;

/* Largest N accepted by this build (the superfast recursion; the Levinson
 * recursion handles N <= 4096).  Transforms that do not fit one CU's LDS
 * (P = 2N > 8192, superfast merges above 4096 points) run on per-instance
 * scratch in device memory. */
#define SFLS_MAX_N 65536

typedef struct sfls_ctx sfls_ctx;

/* Estimator parameters.  sfls_params_default() fills the paper's values:
 * tau = 5 (eq. activate_criterion), J = 10 (Sec. II-D), at most 5 inner
 * L-BFGS steps and a squared-Newton-decrement stop at N*1e-8, outer stop at
 * |dL| < N*1e-7 (Sec. II-E), L = 2^round(log2(8N)) (footnote, Sec. II-F),
 * approximate activation filters Delta L <= Delta L_min / 5 and wrap
 * distance >= 0.05/N (Sec. II-F). */
typedef struct {
    double L_mult;          /* grid oversampling: L = 2^round(log2(L_mult*N)) */
    double tau;             /* activation threshold adjustment */
    int32_t lbfgs_J;        /* L-BFGS memory, 1..16 */
    int32_t max_inner;      /* step-4 repetitions per outer iteration */
    int32_t max_outer;      /* outer iteration cap (then status SFLS_NOTCONV) */
    int32_t approx_max_iters; /* outer iterations that may use approximate activation (0: never) */
    int32_t approx_use_tau; /* 1: tau also in the approximate scheme's criterion (default 0:
                             * eq. activate_derived, as Sec. II-F states) */
    int32_t ls_max;         /* backtracking trials per line search */
    int32_t polish_max_iters; /* final (theta,gamma) polish iterations */
    int32_t cand_cap;       /* max candidates re-checked per approximate sweep */
    double tol_obj;         /* outer stop: |L_i - L_{i-1}| < N*tol_obj */
    double tol_newton;      /* inner stop: lambda^2 < N*tol_newton */
    double eps_beta_rel;    /* beta >= eps_beta_rel * ||y||^2 / N */
    double eps_L;           /* activation needs Delta L < -eps_L */
    double approx_ratio;    /* Delta L <= Delta L_min / approx_ratio */
    double approx_min_dist; /* wrap distance >= approx_min_dist / N */
    double ls_c1;           /* Armijo constant */
    double curv_eps;        /* keep an L-BFGS pair only if s'y > curv_eps |s||y| */
    double polish_tol;      /* polish stops when max |dtheta| < polish_tol / N */
    double polish_ftol;     /* polish accepts f_new <= f + c1 a g'd + polish_ftol (1+|f|) */
    int32_t precision;      /* sfls_precision of the grid stage */
    int32_t reserved;
} sfls_params;

void sfls_params_default(sfls_params* p);

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory of the context's workspace (grown on demand by the calls below to the
 * largest batch seen; about 2.3 MB per instance of N = 4096 for sfls_estimate):
 * a call whose batch would need more returns SFLS_ENOMEM with nothing enqueued
 * beyond what was already done; 0 = no cap.  The twiddle tables (about 6 MB,
 * allocated here) and servers' pools (sfls_server_config.hbm_bytes) are not
 * counted.  Returns SFLS_EDEVICE if the device cannot be used, SFLS_ENOMEM if
 * the tables cannot be allocated. */
sfls_status sfls_create(sfls_ctx** ctx, int device, size_t hbm_budget_bytes);
sfls_status sfls_destroy(sfls_ctx* ctx);
const char* sfls_strerror(sfls_status s);
/* Message of the last error on this context ("" if none).  Valid until the
 * next call on the context. */
const char* sfls_last_error(const sfls_ctx* ctx);
/* Library version string. */
const char* sfls_version(void);

/* ---------------------------------------------------------------------------
 * a1. Toeplitz generator of the covariance (Sec. II-B eq. py; Sec. III):
 *     c_i = beta [i = 0] + sum_k gamma_k exp(j 2 pi i theta_k), i = 0..N-1,
 * the first column of C = beta I + Psi(theta) diag(gamma) Psi(theta)^H.
 *   B instances; n/off (host) describe c; theta, gamma (device, f64) hold
 *   K[b] entries from koff[b] (host arrays K, koff); beta (device, f64 [B]).
 *   c (device, c128, sum n) is written.
 * ------------------------------------------------------------------------- */
sfls_status sfls_toeplitz_column(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                                 const int64_t* K, const int64_t* koff, const double* theta,
                                 const double* gamma, const double* beta, double* c,
                                 void* stream);

/* ---------------------------------------------------------------------------
 * a2. sfls_factor: Gohberg-Semencul generator of a Hermitian positive-definite
 * Toeplitz matrix C with first column c (Sec. III, eq. gohberg-semencul):
 *     C^{-1} = delta_{N-1}^{-1} (T1^H T1 - T0 T0^H),
 *     [T0]_{ik} = rho_{i-k-1}, [T1]_{ik} = rho_{N-1+i-k}, rho_{N-1} = 1,
 * computed by the Levinson-Durbin recursion or the superfast Schur recursion
 * (sfls_set_factor).  The superfast result is followed by one step of
 * iterative refinement of the last column of C^{-1} (residual by an FFT
 * Toeplitz product, correction by the Gohberg-Semencul formula), which
 * updates rho and delta_{N-1}; ln|C| and the other pivots are the recursion's.
 *   c      device c128 [sum n]   first columns; c_0 must be real and > 0
 *   rho    device c128 [sum n]   out: generator rho_0..rho_{N-1}
 *   delta  device f64  [sum n]   out: pivots delta_0..delta_{N-1} of C = L diag(delta) L^H
 *   logdet device f64  [B]       out: ln|C| = sum_i ln delta_i (Sec. III-A)
 *   status device i32  [B]       out: SFLS_OK or SFLS_ENOTPD
 *   failed_step device i64 [B]   out: first step n with delta_n <= 0 (or -1)
 * 1 <= n[b] <= SFLS_MAX_N, else SFLS_EUNSUPPORTED; the Levinson recursion
 * (sfls_set_factor) requires n[b] <= 4096, else SFLS_EUNSUPPORTED.
 * ------------------------------------------------------------------------- */
sfls_status sfls_factor(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                        const double* c, double* rho, double* delta, double* logdet,
                        int32_t* status, int64_t* failed_step, void* stream);

/* ---------------------------------------------------------------------------
 * a3. Choice of the factorisation used by sfls_factor and sfls_estimate.  Both
 * produce the same generator (rho, delta) of eq. gohberg-semencul:
 *   SFLS_FACTOR_LEVINSON  Levinson-Durbin, O(N^2) (Sec. III);
 *   SFLS_FACTOR_SCHUR     superfast doubling Schur recursion, O(N log^2 N)
 *                         (the generalized Schur route of Sec. III): a 2x2
 *                         polynomial-matrix recursion with FFT products;
 *   SFLS_FACTOR_AUTO      Schur for batches whose largest N >= 256 (default).
 * ------------------------------------------------------------------------- */
typedef enum { SFLS_FACTOR_AUTO = 0, SFLS_FACTOR_LEVINSON = 1, SFLS_FACTOR_SCHUR = 2 } sfls_factor_algo;
sfls_status sfls_set_factor(sfls_ctx* ctx, int32_t algo);

/* a3. Largest transform of the superfast recursion's merges kept in LDS
 * (a power of two in 256..4096, default 4096); larger merges run the same
 * passes on the instance's device scratch.  A lower limit shrinks the
 * recursion kernel's LDS so that several instances share a CU; it changes the
 * rounding of the merges it moves (not their arithmetic).  Applies to
 * sfls_factor and sfls_estimate calls, and to servers created afterwards.
 * SFLS_EINVAL outside the range. */
sfls_status sfls_set_schur_lds(sfls_ctx* ctx, int32_t max_f);

/* ---------------------------------------------------------------------------
 * a1, a8. How the products with Psi(theta) at off-grid frequencies are
 * evaluated (Sec. III-B and III-C use the non-uniform FFT): direct O(N) sums
 * per frequency, or Gaussian gridding (Greengard and Lee) on an oversampled
 * grid of P = 2^ceil(log2(2N-1)) points with 32 grid points per frequency,
 * whose relative error is below 1e-13 (measured 1e-15 .. 2e-14).
 *   a8 (sfls_active_eval, sfls_estimate): the type-2 transform at the active
 *   frequencies and grid candidates;
 *   a1 (sfls_toeplitz_column, sfls_estimate, servers): the type-1 transform
 *   for the covariance column, for instances with P > 8192 (N > 4096) and at
 *   most 2048 frequencies (direct sums otherwise).
 *   SFLS_NUFFT_AUTO  per instance: a8 when N >= 512 and (frequencies) x N
 *                    >= 2^23; a1 when K x N >= 2^21 (default)
 *   SFLS_NUFFT_OFF   direct sums everywhere
 *   SFLS_NUFFT_ON    NUFFT for every instance within the sizes above (a8:
 *                    at most 3P/4 frequencies)
 * The choice depends only on the instance, so a result does not depend on
 * the batch around it.  Unknown modes: SFLS_EINVAL.
 * ------------------------------------------------------------------------- */
typedef enum { SFLS_NUFFT_AUTO = 0, SFLS_NUFFT_OFF = 1, SFLS_NUFFT_ON = 2 } sfls_nufft_mode;
sfls_status sfls_set_nufft(sfls_ctx* ctx, int32_t mode);

/* ---------------------------------------------------------------------------
 * Speculative line-search trials in sfls_estimate (complete data, one
 * observation vector, at most one instance per compute unit).  The line
 * searches of the estimator (the inner L-BFGS steps of Sec. II-D and the
 * refinement that follows termination) try a step and, if it is rejected,
 * the step of half the length next.  With speculation on (1, the default)
 * each instance has a shadow evaluation slot (its own copy of the signal and
 * work arrays, doubling the call's workspace): when a trial is requested
 * whose rejection would not end the search, the point of the halved step is
 * written to the shadow.  After the harness passes the shadows are
 * granted evaluation on the compute units whose own instance requested none,
 * and only while at most half the compute units evaluate, so that a shadow
 * never waits behind a busy one.  A rejection then continues with the
 * shadow's evaluation in the same round.  The points evaluated, their
 * arithmetic and every output (K, theta, alpha, gamma, beta, zeta,
 * objective, iters, evals, status) are those with speculation off; only the
 * number of rounds (and the work of unused shadows) changes.  A context
 * created with an HBM budget does not speculate (the shadows would double
 * the workspace its budget was sized for).  0 turns it off; other values:
 * SFLS_EINVAL.
 * ------------------------------------------------------------------------- */
sfls_status sfls_set_speculation(sfls_ctx* ctx, int32_t enable);

/* ---------------------------------------------------------------------------
 * a4. w = C^{-1} y from the generator by four triangular-Toeplitz products
 * done as FFT convolutions (Sec. III-A); yCy[b] = Re(y^H w), ww[b] = ||w||^2.
 *   y device (ydtype) [sum n]; rho device c128; delta device f64 (only
 *   delta_{N-1} of each instance is read); w device c128 out; yCy, ww device
 *   f64 [B] out (either may be NULL).
 * ------------------------------------------------------------------------- */
sfls_status sfls_gs_apply(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                          const void* y, int32_t ydtype, const double* rho, const double* delta,
                          double* w, double* yCy, double* ww, void* stream);

/* ---------------------------------------------------------------------------
 * sfls_gs_apply_noalloc: sfls_gs_apply for callers that cannot allocate device
 * memory during the call (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * sfls_gs_apply; the instance table and the convolution scratch (4 P complex
 * values per instance, plus a P-point transform buffer when P > 8192) come
 * from one static device array of SFLS_NOALLOC_SCRATCH_BYTES that every device
 * the library runs on holds until the process ends (its address is looked up
 * once per device by sfls_create).  The call allocates nothing; it copies the
 * table from host memory on `stream` and returns after the stream has
 * finished the apply.  A batch whose table and scratch exceed the array
 * returns SFLS_EUNSUPPORTED before anything is enqueued (it holds at most 127
 * instances of N = 4096, or 6 of N = 65536).
 * Every call on a device shares that device's array: calls that overlap on
 * one device (from several threads, contexts or streams) race and must be
 * serialised by the caller.
 * ------------------------------------------------------------------------- */
#define SFLS_NOALLOC_SCRATCH_BYTES (64u << 20)
sfls_status sfls_gs_apply_noalloc(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                                  const void* y, int32_t ydtype, const double* rho,
                                  const double* delta, double* w, double* yCy, double* ww,
                                  void* stream);

/* ---------------------------------------------------------------------------
 * a5. Diagonal sums (Sec. III-C, eqs. omega_s, omega_t, omega_v, omega_x):
 *   omega_s(i) = sum_q [C^{-1}]_{q,q+i},   omega_t: D C^{-1},
 *   omega_v: D^2 C^{-1},  omega_x: D C^{-1} D,   D = diag(2 pi n),
 * for lags i = -(N-1)..N-1, computed from (rho, delta_{N-1}) as FFT
 * correlations of rho with its moment sequences n^a rho_n (Appendix B).
 *   out device c128 [sum (2 n - 1)] per requested array (NULL = not wanted);
 *   instance b writes 2n[b]-1 entries from oout[b] (host), lag i at i+n-1.
 * ------------------------------------------------------------------------- */
sfls_status sfls_omega(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                       const int64_t* oout, const double* rho, const double* delta,
                       double* omega_s, double* omega_t, double* omega_v, double* omega_x,
                       void* stream);

/* ---------------------------------------------------------------------------
 * a4-a7. sfls_grid_eval: what the activation step and its refinement need on
 * the grid theta^G_l = l/L (Sec. III-D), from y and the generator (rho, delta):
 *   q^G_l = psi^H(l/L) C^{-1} y,          s^G_l = psi^H(l/L) C^{-1} psi(l/L)
 *           (FFTs of w = C^{-1} y and of the diagonal sums omega_s),
 *   r^G_l = psi^H(l/L) D C^{-1} y,        t^G_l = psi^H(l/L) D C^{-1} psi(l/L)
 *           (eqs. r and t on the grid: FFTs of D w and of omega_t; D = diag(2 pi n);
 *           so that dq/dtheta = -j r and ds/dtheta = 2 Im t on the grid),
 *   Delta L_l = ln((1 + gb s)(1-zeta)/zeta) - |q|^2/(gb^{-1} + s)  (eq. delta_L)
 * with gb = gamma_bar[b] (> 0), or the per-point optimum of eq. activate_gamma
 * when gamma_bar[b] <= 0 (empty active set), and argmin_l Delta L (lowest l
 * on ties).
 *   out_mask   SFLS_GRID_* bits of the outputs to compute; an output whose bit
 *              is set must be non-NULL (else SFLS_EINVAL), the others are ignored.
 *              SFLS_GRID_ARGMIN writes argmin and/or argmin_val (either may be NULL,
 *              not both).  gamma_bar and zeta (device f64 [B]) are read only for
 *              SFLS_GRID_DL / SFLS_GRID_ARGMIN.
 *   L (host i64 [B]) grid sizes: powers of two with L >= 2n-1;
 *   goff (host i64 [B]) offsets of each instance's grid in qG/sG/rG/tG/dL.
 *   Precision (per `precision`): FP64 = c128 qG/rG/tG, f64 sG/dL; MIXED = the
 *   FP32 grid: c64 qG/rG/tG, f32 sG/dL (w, omega and the generator stay FP64).
 *   argmin i64 [B] and argmin_val f64 [B].
 * out_mask = 0 returns SFLS_OK and does nothing; unknown bits are SFLS_EINVAL.
 * ------------------------------------------------------------------------- */
typedef enum {
    SFLS_GRID_Q = 1, SFLS_GRID_S = 2, SFLS_GRID_R = 4, SFLS_GRID_T = 8,
    SFLS_GRID_DL = 16, SFLS_GRID_ARGMIN = 32, SFLS_GRID_ALL = 63
} sfls_grid_out;
sfls_status sfls_grid_eval(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                           const void* y, int32_t ydtype, const double* rho, const double* delta,
                           const int64_t* L, const int64_t* goff, const double* gamma_bar,
                           const double* zeta, uint32_t out_mask, void* qG, void* sG, void* rG,
                           void* tG, void* dL, int64_t* argmin, double* argmin_val,
                           int32_t precision, void* stream);

/* ---------------------------------------------------------------------------
 * a8. Active-set vectors at K[b] frequencies theta (Sec. II-D, eqs. q-x):
 *   q = Psi^H w, r = Psi^H D w, u = Psi^H D^2 w,
 *   s, t, v, x = diag(Psi^H {I, D, D^2, D .. D} C^{-1} Psi)
 * from w = C^{-1} y and the generator (rho, delta).  Outputs are c128 device
 * arrays of sum K entries (instance b from koff[b], host); NULL skips one.
 * Computed by direct sums or by the NUFFT per sfls_set_nufft.
 * ------------------------------------------------------------------------- */
sfls_status sfls_active_eval(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                             const double* w, const double* rho, const double* delta,
                             const int64_t* K, const int64_t* koff, const double* theta,
                             double* q, double* r, double* u, double* s, double* t, double* v,
                             double* x, void* stream);

/* ---------------------------------------------------------------------------
 * a1-a9. sfls_estimate: the full estimator (Sec. II-C..F, Sec. III) for a
 * ragged batch, every step in device kernels, state resident on the device
 * across iterations.
 *   y      device (ydtype) [sum n]  observations
 *   params host (NULL = defaults)
 *   kcap   host i64 [B]  capacity of instance b's component outputs (>= 1)
 *   koff   host i64 [B]  offset of instance b's outputs in theta/alpha/gamma
 *   K      device i64 [B]        out: model order
 *   theta  device f64 [sum kcap] out: frequencies, ascending in [0,1)
 *   alpha  device c128 [sum kcap] out: amplitudes gamma .* q (eq. bmu footnote)
 *   gamma  device f64 [sum kcap] out: component variances
 *   beta, zeta, objective device f64 [B] out
 *   iters  device i32 [B] out: outer iterations;  evals device i32 [B] (may be NULL)
 *   status device i32 [B] out: SFLS_OK, SFLS_NOTCONV, SFLS_ECAPACITY, SFLS_ENOTPD
 * 2 <= n[b] <= SFLS_MAX_N.  The call returns after the batch has finished on
 * `stream`: it runs evaluation rounds (the evaluations the instances asked
 * for, a driver pass, the grid stage, a second driver pass).  The driver
 * writes each round's request bits into pinned host memory; the host reads
 * them one round behind, with round r + 1 already enqueued (every kernel of a
 * round takes only the instances whose bits name it), and stops once a round
 * leaves no request.  A batch of uneven N is dispatched longest first.
 * ------------------------------------------------------------------------- */
sfls_status sfls_estimate(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                          const void* y, int32_t ydtype, const sfls_params* params,
                          const int64_t* kcap, const int64_t* koff, int64_t* K, double* theta,
                          double* alpha, double* gamma, double* beta, double* zeta,
                          double* objective, int32_t* iters, int32_t* evals, int32_t* status,
                          void* stream);

/* ---------------------------------------------------------------------------
 * a1-a9 with multiple measurement vectors (Sec. V): G observation vectors per
 * instance, y^(g) = A(theta) alpha^(g) + w^(g), sharing theta, gamma, beta and
 * zeta.  The covariance C and its generator are those of the single-vector
 * model, so each evaluation factors C once; C^{-1} y, q, r, u, the grid's
 * q^G and y^H C^{-1} y are computed per vector.  The objective is
 * G ln|C| + sum_g y_g^H C^{-1} y_g - prior; its derivatives are the sums over
 * g of eqs. derivative/derivative2; activation, deactivation and gamma come
 * from eq. singlecomp-mmv; beta is the MMV update of Sec. V.  Where Sec. V
 * leaves details to the reader: the activation criterion is eq.
 * activate_criterion applied to the per-vector average |q|^2, i.e.
 * sum_g |q_g|^2 / (G s) > (1 + 1/(gb s)) (ln(1 + gb s) + ln((1-zeta)/zeta)/G)
 * + tau; the stopping rules scale with G N (the objective is a sum of G
 * single-vector objectives); beta starts at 0.01 sum_g ||y_g||^2 / (G N).
 * G = 1 is sfls_estimate.
 *   G         1..SFLS_MAX_VECTORS, the same for every instance of the call
 *   y         device (ydtype): vector g of instance b is n[b] samples at
 *             y + g * ystride + off[b] (elements); ystride >= off[b] + n[b]
 *   alpha     device c128 out: vector g's amplitudes of instance b, K[b] of
 *             them, at alpha + g * alpha_stride + koff[b] (complex elements);
 *             alpha_stride >= koff[b] + kcap[b]
 *   the other arguments and outputs as sfls_estimate.
 * The active-set vectors use direct sums (no NUFFT) when G > 1.  Errors:
 * SFLS_EINVAL for G outside the range or strides smaller than the layout
 * needs, otherwise as sfls_estimate.
 * ------------------------------------------------------------------------- */
#define SFLS_MAX_VECTORS 64
sfls_status sfls_estimate_mmv(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* off,
                              int32_t G, const void* y, int64_t ystride, int32_t ydtype,
                              const sfls_params* params, const int64_t* kcap, const int64_t* koff,
                              int64_t* K, double* theta, double* alpha, int64_t alpha_stride,
                              double* gamma, double* beta, double* zeta, double* objective,
                              int32_t* iters, int32_t* evals, int32_t* status, void* stream);

/* ---------------------------------------------------------------------------
 * Incomplete observations (Sec. IV): Phi keeps M of the N samples, each
 * scaled by a nonzero weight (M rows of a diagonal matrix; the footnote of
 * Sec. IV), so y in C^M and C = beta I_M + A Gamma A^H with A = Phi Psi.  The
 * evaluation uses the semifast method of Sec. IV: Woodbury's identity with the
 * K x K matrix K_s = beta I + Gamma^{1/2} A^H A Gamma^{1/2} (eqs. CfromSigma,
 * AhA), its Cholesky factor, and the matrix determinant lemma for ln|C|;
 * s, t, v, x from the Gram sums A^H D^p A, and on the grid q^G from
 * Phi^H C^{-1} y and s^G from the diagonal sums of Phi^H C^{-1} Phi (one
 * autocorrelation by FFT per active component).
 * Observation arguments of both calls:
 *   n     host i64 [B]  signal lengths N (2 <= n <= SFLS_MAX_N)
 *   m     host i64 [B]  observed samples M (1 <= m <= n)
 *   moff  host i64 [B]  offset of instance b's observations in idx, phi, y
 *   idx   device i32 [sum m] observed sample indices, strictly increasing in
 *         [0, n) per instance (checked on the device first: SFLS_EINVAL)
 *   phi   device c128 [sum m] weights, nonzero and finite; NULL: all 1
 *   y     device (ydtype) [sum m] observed samples
 * Components: at most SFLS_SF_MAX_K per instance (the factor and its inverse
 * are kept on chip); the model order's capacity is min(kcap, m, SFLS_SF_MAX_K)
 * (K_max = M: the footnote of Sec. II-A).
 * ------------------------------------------------------------------------- */
#define SFLS_SF_MAX_K 64

/* One semifast evaluation at K[b] components (theta, gamma device f64 at
 * koff[b]; beta device f64 [B]):
 *   logdet, yCy, ww  device f64 [B] out: ln|C|, y^H C^{-1} y, ||C^{-1} y||^2
 *   q, r, u, s, t, v, x  device c128 out at koff (eqs. q-x with Phi)
 *   L, goff (host i64 [B]; NULL: no grid) with qG (c128) / sG (f64) device
 *   out at goff: q^G and s^G on theta = l/L, FP64 (each may be NULL);
 *   cand (device i32 at coff), ncand, coff (host i64 [B]) with cq (c128),
 *   cs (f64) device out at coff: q and s at theta = cand / L (needs L).
 *   status device i32 [B] out (may be NULL): 0, or SFLS_ENOTPD when K_s is
 *   not positive definite (the instance's other outputs are then undefined).
 * Any output may be NULL; K[b] <= min(m[b], SFLS_SF_MAX_K). */
sfls_status sfls_incomplete_eval(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* m,
                                 const int64_t* moff, const int32_t* idx, const double* phi,
                                 const void* y, int32_t ydtype, const int64_t* K,
                                 const int64_t* koff, const double* theta, const double* gamma,
                                 const double* beta, double* logdet, double* yCy, double* ww,
                                 double* q, double* r, double* u, double* s, double* t, double* v,
                                 double* x, const int64_t* L, const int64_t* goff, double* qG,
                                 double* sG, const int32_t* cand, const int64_t* ncand,
                                 const int64_t* coff, double* cq, double* cs, int32_t* status,
                                 void* stream);

/* The estimator (Sec. II) on incomplete observations, every evaluation by the
 * semifast method: sfls_estimate's algorithm, outputs and round loop, with the
 * count scales of Sec. II-E in M (initial beta = 0.01 ||y||^2 / M, eps_beta,
 * the stopping rules M 1e-7 and M 1e-8, K_max = M in the prior and eq.
 * zetaUpdate) and the frequency scales in N (grid L = 2^round(log2(L_mult N)),
 * distances 0.05/N, the refinement's 1e-12/N).  kcap, koff, K, theta, alpha,
 * gamma, beta, zeta, objective, iters, evals and status as in sfls_estimate
 * (status SFLS_ECAPACITY also when the model order would exceed
 * SFLS_SF_MAX_K).  Every sample observed with unit weights estimates what
 * sfls_estimate does, by another evaluation route. */
sfls_status sfls_estimate_incomplete(sfls_ctx* ctx, int64_t B, const int64_t* n, const int64_t* m,
                                     const int64_t* moff, const int32_t* idx, const double* phi,
                                     const void* y, int32_t ydtype, const sfls_params* params,
                                     const int64_t* kcap, const int64_t* koff, int64_t* K,
                                     double* theta, double* alpha, double* gamma, double* beta,
                                     double* zeta, double* objective, int32_t* iters,
                                     int32_t* evals, int32_t* status, void* stream);

/* ---------------------------------------------------------------------------
 * Measurement of sfls_estimate (no effect on results).
 *
 * sfls_set_timing(ctx, 1) brackets every kernel launch of the estimate round
 * loop (and of the rounds of servers created on the context) with HIP events
 * on the stream the work runs on; sfls_set_timing(ctx, 2) brackets only the
 * recursion's launches (an event between two kernels costs the device a few
 * microseconds of idle time; mode 2 keeps that out of the other kernels);
 * 0 turns timing off, other values are EINVAL.  Per timed kernel the context then
 * accumulates the launch count, the summed event durations, and the
 * algorithmic work of those launches (FP64 flops of the factorisation: 8 N^2
 * per instance for Levinson, the count of the superfast recursion's leaf
 * steps, polynomial products and transforms for Schur; HBM bytes of the
 * streamed arrays), counted from the request bits of each round.  sfls_kernel_stats copies up to `cap` entries
 * and returns the number of kernels tracked; sfls_reset_stats zeroes them.
 * sfls_last_run returns the round / evaluation counts of the last estimate
 * and the host wall time at the end of each round (entry r = after round r,
 * entry 0 = after the initial driver call), so instance b with evals[b] = r
 * completed at timeline[r].
 * ------------------------------------------------------------------------- */
typedef struct {
    char name[24];
    int64_t launches;
    double seconds;
    double flops;
    double bytes;
} sfls_kernel_stat;

typedef struct {
    int64_t rounds;      /* evaluation rounds */
    int64_t evals;       /* instance evaluations, summed over rounds */
    int64_t grid_evals;  /* of which ran the grid stage */
    double wall_seconds; /* host wall time of the call */
} sfls_run_stats;

sfls_status sfls_set_timing(sfls_ctx* ctx, int32_t enable);
void sfls_reset_stats(sfls_ctx* ctx);
int32_t sfls_kernel_stats(const sfls_ctx* ctx, sfls_kernel_stat* out, int32_t cap);
sfls_status sfls_last_run(const sfls_ctx* ctx, sfls_run_stats* stats, double* timeline,
                          int64_t cap, int64_t* ntimeline);

/* ---------------------------------------------------------------------------
 * Serving: the estimator of sfls_estimate (Sec. II-C..F on the Sec. III
 * evaluations) for requests that arrive over time, by continuous batching.
 *
 * A server owns a pool of device memory of cfg.hbm_bytes and cfg.max_slots
 * slots.  sfls_server_submit admits a request when a slot is free and the
 * request's footprint (sfls_server_footprint: every per-request array of the
 * round loop, sized by N rounded up to a power of two, at least 64) fits in
 * the pool (a buddy allocation); otherwise it returns SFLS_EAGAIN and the
 * server is unchanged.  Admission does not wait for the device: the request's
 * tables and a device-resident signal are copied into the pools by a kernel
 * at the start of the next round (a host-resident signal is copied before the
 * call returns).  Each round (sfls_server_launch) runs one
 * evaluation for every admitted request that has asked for one, whatever its
 * N, in the same kernels, then a driver pass, the grid stage for the requests
 * whose step asks for a grid sweep (those at the point the round just
 * evaluated included) and a second driver pass for them; requests admitted
 * since the previous round take their first driver step at its start and are
 * evaluated in it.  Requests of different N are dispatched longest first.
 * sfls_server_wait completes the round: requests
 * whose estimate finished release their slot and memory at once, and a short
 * kernel behind the round packs their outputs for sfls_server_poll (which
 * waits for it), so the next round can be launched before the results are
 * read.  All state of a request (theta, gamma, beta,
 * zeta, the L-BFGS memory, the generator) stays on the device until then.
 *
 * A request's result does not depend on the other requests in the pool: each
 * kernel computes every instance from its own arrays, and the launch shapes
 * that change the order of a computation are fixed per server (the
 * factorisation is chosen from cfg.max_n as sfls_set_factor does, its LDS
 * transform size from the largest N).  Results can differ in rounding from
 * an sfls_estimate call whose batch has a different largest N.
 *
 * Not thread-safe; one host thread drives a server.  Several servers (for
 * instance one per size class, each on its own stream) can run their rounds
 * concurrently: launch each, then wait on each.
 * ------------------------------------------------------------------------- */
typedef struct sfls_server sfls_server;

typedef struct {
    int64_t max_n;       /* largest request length (2..SFLS_MAX_N) */
    int32_t max_slots;   /* requests held on the device at once (1..65536) */
    int32_t ydtype;      /* sfls_dtype of submitted signals */
    uint64_t hbm_bytes;  /* device memory for request state (pool + per-slot arrays) */
    int32_t kcap_shift;  /* component capacity of a request: min(N, max(N,64)-rounded-to-2^k >> kcap_shift), 0..6 */
    int32_t reserved;
    void* stream;        /* hipStream_t for the server's work; NULL: the server creates one */
} sfls_server_config;

typedef struct {
    uint64_t tag;        /* the caller's tag from sfls_server_submit */
    int64_t n;           /* request length */
    int64_t K;           /* model order: number of components */
    int64_t comp_off;    /* components at theta/gamma[comp_off..+K), alpha[2 comp_off..+2K) */
    double beta, zeta, objective;
    int32_t iters, evals, status, reserved;
    double t_submit;     /* seconds since server creation: admission */
    double t_done;       /* seconds since server creation: end of the round that finished it */
} sfls_result;

typedef struct {
    int64_t rounds;        /* rounds completed */
    int64_t admitted;      /* requests admitted */
    int64_t completed;     /* results produced */
    int64_t in_flight;     /* requests holding a slot */
    int64_t units_used;    /* pool units (samples) allocated */
    int64_t units_total;   /* pool units */
    uint64_t bytes_per_unit;
    uint64_t bytes_reserved; /* device memory held by the server */
    double gpu_seconds;    /* host wall time between launch and the end of each round, summed */
} sfls_server_stats;

/* max_n 65536, 1024 slots, c64 input, 8 GiB, kcap_shift 0 (K_max = N, footnote of
 * Sec. II-A), own stream. */
void sfls_server_config_default(sfls_server_config* cfg);
/* Create a server on ctx's device (ctx must outlive it).  params: NULL =
 * sfls_params_default.  SFLS_EINVAL for bad sizes or a pool too small for one
 * request of max_n; SFLS_ENOMEM if the device memory is not available. */
sfls_status sfls_server_create(sfls_ctx* ctx, const sfls_server_config* cfg,
                               const sfls_params* params, sfls_server** out);
/* Waits for outstanding work and frees everything the server holds. */
sfls_status sfls_server_destroy(sfls_server* srv);
/* Device bytes a request of length n reserves from the pool. */
sfls_status sfls_server_footprint(const sfls_server* srv, int64_t n, uint64_t* bytes);
/* Admit a request: y (cfg.ydtype, n elements).  A device pointer (8-byte
 * aligned) is read by the next round, so y must stay valid and unchanged until
 * the next sfls_server_wait returns; a host pointer is copied before return.
 * SFLS_EAGAIN: no free slot or pool memory now (retry after a round);
 * SFLS_EINVAL: n < 2, NULL or misaligned y; SFLS_EUNSUPPORTED: n > max_n. */
sfls_status sfls_server_submit(sfls_server* srv, const void* y, int64_t n, uint64_t tag);
/* Admit requests 0, 1, ... of ys / ns / tags (host arrays of `count`) in order,
 * each as sfls_server_submit does, until all are admitted or one is not
 * (SFLS_EAGAIN ends the call with SFLS_OK); *accepted = the number admitted.
 * Any other status of a request is returned, with *accepted = the requests
 * before it.  One call instead of `count`, for hosts whose per-call overhead
 * would otherwise sit between two rounds.  SFLS_EINVAL: NULL srv or accepted,
 * count < 0, or NULL arrays with count > 0. */
sfls_status sfls_server_submit_many(sfls_server* srv, int32_t count, const void* const* ys,
                                    const int64_t* ns, const uint64_t* tags, int32_t* accepted);
/* Enqueue one round on the server's stream (no-op when nothing is admitted
 * or a round is already in flight).  Returns without waiting. */
sfls_status sfls_server_launch(sfls_server* srv);
/* Complete the round in flight.  block = 0: return at once with *ready = 0
 * if the device has not finished it.  *ready = 1 when the round was completed
 * (or none was in flight).  *finished (may be NULL) = results it produced. */
sfls_status sfls_server_wait(sfls_server* srv, int32_t block, int32_t* ready, int32_t* finished);
/* sfls_server_launch followed by a blocking sfls_server_wait. */
sfls_status sfls_server_step(sfls_server* srv, int32_t* finished);
/* Move up to max_results finished results, oldest first, into res (host),
 * their components into theta, gamma (host f64 [comp_cap]) and alpha (host
 * f64 pairs [2 comp_cap]); stops before a result whose components would not
 * fit.  *nres = results returned. */
sfls_status sfls_server_poll(sfls_server* srv, sfls_result* res, int32_t max_results,
                             double* theta, double* gamma, double* alpha, int64_t comp_cap,
                             int32_t* nres);
sfls_status sfls_server_get_stats(const sfls_server* srv, sfls_server_stats* stats);

#ifdef __cplusplus
}
#endif
#endif /* SFLS_H */
