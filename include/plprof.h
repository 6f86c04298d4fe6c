/*
 * plprof -- profile log-likelihoods of Box-Cox transformed Gaussian
 * geostatistical models with anisotropic Matern correlation, on one
 * MI355X (gfx950) GPU.
 *
 * C ABI.  All entry points return 0 (PL_OK) on success, -i when argument i
 * (1-based) is invalid (LAPACK convention), or a positive PL_E_* code for a
 * runtime failure.  Every device-side call is asynchronous on the HIP stream
 * passed in `stream` (a hipStream_t; NULL means the default stream); results
 * are valid once the caller has synchronised that stream.
 *
 * Ownership: the caller allocates and owns every device buffer, including the
 * workspace sized by the matching *_workspace_size call.  The library keeps
 * no device state between calls, except the fixed scratch array of
 * pl_profile_loglik_noalloc.  Host arrays (omega, lambda, options) are read
 * during the call only.
 *
 * Notation and definitions (Xu & Brown, "Profile likelihoods for parameters
 * in trans-Gaussian geostatistical models"):
 *   omega = (phi_X range, kappa shape, nu^2 nugget, phi_R ratio, phi_A angle),
 *   phi_Y = phi_X / phi_R, Section 2.1 and the parameter tables of Sections 6-7;
 *   rho(x) = 2^(1-kappa)/Gamma(kappa) (sqrt(8 kappa) d)^kappa K_kappa(sqrt(8 kappa) d),
 *   d(x) = || diag(1/phi_X, 1/phi_Y) Rot(phi_A) x ||, Section 2.1 (the printed
 *   constant 2^(kappa-1) is read as 2^(1-kappa), the value with rho(0) = 1);
 *   V = R(omega) + nu^2 I, equation (1);
 *   Box-Cox y' = (y^lambda - 1)/lambda, log y at lambda = 0, Section 2;
 *   profile log-likelihood l_p(omega, lambda), equation "profile" (returned as
 *   l_p itself, not -2 l_p), with the statistics of Table "tab:tocpu".
 */
#ifndef PLPROF_H
#define PLPROF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* precision modes */
#define PL_FP64  0      /* every step in FP64                                  */
#define PL_MIXED 1      /* FP32 trailing updates / solves on MFMA, FP64 diagonal
                           tiles, log-determinant, p x p stage and residual,
                           one FP64 iterative-refinement step                   */

/* storage types of pl_matern_cov */
#define PL_F64   0      /* double                                              */
#define PL_F32   1      /* float: each element computed in FP64, rounded once  */

/* runtime error codes (positive returns) */
#define PL_OK            0
#define PL_E_HIP         1   /* a HIP runtime call failed                       */
#define PL_E_WORKSPACE   2   /* workspace too small for even one omega          */
#define PL_E_UNSUPPORTED 3   /* size outside the compiled limits                */
#define PL_E_SCRATCH     4   /* pl_profile_loglik_noalloc: one omega needs more
                                than PL_NOALLOC_SCRATCH_BYTES                   */
#define PL_TUNE_MISS     5   /* pl_tune_lookup: no stored choice (not an error) */

/* per-record info codes */
#define PL_INFO_RANK     (-1)        /* X^T V^-1 X not positive definite        */
#define PL_INFO_BAD_Y    (-2)        /* some y_i <= 0 or not finite             */
#define PL_INFO_FALLBACK (1 << 30)   /* mixed form: point redone in FP64        */

/* compiled limits */
#define PL_MAX_P      32     /* covariates                                      */
#define PL_MAX_M      64     /* Box-Cox values per call                         */
#define PL_MAX_Q_MIXED 64    /* PL_MIXED: M + p (bordered right-hand sides)      */
#define PL_MIN_SHAPE  0.05
#define PL_MAX_SHAPE  100.0

/* One record per (omega_k, lambda_m), stored at index k*M + m (80 bytes). */
typedef struct pl_result {
  double loglik;        /* l_p(omega, lambda), equation "profile"               */
  double logdet_v;      /* log|V| (detVar)                                      */
  double logdet_xvx;    /* log|X^T V^-1 X| (detReml)                             */
  double ssq_y;         /* y'^T V^-1 y'                                         */
  double ssq_betahat;   /* (X b)^T V^-1 (X b) (ssqBetahat)                        */
  double ssq_resid;     /* (y' - X b)^T V^-1 (y' - X b) (ssqResidual)            */
  double sigma2_hat;    /* ssq_resid / n                                        */
  double jacobian;      /* sum_i log y_i                                         */
  double loglik_reml;   /* restricted profile log-likelihood, Appendix "remlpro" */
  int32_t info;         /* 0; j > 0: first non-positive pivot of V (column j,
                           1-based), loglik = -inf; PL_INFO_RANK; PL_INFO_BAD_Y
                           (loglik = NaN); PL_INFO_FALLBACK may be or-ed in      */
  int32_t pad;
} pl_result;

typedef struct pl_opts {
  int32_t precision;    /* PL_FP64 (default) or PL_MIXED                         */
  int32_t refine;       /* PL_MIXED: 1 (default) = one FP64 refinement of the
                           cross products (see pl_profile_loglik); 0 = none      */
  int64_t chunk;        /* max omega per device pass; 0 = as many as fit          */
  int32_t flags;        /* PL_OPT_* bits                                         */
  int32_t flush;        /* PL_MIXED: FP32 MFMA k-steps (4 products each) summed
                           in FP32 before each FP64 fold in the off-diagonal
                           updates: 1, 2 or 4; 0 = default (4).  Longer runs are
                           faster and less accurate; see pl_autotune            */
  int32_t wait_us;      /* pl_batch_create: wall-time limit of one task wait of
                           the persistent launch, microseconds; 0 = default
                           (PL_BATCH_WAIT_US).  A wait that outlives it makes
                           the launch drain without results (pl_batch_error)  */
  int32_t lanes;        /* pl_batch_create, size-bucketed schedule: streams the
                           passes are spread over (1-16; 0 = 4)               */
} pl_opts;

#define PL_BATCH_WAIT_US 4000000  /* 4 s: far above any legitimate task wait */

/* pl_opts.flags */
#define PL_OPT_NO_FALLBACK 1  /* PL_MIXED: do not synchronise to redo FP32
                                 breakdowns in FP64 (they keep info > 0)        */
#define PL_OPT_BATCH_PERSISTENT 2  /* pl_batch_create: the persistent-kernel
                                      schedule (PL_FP64 only)                   */

/* Library version string. */
const char* pl_version(void);

/* Human-readable text for a return code. */
const char* pl_error_string(int code);

/*
 * Workspace for pl_profile_loglik.  `bytes` receives the size that holds all
 * K points in one device pass; any workspace of at least the one-point size
 * (K = 1) is accepted, and the call then runs in chunks.
 * Errors: -1 n < 2, -2 p < 1 or p >= n or p > PL_MAX_P, -3 K < 1,
 * -4 M < 1 or M > PL_MAX_M, -6 bytes NULL.
 */
int pl_workspace_size(int64_t n, int64_t p, int64_t K, int64_t M,
                      const pl_opts* opts, size_t* bytes);

/*
 * Matern correlation-plus-nugget matrices V_k = R(omega_k) + nu_k^2 I
 * (Section 2.1, equation (1); Step 1 of Section 3.3, the paper's maternBatch,
 * whose precision is a per-call choice).
 *   locs   device, n x 2 row-major (x_i, y_i)
 *   omega  host, K x 5 row-major natural parameters
 *   dtype  PL_F64: V holds doubles; PL_F32: V holds floats, each element
 *          computed in FP64 and rounded once (the input of pl_chol_batched
 *          with PL_MIXED)
 *   V      device, K matrices, each n x n column-major with leading dimension
 *          ld >= n; matrix k starts at element k*ld*n.  The lower triangle and
 *          the diagonal are written; the strict upper triangle is not touched.
 *   work   device workspace of pl_matern_workspace_size(K) bytes.
 * Errors: -1 locs NULL, -2 n < 1, -3 omega NULL or a parameter out of domain
 * (range <= 0, shape outside [PL_MIN_SHAPE, PL_MAX_SHAPE], nugget < 0,
 * ratio <= 0, any value not finite), -4 K < 1, -5 dtype not PL_F64 or
 * PL_F32, -6 V NULL, -7 ld < n, -8/-9 workspace NULL or too small.
 */
int pl_matern_workspace_size(int64_t K, size_t* bytes);
int pl_matern_cov(const double* locs, int64_t n, const double* omega, int64_t K, int dtype,
                  void* V, int64_t ld, void* work, size_t work_bytes, void* stream);

/*
 * In-place batched Cholesky V_k = L_k L_k^T (Step 2 of Section 3.3, the
 * paper's cholBatch; it factors L D L^T, whose determinant is the same) with
 * logdet[k] = log|V_k| = 2 sum_i log L_k,ii.
 *   V         device, K matrices, n x n column-major, leading dimension ld,
 *             matrix k at element k*ld*n; the lower triangle is read and
 *             overwritten by L, the strict upper triangle is not referenced.
 *   precision PL_FP64: V holds doubles and every step is FP64.
 *             PL_MIXED: V holds floats (pl_matern_cov with PL_F32) and L is
 *             stored in FP32; off-diagonal updates and panel solves run on
 *             FP32 MFMA with their partial sums folded into FP64 every 16
 *             products, each diagonal tile is updated with FP64 accumulation
 *             and factored in FP64, so logdet is accumulated in FP64.  V must
 *             be 16-byte aligned and ld a multiple of 4.
 *   logdet    device, K doubles.  info device, K int32: 0, or j > 0 when the
 *             leading minor of order j is not positive definite (that matrix
 *             is left partly factored and logdet[k] is not meaningful).
 *   work      device workspace of pl_chol_workspace_size(K, precision) bytes.
 * Errors: -1 V NULL (or, PL_MIXED, not 16-byte aligned), -2 n < 1, -3 K < 1,
 * -4 ld < n (or, PL_MIXED, not a multiple of 4), -5 precision not PL_FP64 or
 * PL_MIXED, -6 logdet NULL, -7 info NULL, -8/-9 workspace NULL or too small.
 * pl_chol_workspace_size: -1 K < 1, -2 precision, -3 bytes NULL.
 */
int pl_chol_workspace_size(int64_t K, int precision, size_t* bytes);
int pl_chol_batched(void* V, int64_t n, int64_t K, int64_t ld, int precision,
                    double* logdet, int32_t* info, void* work, size_t work_bytes,
                    void* stream);

/*
 * Profile log-likelihood at every (omega_k, lambda_m) (Section 3.3, Steps 1-8;
 * equations "betahat", (4) and "profile"; Appendix "remlpro").
 *   locs     device, n x 2 row-major        y  device, n (must be > 0)
 *   X        device, n x p column-major (column j at X + j*n)
 *   omega    host, K x 5                      lambda host, M
 *   out      device, K*M pl_result records, record k*M + m
 *   beta_hat device, K*M*p doubles (GLS estimate for record k*M+m at
 *            beta_hat + (k*M+m)*p), or NULL
 *   xvx_inv  device, K*p*p doubles: (X^T V_k^-1 X)^-1 row-major at
 *            xvx_inv + k*p*p (NaN where it does not exist), or NULL.  With
 *            the records it gives the profiles of single coefficients and of
 *            sigma (Section 3.4, "Profile likelihood for beta_p" and "for
 *            sigma"); see pl_profile_curves.
 *   opts     NULL for defaults
 *   work     device workspace, see pl_workspace_size
 * Errors: -1 locs, -2 y, -3 X NULL; -4 n < 2; -5 p < 1, p >= n or p > PL_MAX_P;
 * -6 omega NULL or out of domain (as pl_matern_cov); -7 K < 1;
 * -8 lambda NULL or not finite; -9 M < 1 or M > PL_MAX_M; -10 out NULL;
 * -13 bad option; -14/-15 workspace NULL or too small; PL_E_UNSUPPORTED for
 * PL_MIXED with M + p > PL_MAX_Q_MIXED.
 * y <= 0 is detected on the device: every record then carries PL_INFO_BAD_Y.
 *
 * PL_MIXED: V is factored in FP32 (FP32 MFMA off-diagonal updates and panel
 * solves) with each diagonal tile updated from the FP64 V in FP64 and factored
 * in FP64, so log|V| is accumulated in FP64; x0 = V^-1 [Y'|X] comes from FP32
 * substitution; the cross products are then evaluated in FP64 as
 * 2 B^T x0 - x0^T V x0 (B = [Y'|X]), whose error is second order in the error
 * of x0 -- one FP64 refinement step applied to the quadratic forms; the p x p
 * stage is FP64.  Points whose FP32 factorisation breaks down are recomputed
 * with the FP64 form (info |= PL_INFO_FALLBACK); that check synchronises the
 * stream once at the end of the call unless PL_OPT_NO_FALLBACK is set.
 */
int pl_profile_loglik(const double* locs, const double* y, const double* X,
                      int64_t n, int64_t p, const double* omega, int64_t K,
                      const double* lambda, int64_t M, pl_result* out,
                      double* beta_hat, double* xvx_inv, const pl_opts* opts, void* work,
                      size_t work_bytes, void* stream);

/*
 * pl_profile_loglik without a caller workspace and without any device
 * allocation, for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * Arguments, results, error codes 1-13 and stream semantics are those of
 * pl_profile_loglik (stream is argument 14).  The workspace is a fixed device
 * array of PL_NOALLOC_SCRATCH_BYTES inside the library; each GPU holds its
 * own copy from the first call on it until the process ends.  The omega
 * points run in as many stream-ordered passes as the array needs.  The call
 * allocates no device memory and calls no allocating library routine; the
 * stream must belong to the current device.
 * Limits: PL_E_SCRATCH when one omega's workspace exceeds the array: FP64
 * n above about 8,050 (M + p <= 16) or 7,900 (M + p <= 32); PL_MIXED n above
 * about 6,400 (M + p <= 16), 6,250 (M + p <= 32) or somewhat less for taller
 * borders (M + p <= 64).
 * Calls that overlap on one GPU (different streams or host threads without
 * ordering between them) share the array and race; serialise them.
 */
#define PL_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)   /* 256 MiB per GPU */
int pl_profile_loglik_noalloc(const double* locs, const double* y, const double* X,
                              int64_t n, int64_t p, const double* omega, int64_t K,
                              const double* lambda, int64_t M, pl_result* out,
                              double* beta_hat, double* xvx_inv, const pl_opts* opts,
                              void* stream);

/*
 * Profile curves of sigma and of single regression coefficients from the
 * output of pl_profile_loglik (Sections 3.4 and 3.5, the profile
 * likelihoods for beta_p and for sigma, maximised over
 * the evaluated points as in Step 6).  For every grid value the curve is the
 * maximum over the usable records (info 0 or PL_INFO_FALLBACK) of
 *   sigma:   -1/2 [SSR/sigma^2 + n log sigma^2 + log|V| + n log 2 pi]
 *            + (lambda - 1) J                    (equation "profileSigma");
 *   beta_j:  the likelihood with beta_j fixed at b and the other coefficients
 *            and sigma at their constrained maximum-likelihood values,
 *            -1/2 [n log(SSR_b/n) + log|V| + n log 2 pi + n] + (lambda - 1) J
 *            with SSR_b = SSR + (b - betahat_j)^2 / [(X^T V^-1 X)^-1]_jj, the
 *            closed form of the cross-product identities of equation
 *            "profilebetai".
 *   rec, beta_hat, xvx_inv  device, as written by one pl_profile_loglik call
 *            (K*M records; beta_hat and xvx_inv may be NULL when Gb = 0)
 *   n, p, K, lambda (host, M values), M        as in that call
 *   sigma_grid  host, Gs values > 0          beta_grid  host, p x Gb row-major
 *   prof_sigma  device, Gs doubles           arg_sigma  device, Gs int64 or NULL
 *   prof_beta   device, p*Gb doubles         arg_beta   device, p*Gb int64 or NULL
 *   (arg: record index k*M + m attaining the maximum, the smallest on ties;
 *   -1 and a curve value of -inf when no record is usable)
 *   work     device, pl_curves_workspace_size(p, M, Gs, Gb) bytes.
 * Asynchronous on `stream`.  Errors: -1 rec NULL, -2/-3 beta_hat/xvx_inv NULL
 * with Gb > 0, -4 n < 2, -5 p out of range, -6 K < 1, -7 lambda NULL or not
 * finite, -8 M out of range, -9 a sigma value <= 0 or not finite, -10 Gs out
 * of range or sigma_grid NULL, -11 a beta value not finite, -12 Gb out of
 * range or beta_grid NULL, -13 prof_sigma NULL, -15 prof_beta NULL, -17/-18
 * workspace NULL or too small.
 */
int pl_curves_workspace_size(int64_t p, int64_t M, int64_t Gs, int64_t Gb, size_t* bytes);
int pl_profile_curves(const pl_result* rec, const double* beta_hat, const double* xvx_inv,
                      int64_t n, int64_t p, int64_t K, const double* lambda, int64_t M,
                      const double* sigma_grid, int64_t Gs, const double* beta_grid, int64_t Gb,
                      double* prof_sigma, int64_t* arg_sigma, double* prof_beta,
                      int64_t* arg_beta, void* work, size_t work_bytes, void* stream);

/*
 * Univariate profile likelihood of one correlation parameter or of lambda
 * from the records of one pl_profile_loglik call, and its likelihood interval
 * (Step 4 of the method; Section 3.6, "Profile likelihood for correlation
 * parameters"; the likelihood-based interval of Section 2).  Host arrays,
 * host computation (a few thousand points).
 *   which 0..4: column of omega (range, shape, nugget, ratio, angle).  The
 *           point cloud is (omega_k[which], max over m of l_p(omega_k,
 *           lambda_m)); its upper convex hull, linear between vertices, is
 *           the profile curve.
 *   which 5: lambda.  The curve is the interpolation of (lambda_m, max over
 *           k of l_p).
 *   Only usable records (info 0 or PL_INFO_FALLBACK) count; equal abscissae
 *   keep their largest likelihood.
 *   rec     host, K*M records; omega host K x 5; lambda host M
 *   drop    the interval is {theta : curve(theta) >= max - drop}; drop =
 *           c_{1,alpha}/2 with Pr(chi^2_1 <= c_{1,alpha}) = 1 - alpha (1.92
 *           for 95%), the reading of the paper's interval display
 *   curve_x, curve_y  host, room for max(K, M) values: the curve's vertices by
 *           increasing abscissa; *npts receives their count
 *   interval host, 3 doubles: the maximising abscissa, the lower and upper
 *           ends (linear interpolation at the crossing)
 *   open_ends host or NULL: bit 0 (1) when the curve never falls below the
 *           threshold on the left (the lower end is then the first vertex),
 *           bit 1 (2) likewise on the right
 * Errors: -1 rec NULL, -2 K, -3 M out of range, -4 omega NULL, -5 lambda NULL,
 * -6 which out of range, -7 drop not > 0, -8..-11 output NULL.
 */
int pl_profile_param(const pl_result* rec, int64_t K, int64_t M, const double* omega,
                     const double* lambda, int which, double drop, double* curve_x,
                     double* curve_y, int64_t* npts, double* interval, int32_t* open_ends);

/*
 * Internal parameters of Step 2 (Section 3.2, "Reparameterization"):
 *   omega' = (gamma1, kappa~, nu, gamma2, gamma3),
 *   gamma1 = log phi_X + log phi_Y (exp(gamma1/2) is the combined range),
 *   gamma2 = sqrt(phi_X/phi_Y - 1) cos(2 phi_A),
 *   gamma3 = sqrt(phi_X/phi_Y - 1) sin(2 phi_A),
 *   kappa~ = log kappa (shape_transform 0, for kappa-hat < 4) or
 *            1/sqrt(kappa) (shape_transform 1, kappa-hat >= 4),
 *   nu = sqrt(nu^2).
 * A natural omega with phi_R = phi_X/phi_Y < 1 is first rewritten as the same
 * model with the axes exchanged (phi_X/phi_R, 1/phi_R, phi_A + pi/2), so
 * gamma2, gamma3 are real; the inverse returns phi_R >= 1 and phi_A in
 * (-pi/2, pi/2].  The inverse maps a negative nu to the negative nugget
 * -nu^2 (points drawn from a quadratic approximation can fall there; Step 2's
 * nugget repair then applies).  Host arrays, K x 5 row-major, host code.
 * Errors: -1 omega / internal NULL or a value out of domain (omega: range,
 * ratio <= 0, shape <= 0, nugget < 0, not finite; internal: not finite, or
 * kappa~ <= 0 with shape_transform 1), -2 K < 1, -3 shape_transform not 0
 * or 1, -4 output NULL.
 */
int pl_to_internal(const double* omega, int64_t K, int shape_transform, double* internal);
int pl_from_internal(const double* internal, int64_t K, int shape_transform, double* omega);

/*
 * Maximum-likelihood estimates of (omega, lambda) (Step 1 of the method,
 * Section 3.1: numerical maximisation of equation "profile", or with reml = 1
 * of the restricted profile log-likelihood of Appendix "remlpro").
 *
 * Batched compass search in the coordinates (gamma1, log kappa, log nu^2,
 * gamma2, gamma3) -- the internal parameters above with log nu^2 for the
 * nugget.  Every iteration evaluates the +-h neighbours along each free
 * coordinate of every start in one pl_profile_loglik call (10 points per
 * start), moves each start to its best improving neighbour (doubling that
 * step, capped at 2) or halves its steps; a start stops when its largest step
 * is below tol.  Steps start at 0.5.  lambda is maximised over the M values
 * of every call; after the search, the best start is re-evaluated on a fine
 * lambda set (its value plus min(64, PL_MAX_Q_MIXED - p for PL_MIXED) - 1 evenly spaced
 * values between the neighbouring caller values) and polished by a second
 * search (initial step min(0.5, 16 tol)) on that set.
 *   omega0     host, starts x 5 natural starting points (shape in
 *              [PL_MIN_SHAPE, PL_MAX_SHAPE], nugget > 0)
 *   lambda     host, M Box-Cox values
 *   fixed_mask bit i holds search coordinate i at its start value (bit 1:
 *              kappa, the paper's fits with kappa fixed at 0.5 and 10;
 *              bits 3|4: the anisotropy, isotropic when the starts are)
 *   tol        step at which a start stops, in search coordinates (0 < tol < 0.5)
 *   max_iter   iterations per search (each one call of pl_profile_loglik)
 *   omega_hat  host, 5 doubles; lambda_hat, loglik_hat host, 1 double each;
 *   iterations host or NULL: total iterations of both searches
 *   opts       as pl_profile_loglik (NULL for FP64 defaults)
 *   work       device, pl_mle_workspace_size bytes (same starts, M, opts)
 * The shape is kept in [PL_MIN_SHAPE, PL_MAX_SHAPE] (candidates beyond are
 * evaluated at the bound).  The call synchronises `stream` once per
 * iteration (it reads the records back).
 * Errors: -1..-5 as pl_profile_loglik; -6 omega0 NULL or out of domain;
 * -7 starts < 1 or > PL_MLE_MAX_STARTS; -8 lambda NULL or not finite;
 * -9 M out of range; -10 fixed_mask outside [0, 31]; -11 reml not 0 or 1;
 * -12 tol out of range; -13 max_iter < 1; -14..-16 output NULL; -18 bad
 * option; -19/-20 workspace NULL or too small; PL_E_UNSUPPORTED for PL_MIXED
 * with M + p > PL_MAX_Q_MIXED or when no start has a usable record.
 * pl_mle_workspace_size: -1/-2 as pl_workspace_size, -3 starts out of range,
 * -4 M out of range, -5 bad option, -6 bytes NULL.
 */
#define PL_MLE_MAX_STARTS 256
int pl_mle_workspace_size(int64_t n, int64_t p, int64_t starts, int64_t M,
                          const pl_opts* opts, size_t* bytes);
int pl_mle(const double* locs, const double* y, const double* X, int64_t n, int64_t p,
           const double* omega0, int64_t starts, const double* lambda, int64_t M,
           int32_t fixed_mask, int32_t reml, double tol, int32_t max_iter, double* omega_hat,
           double* lambda_hat, double* loglik_hat, int32_t* iterations, const pl_opts* opts,
           void* work, size_t work_bytes, void* stream);

/*
 * Representative parameter points (Step 2 of the method, Section 3.2,
 * "Hessian matrix" and "Obtaining representative points").
 *
 * pl_hessian: the Hessian H of l_p(omega', lambda_hat) in the internal
 * parameters omega' (see pl_to_internal; d = 5, or d = 4 without kappa~ when
 * fix_shape = 1 -- the fits with the shape held fixed) at omega_hat, by
 * central differences with step delta:
 *   H_ii = [f(w + delta e_i) - 2 f(w) + f(w - delta e_i)] / delta^2,
 *   H_ij = [f(++) - f(+-) - f(-+) + f(--)] / (4 delta^2),
 * on 1 + 2d + 2d(d - 1) points (51 for d = 5, 33 for d = 4), each at lambda
 * in {lambda_hat - delta, lambda_hat, lambda_hat + delta}: one
 * pl_profile_loglik call of PL_HESS_POINTS x 3 records at most.  A point's
 * nugget is nu^2 (so nu - delta < 0 is the nugget (nu - delta)^2).
 *   omega_hat  host, 5 natural values (e.g. from pl_mle); lambda_hat
 *   shape_transform  0: kappa~ = log kappa, 1: 1/sqrt(kappa) (the paper uses
 *              1 when kappa_hat >= 4)
 *   hess       host, d x d row-major; lambda_curv (host or NULL): the second
 *              derivative of l_p in lambda at (omega_hat, lambda_hat) from the
 *              same records; loglik_center (host or NULL): l_p there
 *   work       device, pl_hessian_workspace_size bytes
 * Synchronises `stream` once.  Errors: -1..-5 as pl_profile_loglik; -6
 * omega_hat NULL or out of domain; -7 lambda_hat not finite; -8/-9 flags not
 * 0 or 1; -10 delta not in (0, 1]; -11 hess NULL; -14 bad option; -15/-16
 * workspace NULL or too small; PL_E_UNSUPPORTED when a stencil point has a
 * shape outside [PL_MIN_SHAPE, PL_MAX_SHAPE] or no usable record.
 * pl_hessian_workspace_size: -1/-2 as pl_workspace_size, -3 bad option, -4
 * bytes NULL.
 */
#define PL_HESS_POINTS 51
int pl_hessian_workspace_size(int64_t n, int64_t p, const pl_opts* opts, size_t* bytes);
int pl_hessian(const double* locs, const double* y, const double* X, int64_t n, int64_t p,
               const double* omega_hat, double lambda_hat, int shape_transform, int fix_shape,
               double delta, double* hess, double* lambda_curv, double* loglik_center,
               const pl_opts* opts, void* work, size_t work_bytes, void* stream);

/*
 * pl_config_points: configuration points around omega_hat from a Hessian of
 * pl_hessian (same shape_transform and fix_shape).  -H = E D E^T
 * (eigenvalues ascending, each eigenvector with its largest entry positive);
 * negative eigenvalues are replaced by their absolute values and, when the
 * largest exceeds 100, every eigenvalue below 0.1 by 0.1.  For every level l
 * and sphere point x_t (unit vectors, npts x d):
 *   omega' = omega_hat' + sqrt(q_l) E D^(-1/2) x_t,
 * q_l the chi-square (d degrees of freedom) quantile of upper-tail
 * probability alpha[l], so that (omega' - omega_hat')^T (-H) (omega' -
 * omega_hat') = q_l with the repaired -H; then natural values (phi_R >= 1,
 * shape clamped to [PL_MIN_SHAPE, PL_MAX_SHAPE], 1/sqrt(kappa) <= 0 read as
 * the largest shape, the held shape when fix_shape).  A point with nu < 0 has
 * a negative nugget: the first, third, ... such point (in output order) gets
 * nugget 0, the second, fourth, ... 2 u with u = uniforms[its index].
 *   alpha    host, nlev values in (0, 1); sphere host npts x d
 *   uniforms host, nlev*npts values in [0, 1) (only those of repaired points
 *            are read)
 *   omega_out host, nlev*npts x 5, level-major
 *   eigvals  host, d repaired eigenvalues ascending, or NULL
 *   nugget_repaired host or NULL: the number of repaired nuggets
 * Host code.  Errors: -1 omega_hat NULL or out of domain, -2/-3 flags, -4
 * hess NULL or not finite, -5 alpha NULL or out of (0, 1), -6 nlev out of
 * range, -7 sphere NULL, -8 npts out of range, -9 uniforms NULL, -10
 * omega_out NULL; PL_E_UNSUPPORTED when a repaired eigenvalue is 0.
 *
 * pl_sphere_points: npts well-spread unit vectors in R^d, starting from the
 * directions of `init` (npts x d, nonzero rows; e.g. normal draws): `iters`
 * steps of a repulsion (the gradient of the Riesz 8-energy, tangential part,
 * step 0.3 x the current closest distance, shrinking linearly), keeping the
 * arrangement with the largest closest distance, which *min_dist (or NULL)
 * receives.  The paper maximises the closest distance with an unspecified
 * stochastic optimiser.  Host code.  Errors: -1 d not in [2, 16], -2 npts
 * not in [2, 100000], -3 init NULL or a zero row, -4 iters < 0, -5 out NULL.
 *
 * pl_lambda_grid: m values evenly spaced between the tail and 1 - tail
 * quantiles of the normal approximation N(lambda_hat, 1/|lambda_curv|) of
 * the likelihood in lambda (the paper: 30 values, tail 0.01).  Host code.
 * Errors: -1 lambda_hat, -2 lambda_curv (0 or not finite), -3 tail not in
 * (0, 0.5), -4 m not in [2, PL_MAX_M], -5 out NULL.
 *
 * pl_chisq_quantile: *q with Pr(chi^2_dof > q) = upper.  Host code.
 * Errors: -1 dof not in [1, 1000], -2 upper not in (0, 1), -3 q NULL.
 */
int pl_config_points(const double* omega_hat, int shape_transform, int fix_shape,
                     const double* hess, const double* alpha, int64_t nlev, const double* sphere,
                     int64_t npts, const double* uniforms, double* omega_out, double* eigvals,
                     int64_t* nugget_repaired);
int pl_sphere_points(int d, int64_t npts, const double* init, int iters, double* out,
                     double* min_dist);
int pl_lambda_grid(double lambda_hat, double lambda_curv, double tail, int64_t m, double* out);
int pl_chisq_quantile(int dof, double upper, double* q);

/*
 * Autotuner for the form of pl_profile_loglik on one workload.  Candidates:
 * PL_FP64, and PL_MIXED with flush 4, 2 and 1 (the k-depth, 16/8/4 products,
 * of the FP32 partial-sum tiles of the mixed update).  Each is run on the
 * first S = min(K, sample) omega points (sample 0: 64) -- one untimed call,
 * then two timed with HIP events on `stream` -- and every mixed candidate's
 * records are compared with the FP64 records of the same points.  The time
 * per point depends on how many points share a launch (the mixed form issues
 * more launches per block column), so S should be close to the number of
 * points the caller will evaluate per call.  The fastest candidate whose
 * largest |delta loglik| over the sampled records is <= tol is written to
 * opts->precision and opts->flush (FP64 always qualifies; opts->refine, chunk
 * and flags are used as given).  Mixed candidates are skipped when
 * M + p > PL_MAX_Q_MIXED.
 *   report  host, 8 doubles or NULL: per candidate (FP64, mixed flush 4, 2,
 *           1) the measured milliseconds per omega point, then the max
 *           |delta loglik| against FP64 (0 for FP64 itself, -1 if skipped;
 *           -2 throughout when the choice came from the tuning cache).
 * With a tuning cache set (pl_tune_cache_set), a choice stored for the same
 * device architecture, floor(log2 n), M + p and tol is returned without
 * timing anything; a new choice is stored.
 *   work    device workspace of pl_autotune_workspace_size bytes (same
 *           sample).
 * The call synchronises `stream` (it reads the records back).
 * Errors: as pl_profile_loglik for arguments 1-9; -10 sample < 0; -11 tol not
 * finite or < 0; -12 opts NULL; -14/-15 workspace NULL or too small.
 * pl_autotune_workspace_size: -1..-4 as pl_workspace_size, -5 sample < 0,
 * -6 bytes NULL.
 */
int pl_autotune_workspace_size(int64_t n, int64_t p, int64_t K, int64_t M, int64_t sample,
                               size_t* bytes);
int pl_autotune(const double* locs, const double* y, const double* X, int64_t n, int64_t p,
                const double* omega, int64_t K, const double* lambda, int64_t M, int64_t sample,
                double tol, pl_opts* opts, double* report, void* work, size_t work_bytes,
                void* stream);

/*
 * Many independent datasets of uneven size (each with its own omega points)
 * evaluated by one graph launch (Section 3.3's Step 3 per (dataset, omega)
 * unit; the paper's memory-bounded chunking of parameter sets, Section 3.3,
 * becomes passes over workspace regions that are reused).  Two schedules:
 *   size-bucketed (default; PL_FP64 or PL_MIXED): units grouped by their
 *     number of 128-row tiles run through the step kernels of
 *     pl_profile_loglik in passes of many units, each unit with its own n;
 *     the passes are spread over opts->lanes streams (largest first, to the
 *     least loaded), all captured into one HIP graph;
 *   persistent (PL_OPT_BATCH_PERSISTENT, PL_FP64): one persistent kernel
 *     pulls tile tasks from a queue, units recycling a pool of matrix slabs.
 *
 * One dataset: locs (device, n x 2 row-major), y (device, n, > 0), X (device,
 * n x p column-major), omega (host, K x 5), all shared lambda values.
 */
typedef struct pl_dataset {
  const double* locs;
  const double* y;
  const double* X;
  int64_t n;
  const double* omega;
  int64_t K;
} pl_dataset;

/* Opaque plan: the task list of every unit, its slab assignment and, after
 * the first pl_batch_run, a captured HIP graph of the whole launch sequence. */
typedef struct pl_batch pl_batch;

/*
 * Build a plan on the host (no GPU call).  opts (NULL for defaults):
 * precision, refine, flush and PL_OPT_NO_FALLBACK as for pl_profile_loglik;
 * PL_OPT_BATCH_PERSISTENT selects the persistent schedule; opts->chunk, when
 * > 0, caps the units per pass (size-bucketed; default: as many as fit
 * 4 GiB) or the number of matrix slabs (persistent; default min(units,
 * 2048)); opts->lanes, opts->wait_us as documented in pl_opts.  The plan
 * keeps the dataset pointers, which must stay valid.
 * Errors: -1 datasets NULL or a dataset invalid (n < 2, n <= p, pointers
 * NULL, K < 1, omega out of domain), -2 D out of range, -3 p out of range,
 * -4 lambda NULL or not finite, -5 M out of range, -6 bad option (including
 * PL_MIXED with the persistent schedule), -7 plan NULL; PL_E_UNSUPPORTED if
 * the task list cannot be built or PL_MIXED has M + p > PL_MAX_Q_MIXED.
 */
int pl_batch_create(const pl_dataset* datasets, int64_t D, int64_t p, const double* lambda,
                    int64_t M, const pl_opts* opts, pl_batch** plan);
int pl_batch_workspace_size(const pl_batch* plan, size_t* bytes);
/* Units (sum of K over datasets), tasks and slabs of a plan (NULL to skip):
 * persistent: tile tasks and matrix slabs; size-bucketed: device passes and
 * streams. */
int pl_batch_stats(const pl_batch* plan, int64_t* units, int64_t* tasks, int64_t* slabs);
/*
 * Evaluate every record: out (device) receives sum_d K_d * M records, dataset
 * by dataset, omega-major then lambda; beta_hat (device, or NULL) p doubles per
 * record.  The first call (and any call with a different work, out or
 * beta_hat) uploads the plan into the workspace and captures the launch
 * sequence into a HIP graph; every call then launches that graph on `stream`.
 * PL_MIXED without PL_OPT_NO_FALLBACK then synchronises `stream` once and
 * redoes FP32 breakdowns with the FP64 form (info |= PL_INFO_FALLBACK).
 * Errors: -1 plan NULL, -2 out NULL, -4 work NULL, -5 work too small, PL_E_HIP.
 */
int pl_batch_run(pl_batch* plan, pl_result* out, double* beta_hat, void* work, size_t work_bytes,
                 void* stream);
/* After the stream has been synchronised: *err = 1 if a task wait outlived
 * its wall-time limit (opts->wait_us of pl_batch_create); every later wait
 * then returned at once and every later task skipped its work, so the launch
 * ended, but its results are not valid.  Else 0.  Synchronous. */
int pl_batch_error(const pl_batch* plan, void* work, int32_t* err);
void pl_batch_destroy(pl_batch* plan);

/*
 * Optional timing of the library's own kernels with HIP events recorded on
 * the caller's stream around every launch (benchmarks and tracing; off by
 * default, no cost when off).  Kernel classes:
 *   PL_KC_TABLES  per-omega Chebyshev tables of the Matern correlation
 *   PL_KC_MATERN  covariance tiles
 *   PL_KC_GEMM    left-looking block-column update (the dominant kernel)
 *   PL_KC_POTRF   diagonal-tile factorisation and inverse
 *   PL_KC_TRSM    panel solve
 *   PL_KC_OTHER   Box-Cox right-hand sides, bordering, p x p stage, fills
 * pl_profiling_enable(1) clears the counters and starts recording;
 * pl_profiling_enable(0) stops.  pl_profiling_read waits for the recorded
 * events, then writes per class (arrays of length nclass <= PL_KC_COUNT):
 * total milliseconds, the algorithmic floating-point operations of those
 * launches (for PL_KC_GEMM: the lower-triangle update flops the method
 * needs, 2 r c k per off-diagonal tile and r (r+1) k per diagonal tile),
 * and the launch count.  Errors: -1 bad nclass, -2..-4 NULL array;
 * PL_E_HIP if an event failed.
 */
#define PL_KC_TABLES 0
#define PL_KC_MATERN 1
#define PL_KC_GEMM   2
#define PL_KC_POTRF  3
#define PL_KC_TRSM   4
#define PL_KC_OTHER  5
#define PL_KC_COUNT  6
int pl_profiling_enable(int on);
int pl_profiling_read(double* ms, double* alg_flops, int64_t* launches, int nclass);

/*
 * Autotuner of the uneven batch (Section 4's hand-set launch sizes --
 * parameter sets per iteration, global and local work sizes -- measured
 * instead).  Candidates of pl_batch_create on the caller's datasets: the
 * size-bucketed schedule in FP64 with 2, 4 and 8 streams and the default
 * pass size, with 4 streams and passes of at most 256 units; the persistent
 * kernel (FP64); the mixed form, 4 streams, flush 4 and 2 (skipped when
 * M + p > PL_MAX_Q_MIXED).  Each candidate's plan runs once (graph capture), then twice
 * timed with HIP events on `stream`; its records are compared with the first
 * (FP64) candidate's.  The fastest whose largest |delta loglik| is <= tol is
 * written to opts (precision, flush, lanes, chunk and the
 * PL_OPT_BATCH_PERSISTENT bit; the other fields are used as given), ready for
 * pl_batch_create.  With a tuning cache set, a choice stored for the same
 * architecture, floor(log2 of the largest n), floor(log2 of the number of
 * units), M + p and tol is returned without timing; a new one is stored.
 *   datasets, D, p, lambda, M   as pl_batch_create
 *   report  host, 14 doubles or NULL: per candidate (in the order above)
 *           milliseconds per replay (-1 if skipped), then the max |delta
 *           loglik| against FP64; -2 throughout for a cached choice
 *   work    device, pl_batch_autotune_workspace_size bytes
 * The call synchronises `stream`.  Errors: those of pl_batch_create for the
 * datasets and options, -6 tol not finite or < 0, -7 opts NULL, -9/-10
 * workspace NULL or too small; PL_E_UNSUPPORTED if no candidate ran.
 */
int pl_batch_autotune_workspace_size(const pl_dataset* datasets, int64_t D, int64_t p,
                                     const double* lambda, int64_t M, size_t* bytes);
int pl_batch_autotune(const pl_dataset* datasets, int64_t D, int64_t p, const double* lambda,
                      int64_t M, double tol, pl_opts* opts, double* report, void* work,
                      size_t work_bytes, void* stream);

/*
 * Tuning cache: the choices of pl_autotune (kind 0) and pl_batch_autotune
 * (kind 1), keyed by (device architecture, kind, floor(log2 n) -- of the
 * largest n for a batch --, floor(log2 units) for a batch, M + p, tol printed
 * with 6 significant digits).  Process-wide and thread-safe; host code.
 * pl_tune_cache_set(path): clears the table and loads `path`, a text file of
 *   one line per choice (created on the first store; later lines of a key
 *   win), to which every new choice is then appended; "" keeps the table in
 *   memory only.  Until the first call, and after a call with NULL, the
 *   autotuners neither consult nor fill the table (every call measures).
 *   -1 if the file cannot be opened for writing.
 * pl_tune_store / pl_tune_lookup: store or look up a choice directly (arch
 *   NULL or "": the current device's).  Lookup returns PL_TUNE_MISS (no
 *   change to opts) when nothing is stored; on a hit it writes precision,
 *   flush, chunk, lanes and the PL_OPT_BATCH_PERSISTENT bit.  Errors: -2 kind,
 *   -3 n < 2, -4 units < 1 for kind 1, -5 q out of range, -6 tol, -7 opts
 *   NULL, -1 file write failure (store), PL_E_HIP when the architecture is
 *   needed and no device is usable.
 * pl_tune_cache_stats: entries, hits and misses (NULL to skip) since the last
 *   pl_tune_cache_set.
 */
int pl_tune_cache_set(const char* path);
int pl_tune_store(const char* arch, int kind, int64_t n, int64_t units, int64_t q, double tol,
                  const pl_opts* opts, double ms);
int pl_tune_lookup(const char* arch, int kind, int64_t n, int64_t units, int64_t q, double tol,
                   pl_opts* opts);
int pl_tune_cache_stats(int64_t* entries, int64_t* hits, int64_t* misses);

#ifdef __cplusplus
}
#endif

#endif /* PLPROF_H */
