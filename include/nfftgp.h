/*
 * nfftgp.h -- C ABI of the MI355X (gfx950) additive-kernel fast summation.
 *
 * The library applies the regularised additive kernel matrix of
 * "Preconditioned Additive Gaussian Processes with Fourier Acceleration"
 * (Wagner, Xu, Nestler, Xi, Stoll) and its hyper-parameter derivatives to
 * blocks of vectors, and runs CG on it:
 *
 *   Khat = sigma_f^2 (K_1 + ... + K_P) + sigma_eps^2 I          (Sec. 2.1, Sec. 1)
 *   (K_s)_ij = kappa_s(x_i^{W_s} - x_j^{W_s})                  (eq. def_additive_kernel)
 *   kappa_s = exp(-r^2/(2 ell_s^2)) or exp(-r/ell_s)          (Gaussian / Matern-1/2)
 *
 * Each K_s is replaced by the matrix of the N_s^d-term trigonometric
 * interpolant of its periodically continued kernel (Sec. 3.1, eq. nfftkappa,
 * eq. discrete_fourier_coefficients1) and applied by the NFFT-based fast
 * summation (eq. Fourier_sum; Appendix A): window spreading onto a (2N)^d
 * grid, FFT, a diagonal multiply by the kernel's Fourier coefficients divided
 * by the squared window coefficients, inverse FFT, window interpolation.
 * Derivative products reuse the same pipeline with the coefficients of the
 * sampled ell-derivative (Sec. 3.2, eq. exact_derivative).
 *
 * Conventions for every call:
 *  - All matrices are row-major.  Device pointers point to memory allocated
 *    on the device the plan was created on; host pointers are ordinary host
 *    memory.  The caller owns every buffer it passes; the plan owns its own
 *    workspaces and frees them in nfftgp_plan_destroy.
 *  - Floating point buffers passed to a plan have the plan's precision
 *    (float for NFFTGP_F32, double for NFFTGP_F64).  CG scalars, dot
 *    products and the Lanczos history are always double.
 *  - Work is enqueued on the stream given at plan creation (NULL = the null
 *    stream).  nfftgp_apply allocates nothing and does not synchronise the
 *    host, so it can be captured into a HIP graph.
 *  - Argument errors are detected before any work is enqueued and leave the
 *    plan unchanged.  Every call returns NFFTGP_OK or a negative status;
 *    nfftgp_last_error() then gives a message (thread-local, valid until the
 *    next call on the same thread).
 *  - One plan must not be used from two threads at once.
 */
#ifndef NFFTGP_H
#define NFFTGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NFFTGP_OK = 0,
    NFFTGP_E_ARG = -1,    /* invalid argument (null pointer, size, overlap, ...)   */
    NFFTGP_E_DIM = -2,    /* unsupported window dimension, bandwidth or cutoff     */
    NFFTGP_E_BOX = -3,    /* SCALE_NONE but a point lies outside [-1/4, 1/4)^d     */
    NFFTGP_E_HIP = -4,    /* a HIP runtime call failed                             */
    NFFTGP_E_NOMEM = -5,  /* device allocation failed                              */
    NFFTGP_E_NOTPD = -6,  /* CG met p^T Khat p <= 0: the operator is not definite  */
    NFFTGP_E_NOCONV = -7, /* CG stopped at maxit before reaching tol               */
    NFFTGP_E_STATE = -8   /* call order violated (e.g. apply before set_hyper)     */
} nfftgp_status;

/* Sub-kernels (unit variance, distance r, length-scale ell; eq. kernel_definition):
 * GAUSS     exp(-r^2 / (2 ell^2))
 * MATERN12  exp(-r / ell)
 * MATERN32  (1 + sqrt(3) r / ell) exp(-sqrt(3) r / ell), the order-3/2 Matern
 *           kernel of Sec. 4 (generalization to other orders); same pipeline,
 *           only the sampled kernel and its ell-derivative differ.
 * The kernels the paper names beside them for the fast summation (its software
 * section), with the shape parameter c in the place of ell (so the "ell"
 * derivative outputs are d/dc) and no normalisation of kappa(0):
 * MQ        multiquadric (r^2 + c^2)^(1/2)            (not positive definite)
 * IMQ       inverse multiquadric (r^2 + c^2)^(-1/2)
 * SINC      sin(c r) / r, value c at r = 0 */
typedef enum {
    NFFTGP_GAUSS = 0,
    NFFTGP_MATERN12 = 1,
    NFFTGP_MATERN32 = 2,
    NFFTGP_MQ = 3,
    NFFTGP_IMQ = 4,
    NFFTGP_SINC = 5
} nfftgp_kernel;
/* Precision values: entry points take them as int32_t (any other value is
 * rejected with NFFTGP_E_ARG), so a caller's out-of-range value never becomes
 * an invalid enumeration value inside the library. */
typedef enum { NFFTGP_F32 = 0, NFFTGP_F64 = 1 } nfftgp_prec;

/* Scaling of each window into the box [-1/4, 1/4)^d required by Sec. 3.1.
 * AUTO: centre c0 = per-feature midrange, one isotropic factor
 *       c = (1/4)(1 - 2^-20) / max_j ||x_j - c0||_inf, so x~ = c (x - c0);
 *       a window whose coordinates already lie in [-1/4, 1/4) is kept as is
 *       (c = 1, c0 = 0).
 * NONE: c = 1, c0 = 0; every coordinate must lie in [-1/4, 1/4) (else E_BOX).
 * Length-scales are always given in the caller's units; the box kernel is
 * kappa(r~ / c; ell). */
enum { NFFTGP_SCALE_AUTO = 0, NFFTGP_SCALE_NONE = 1 };

/* Limits of this build. */
#define NFFTGP_MAX_WINDOWS 64
#define NFFTGP_MAX_WINDOW_DIM 3
/* CG iterations whose Lanczos coefficients nfftgp_cg can record (the history
 * buffer, NFFTGP_MAX_CG_HISTORY x max_nrhs x 2 doubles, is allocated with the
 * plan, so that nfftgp_cg allocates nothing). */
#define NFFTGP_MAX_CG_HISTORY 4096

typedef struct nfftgp_plan_s *nfftgp_plan;

/* Create a plan for fixed points and windows (Sec. 2.1: the points stay fixed
 * while the hyper-parameters change).
 *   X_dev    device, n x p row-major, leading dimension ldx >= p, precision prec
 *            (NFFTGP_F32 or NFFTGP_F64; E_ARG otherwise).
 *            Read during this call only (the plan keeps scaled, sorted copies).
 *   n        number of points, 0 <= n < 2^31.
 *   P        number of windows, 1..NFFTGP_MAX_WINDOWS.
 *   win_ptr  host, P+1 offsets into win_idx; window s has d_s = win_ptr[s+1]-win_ptr[s]
 *            features, 1 <= d_s <= 3.
 *   win_idx  host, 0-based feature indices; windows must be disjoint (eq. additive_kernel).
 *   kernel   host, P entries of nfftgp_kernel.
 *   N        host, P bandwidths: powers of two, 8..64 for d_s = 3, 8..128 otherwise.
 *            The index set is I_N = {-N/2, ..., N/2-1}^d (eq. nfftkappa) and the
 *            oversampled FFT grid has (2N)^d points.
 *   m        window cutoff (Kaiser-Bessel support m/(2N) per dimension, Appendix A),
 *            m in {2, 4, 6, 8} and m < N/2 (E_DIM otherwise).
 *   max_nrhs largest nrhs that nfftgp_apply / nfftgp_cg will be given (1..64);
 *            workspaces are sized for it here.
 *   stream   hipStream_t to enqueue on (NULL = null stream).
 * On success *out receives the plan.  Synchronises the stream once. */
nfftgp_status nfftgp_plan_create(nfftgp_plan *out,
                                 const void *X_dev, int64_t n, int32_t p, int64_t ldx,
                                 int32_t P, const int32_t *win_ptr, const int32_t *win_idx,
                                 const int32_t *kernel, const int32_t *N, int32_t m,
                                 int32_t prec, int32_t scale_mode, int32_t max_nrhs,
                                 void *stream);

/* As nfftgp_plan_create, with the scaling of every window into
 * [-1/4, 1/4)^d given by the caller instead of computed from X (Sec. 3.1):
 * x~ = c_s (x - c0_s).  Lets several plans on different point sets (e.g.
 * training points, and training plus test points for a cross product) share
 * one kernel in box units.
 *   c0  host, sum_s d_s doubles: centre of window s at c0[win_ptr[s] ...].
 *   c   host, P doubles: factor of window s, finite and > 0.
 * Every scaled coordinate must lie in [-1/4, 1/4) (E_BOX otherwise).
 * Length-scales stay in the caller's units, as for nfftgp_plan_create. */
nfftgp_status nfftgp_plan_create_scaled(nfftgp_plan *out,
                                        const void *X_dev, int64_t n, int32_t p, int64_t ldx,
                                        int32_t P, const int32_t *win_ptr, const int32_t *win_idx,
                                        const int32_t *kernel, const int32_t *N, int32_t m,
                                        int32_t prec, const double *c0, const double *c,
                                        int32_t max_nrhs, void *stream);

/* Set the hyper-parameters theta = (sigma_f, ell, sigma_eps) (Sec. 1).
 *   ell   host, P length-scales in caller units (one per window; the paper's
 *         shared ell is the case of P equal values), each > 0.
 *   sigma_f, sigma_eps >= 0.
 * Computes, on the device in FP64, the coefficients b_k and b^der_k of every
 * window (eq. discrete_fourier_coefficients1, eq. exact_derivative) and the
 * diagonal applied between the two FFTs (for window groups whose kernels are
 * all Gaussian the samples factor over dimensions, and the coefficients are
 * computed as products of 1-D transforms: the same values up to rounding;
 * for such groups this call only records theta, and the coefficients are
 * computed by the next nfftgp_apply in extra work-groups of its fold launch,
 * or by their own launch when nfftgp_cg or nfftgp_get_window_info comes
 * first).  Asynchronous (no host wait);
 * min_k b_k per window is reduced from per-block minima when
 * nfftgp_get_window_info asks for it. */
nfftgp_status nfftgp_set_hyper(nfftgp_plan plan, double sigma_f, const double *ell,
                               double sigma_eps);

/* Apply the operator to nrhs vectors (eq. Fourier_sum, summed over windows as
 * in Sec. 3.1, last paragraph).
 *   V_dev        device, n x nrhs, leading dimension ldv >= nrhs.
 *   KV_dev       device, n x nrhs (leading dimension nrhs), required:
 *                sigma_f^2 sum_s K_s V + sigma_eps^2 V.
 *   dKV_dell_dev device or NULL: P blocks of n x nrhs, block s =
 *                dKhat/d ell_s V = sigma_f^2 K_s^der V (eq. def_der_additive_kernels).
 *   dKV_dsf_dev  device or NULL: dKhat/d sigma_f V = 2 sigma_f sum_s K_s V.
 *   dKV_dse_dev  device or NULL: dKhat/d sigma_eps V = 2 sigma_eps V.
 * Output buffers must not overlap V.  1 <= nrhs <= max_nrhs.  Asynchronous. */
nfftgp_status nfftgp_apply(nfftgp_plan plan, const void *V_dev, int64_t ldv, int32_t nrhs,
                           void *KV_dev, void *dKV_dell_dev, void *dKV_dsf_dev,
                           void *dKV_dse_dev);

/* Solve Khat X = B column by column with CG (Sec. 1; Sec. 2.3) from a zero
 * start; column c stops when ||r_c||_2 <= tol ||b_c||_2 or after maxit steps.
 * Dot products, step lengths and residual norms are FP64 on the device.
 *   B_dev, X_dev   device, n x nrhs (leading dimension nrhs), prec of the plan.
 *   iters_host     host or NULL: nrhs iteration counts.
 *   alpha_beta_host host or NULL: maxit x nrhs x 2 doubles; entry [j][c] holds
 *                  (alpha_j, beta_j) of column c for j < iters[c] -- the Lanczos
 *                  coefficients used by stochastic Lanczos quadrature.  Needs
 *                  maxit <= NFFTGP_MAX_CG_HISTORY (E_ARG otherwise).
 *   resid_host     host or NULL: nrhs final relative residuals ||r||/||b||.
 * Returns NFFTGP_E_NOTPD if some column met p^T Khat p <= 0 (that column is
 * frozen at its last iterate), NFFTGP_E_NOCONV if a column did not reach tol,
 * NFFTGP_OK otherwise.  Synchronises the stream every check_every iterations
 * (check_every <= 0 means 8).  Allocates no device memory: its vectors,
 * scalars and history are plan workspaces.  Iterations are enqueued eagerly;
 * with the environment variable NFFTGP_CG_GRAPH=1 the check_every iterations
 * between two checks (at most 16) are captured once into a HIP graph and
 * replayed (bit-identical results; the graph is captured again when nrhs,
 * X_dev, tol, sigma_f, sigma_eps or check_every change). */
nfftgp_status nfftgp_cg(nfftgp_plan plan, const void *B_dev, int32_t nrhs, void *X_dev,
                        double tol, int32_t maxit, int32_t check_every,
                        int32_t *iters_host, double *alpha_beta_host, double *resid_host);

/* Column dot products out[c] = sum_i A[i][c] * B[i][c] accumulated in FP64
 * (Sec. 1 eq. div needs alpha^T dKhat alpha and z_i^T (...) terms).
 *   A_dev, B_dev device, n x ncol with leading dimensions lda, ldb, precision prec.
 *   out_host     host, ncol doubles.  Synchronises the stream. */
nfftgp_status nfftgp_col_dots(nfftgp_plan plan, const void *A_dev, int64_t lda,
                              const void *B_dev, int64_t ldb, int64_t n, int32_t ncol,
                              double *out_host);

/* Allocation-free variant of nfftgp_col_dots, for callers that cannot
 * allocate (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc): needs no plan, allocates nothing, does not synchronise.
 * The partial sums live in a static device array of the library (61 440
 * bytes per device, held until the process ends); it is looked up once per
 * device on the first call there.  Calls that overlap on one device (other
 * streams or threads) race on that array.
 *   prec         precision of A and B (NFFTGP_F32 or NFFTGP_F64).
 *   A_dev, B_dev device, n x ncol with leading dimensions lda, ldb.
 *   ncol         1..64 (E_ARG beyond: the array holds 64 columns).
 *   out_dev      device, ncol doubles: out[c] = sum_i A[i][c] B[i][c] in FP64.
 *   stream       hipStream_t to enqueue on (NULL = null stream). */
nfftgp_status nfftgp_col_dots_noalloc(int32_t prec, const void *A_dev, int64_t lda,
                                      const void *B_dev, int64_t ldb, int64_t n, int32_t ncol,
                                      double *out_dev, void *stream);

/* Stochastic Lanczos quadrature (Sec. 1): for each column c,
 *   out[c] = znorm2[c] * e_1^T log(T_c) e_1,
 * where T_c is the Lanczos tridiagonal matrix built from the CG coefficients
 * (alpha_j, beta_j), j < iters[c], in the layout nfftgp_cg writes.  Host-only
 * FP64 computation (symmetric tridiagonal QL eigen-solver).  Returns
 * NFFTGP_E_NOTPD if some T_c has a non-positive eigenvalue. */
nfftgp_status nfftgp_slq_logquad(const double *alpha_beta_host, const int32_t *iters,
                                 int32_t ncol, int32_t maxit, const double *znorm2,
                                 double *out_host);

/* Per-window information: centre c0 (d_s doubles), factor c, dimension, bandwidth,
 * and the smallest coefficients min_k b_k and min_k b^der_k from the last
 * set_hyper (min_b < 0 means K_{s,RF} can be indefinite).  Any output may be NULL.
 * When a set_hyper result has not been read yet, enqueues the reduction of
 * the smallest coefficients and synchronises the stream. */
nfftgp_status nfftgp_get_window_info(nfftgp_plan plan, int32_t s, double *c0, double *c,
                                     int32_t *d, int32_t *N, double *min_b, double *min_bder);

/* Autotuning (setup time).  Times nrhs-column applies (with the derivative
 * outputs when with_derivs != 0) for each window group under candidate
 * settings -- points per spreading subproblem (64 ... 4096), vectors per
 * spreading work-group (1, 2, 4), the spreading form (four-point or
 * run-ordered), waves per 3-D spreading tile (4 or 2) and the interpolation
 * variant (per-point tile reads with 1 or 2 points per thread and, for 3-D
 * windows, the whole padded tile or a window of its rows; or register-held
 * runs) -- by coordinate search, best of two trials of `reps` applies each
 * (more when an apply is short: about 5 ms per trial), and keeps the fastest
 * settings in the plan.  Requires nfftgp_set_hyper.  Allocates and
 * frees its own input and output buffers (and may grow the plan's tile
 * workspace); synchronises the stream; drops a captured CG iteration.  A
 * one-line summary per group is written to `report` (NUL-terminated,
 * truncated to report_len; may be NULL). */
nfftgp_status nfftgp_autotune(nfftgp_plan plan, int32_t nrhs, int32_t with_derivs, int32_t reps,
                              char *report, int64_t report_len);

/* Kernel timing with HIP events (a profiling aid).  `categories` is a bit
 * mask: bit c set times the launches of category c below (NFFTGP_PROF_ALL:
 * every launch, 0: off).  Every timed kernel is bracketed by two events on
 * the plan's stream; each event pair adds a few microseconds to the stream,
 * so time only the categories of interest when the total matters.
 * nfftgp_profile_read synchronises the stream and returns, per category, the
 * summed duration in milliseconds and the number of launches since the last
 * nfftgp_profile call.  Timing allocates events, so do not enable it while
 * capturing a graph; CG runs its iterations eagerly while any category is
 * timed. */
enum {
    NFFTGP_PROF_FILL = 0,     /* reserved (no kernel in this version)         */
    NFFTGP_PROF_SPREAD = 1,   /* window spreading onto the tiles              */
    NFFTGP_PROF_FOLD = 2,     /* sum of overlapping tiles into the grid       */
    NFFTGP_PROF_FFT_FWD = 3,  /* forward FFT passes of axes d-1..1            */
    NFFTGP_PROF_DIAG = 4,     /* axis 0: forward FFT, diagonal, inverse FFT   */
    NFFTGP_PROF_FFT_INV = 5,  /* inverse FFT passes of axes 1..d-1            */
    NFFTGP_PROF_INTERP = 6,   /* window interpolation into per-window outputs */
    NFFTGP_PROF_ASSEMBLE = 7, /* window sum, sigma scaling, derivative blocks */
    NFFTGP_PROF_COEF = 8,     /* per-theta coefficient kernels                */
    NFFTGP_PROF_CG = 9,       /* CG dot products and vector updates           */
    NFFTGP_PROF_GATHER = 10,  /* reserved (no kernel in this version)         */
    NFFTGP_PROF_PRECOND = 11, /* preconditioner factors and applications      */
    NFFTGP_PROF_COUNT = 12,
    NFFTGP_PROF_ALL = (1 << 12) - 1
};
nfftgp_status nfftgp_profile(nfftgp_plan plan, int32_t categories);
nfftgp_status nfftgp_profile_read(nfftgp_plan plan, double *ms_host, int32_t *count_host);

/* ---------------------------------------------------------------- AAFN
 * Additive adaptive factorised Nystrom preconditioner (Sec. 2.3) and
 * preconditioned CG (Sec. 1; Sec. 2.3; eq. log_det_decomp,
 * eq. GP_approx_objective, eq. div).
 *
 * Landmarks: in every window, farthest point sampling of per_window points
 * (the first is the point farthest from the window centre c0, every further
 * one maximises the distance to those already chosen; ties to the smallest
 * index); the windows' lists are merged rank by rank, duplicates skipped, up
 * to max_rank points, held in ascending index order.  The other points,
 * ordered by their grid cell of window 0 (tiles, then cells), are cut into
 * blocks of at most `block` points.  With the landmarks first,
 *   M = [[K11, K12], [K21, K21 K11^-1 K12 + blockdiag(S_BB)]] = F F^T,
 *   F = [[L11, 0], [K21 L11^-T, blockdiag(L_B)]],
 * K11 = L11 L11^T (Cholesky of the landmark block), S_BB = L_B L_B^T the
 * diagonal blocks of the Schur complement K22 - K21 K11^-1 K12 (the
 * approximate inverse of the Schur complement keeps them).  Kernel entries
 * are those of the exact kernel (Sec. 1, eq. kernel_definition) at the
 * plan's theta, in FP64; M approximates Khat.
 *
 * Attach once per plan; every nfftgp_set_hyper then enqueues the factors
 * for the new theta (asynchronously).  nfftgp_pcg, nfftgp_precond_apply and
 * nfftgp_precond_dquad allocate nothing. */

/* Attach the preconditioner.  X_dev: the same n x p points (device, plan
 * precision, leading dimension ldx) the plan was created from.  Limits:
 * plan windows <= 16, 1 <= max_rank <= 512, 1 <= block <= 128, per_window
 * >= 1.  Allocates the preconditioner's workspaces (FP64: about
 * (4 k + 2 block) doubles per point, k the number of landmarks).  E_STATE if
 * a preconditioner is already attached.  Synchronises the stream. */
nfftgp_status nfftgp_precond_attach(nfftgp_plan plan, const void *X_dev, int64_t ldx, int32_t per_window,
                                    int32_t max_rank, int32_t block);

/* k (landmarks), number of Schur-complement blocks, log det M and
 * tr(M^-1 dM/dtheta_j) for theta = (sigma_f, ell_1, ..., ell_P, sigma_eps)
 * (the second term of eq. div); any output may be NULL.  Synchronises the
 * stream when log det M or the traces are asked for; E_NOTPD if a Cholesky
 * pivot of the landmark block or of a Schur-complement block was not
 * positive. */
nfftgp_status nfftgp_precond_info(nfftgp_plan plan, int32_t *k, int32_t *nblocks, double *logdet,
                                  double *dlogdet);

/* The k landmark indices (host, ascending).  Synchronises the stream. */
nfftgp_status nfftgp_precond_landmarks(nfftgp_plan plan, int32_t *idx_host);

/* out = op(V) for nrhs vectors (device, n x nrhs, leading dimension nrhs,
 * plan precision; out must not overlap V):
 *   NFFTGP_PC_MINV   M^-1 V
 *   NFFTGP_PC_FINVT  F^-T V          (= M^-1 F V)
 *   NFFTGP_PC_F      F V             (probes with covariance M from V)
 * Asynchronous. */
enum { NFFTGP_PC_MINV = 0, NFFTGP_PC_FINVT = 1, NFFTGP_PC_F = 2 };
nfftgp_status nfftgp_precond_apply(nfftgp_plan plan, int32_t op, const void *V_dev, int32_t nrhs,
                                   void *out_dev);

/* out_host[j * nrhs + c] = w_c^T (dM/dtheta_j) w_c for the nrhs columns of W
 * (device, n x nrhs, leading dimension nrhs), theta as for
 * nfftgp_precond_info: the control-variate term of the trace estimator of
 * eq. div.  Synchronises the stream. */
nfftgp_status nfftgp_precond_dquad(nfftgp_plan plan, const void *W_dev, int32_t nrhs, double *out_host);

/* Preconditioned CG with the attached M, otherwise as nfftgp_cg (same
 * arguments, stopping rule ||r_c|| <= tol ||b_c||, FP64 scalars, Lanczos
 * coefficients (alpha_j, beta_j) of the preconditioned iteration in
 * alpha_beta_host).  E_STATE without a preconditioner.  Runs its iterations
 * eagerly. */
nfftgp_status nfftgp_pcg(nfftgp_plan plan, const void *B_dev, int32_t nrhs, void *X_dev, double tol,
                         int32_t maxit, int32_t check_every, int32_t *iters_host, double *alpha_beta_host,
                         double *resid_host);

/* Device bytes the plan holds. */
nfftgp_status nfftgp_get_workspace_bytes(nfftgp_plan plan, size_t *bytes);

/* The kernel forms an apply of nrhs vectors (1..max_nrhs) takes (a reporting
 * aid for the spreading and interpolation steps of Sec. 3.1 / Appendix A):
 * one line per window group, "group d=<d> N=<N> windows=<k>: spread=<form>
 * ...; interp=<variant> ...", where the spreading form is "mfma" (matrix
 * cores), "four-point" or "run" and the interpolation variant "mfma", "tile",
 * "tile2", "tilepair", "tileslot" or "run".  Written NUL-terminated into
 * `out` (host), truncated to len bytes.  Host work only. */
nfftgp_status nfftgp_describe(nfftgp_plan plan, int32_t nrhs, char *out, int64_t len);

/* Free the plan and everything it owns (NULL is allowed).  Synchronises. */
void nfftgp_plan_destroy(nfftgp_plan plan);

/* Message of the last failed call on this thread ("" if none). */
const char *nfftgp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NFFTGP_H */
