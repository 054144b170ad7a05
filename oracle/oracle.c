/*
 * oracle.c -- plain FP64 CPU reference for the additive-kernel fast summation
 * of "Preconditioned Additive Gaussian Processes with Fourier Acceleration"
 * (Wagner, Xu, Nestler, Xi, Stoll).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * execute this file: it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the GPU library against a slow,
 * obviously correct evaluation.  It shares no code, header, table or helper
 * with the GPU library.
 *
 * Two results are computed here, both straight from their definitions:
 *
 *   O1  the exact additive kernel product
 *         y_i = sigma_f^2 sum_s sum_j kappa_s(x_i^{W_s} - x_j^{W_s}) v_j
 *               + sigma_eps^2 v_i
 *       (Sec. 2.1, eq. additive_kernel / def_additive_kernel, regularised
 *       matrix K + sigma_eps^2 I of Sec. 1) and the length-scale derivative
 *       blocks sigma_f^2 sum_j kappa_s^der(...) v_j (eq. def_der_additive_kernels).
 *
 *   O2  the product with each sub-kernel replaced by its N^d-term
 *       trigonometric interpolant (Sec. 3.1, eq. nfftkappa, eq. Fourier_sum):
 *         h_i = Re sum_{k in I_N} b_k ( sum_j v_j e^{-2 pi i k.x~_j} ) e^{2 pi i k.x~_i}
 *       evaluated either pairwise (tiny n) or through the inner sums
 *       a_k = sum_j v_j e^{-2 pi i k.x~_j} (direct non-equispaced DFT).
 *       The coefficients b_k are an input (computed by coefficients() in
 *       oracle/__init__.py from eq. discrete_fourier_coefficients1).
 *
 * Layouts: X is row-major n x p (leading dimension ldx), V is row-major
 * n x nrhs, windows are given in CSR form (win_ptr[P+1], win_idx[...],
 * 0-based feature indices).  Coefficient arrays for window s hold N_s^d_s
 * real values, index (k_1+N/2, ..., k_d+N/2) row-major (last fastest).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846264338327950288

enum { ORC_GAUSS = 0, ORC_MATERN12 = 1, ORC_MATERN32 = 2, ORC_MQ = 3, ORC_IMQ = 4, ORC_SINC = 5 };

/* Kernel value and its derivative with respect to ell, for distance r >= 0.
 * Gaussian:   exp(-r^2/(2 ell^2)),   derivative (r^2/ell^3) exp(...)
 * Matern-1/2: exp(-r/ell),           derivative (r/ell^2)   exp(...)
 * Matern-3/2: (1 + a) exp(-a) with a = sqrt(3) r / ell,
 *             derivative (3 r^2/ell^3) exp(-a)
 * (eq. kernel_definition with unit variance, eq. def_der_additive_kernels;
 * the order-3/2 Matern kernel of Sec. 4, generalization to other orders).
 * The kernels the paper names for the fast summation in its software section,
 * with the shape parameter c in the place of ell (derivative d/dc):
 * multiquadric sqrt(r^2 + c^2),     derivative c / sqrt(r^2 + c^2)
 * inverse MQ   1 / sqrt(r^2 + c^2), derivative -c / (r^2 + c^2)^(3/2)
 * sinc         sin(c r) / r (c at r = 0), derivative cos(c r) */
void orc_kernel(int type, double r, double ell, double *val, double *dval)
{
    if (type == ORC_MQ || type == ORC_IMQ) {
        double q = sqrt(r * r + ell * ell);
        *val = type == ORC_MQ ? q : 1.0 / q;
        *dval = type == ORC_MQ ? ell / q : -ell / (q * q * q);
        return;
    }
    if (type == ORC_SINC) {
        double x = ell * r;
        *val = r == 0.0 ? ell : sin(x) / r;
        *dval = cos(x);
        return;
    }
    if (type == ORC_GAUSS) {
        double e = exp(-(r * r) / (2.0 * ell * ell));
        *val = e;
        *dval = (r * r) / (ell * ell * ell) * e;
    } else if (type == ORC_MATERN32) {
        double a = sqrt(3.0) * r / ell, e = exp(-a);
        *val = (1.0 + a) * e;
        *dval = 3.0 * r * r / (ell * ell * ell) * e;
    } else {
        double e = exp(-r / ell);
        *val = e;
        *dval = r / (ell * ell) * e;
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* O1: exact dense product for the target rows rows[0..nrows).
 *   Y    [nrows x nrhs]          sigma_f^2 sum_s K_s V + sigma_eps^2 V (rows only)
 *   DL   [P x nrows x nrhs] or 0 sigma_f^2 K_s^der V   (one block per window)
 *   KS   [P x nrows x nrhs] or 0 K_s V (unscaled, per window)
 * O(nrows * n * sum_s d_s); OpenMP over target rows. */
void orc_dense_apply(int64_t n, int32_t p, const double *X, int64_t ldx,
                     int32_t P, const int32_t *win_ptr, const int32_t *win_idx,
                     const int32_t *ktype, const double *ell,
                     double sigma_f, double sigma_eps,
                     const double *V, int32_t nrhs,
                     const int64_t *rows, int64_t nrows,
                     double *Y, double *DL, double *KS)
{
    (void)p;
    const double sf2 = sigma_f * sigma_f, se2 = sigma_eps * sigma_eps;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nrows; ++t) {
        const int64_t i = rows[t];
        double *y = Y + t * nrhs;
        for (int r = 0; r < nrhs; ++r) y[r] = se2 * V[i * nrhs + r];
        double acc[64], dacc[64];
        for (int32_t s = 0; s < P; ++s) {
            for (int r = 0; r < nrhs; ++r) { acc[r] = 0.0; dacc[r] = 0.0; }
            for (int64_t j = 0; j < n; ++j) {
                double r2 = 0.0;
                for (int32_t q = win_ptr[s]; q < win_ptr[s + 1]; ++q) {
                    double diff = X[i * ldx + win_idx[q]] - X[j * ldx + win_idx[q]];
                    r2 += diff * diff;
                }
                double kv, dkv;
                orc_kernel(ktype[s], sqrt(r2), ell[s], &kv, &dkv);
                for (int r = 0; r < nrhs; ++r) {
                    acc[r] += kv * V[j * nrhs + r];
                    dacc[r] += dkv * V[j * nrhs + r];
                }
            }
            for (int r = 0; r < nrhs; ++r) {
                y[r] += sf2 * acc[r];
                if (DL) DL[((int64_t)s * nrows + t) * nrhs + r] = sf2 * dacc[r];
                if (KS) KS[((int64_t)s * nrows + t) * nrhs + r] = acc[r];
            }
        }
    }
}

/* Dense kernel matrix of one window (or its ell-derivative), n x n row-major:
 * M_ij = kappa_s(x_i - x_j) (deriv = 0) or kappa_s^der(x_i - x_j) (deriv = 1). */
void orc_dense_matrix(int64_t n, const double *X, int64_t ldx,
                      int32_t nfeat, const int32_t *feat, int32_t ktype,
                      double ell, int deriv, double *M)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double r2 = 0.0;
            for (int32_t q = 0; q < nfeat; ++q) {
                double diff = X[i * ldx + feat[q]] - X[j * ldx + feat[q]];
                r2 += diff * diff;
            }
            double kv, dkv;
            orc_kernel(ktype, sqrt(r2), ell, &kv, &dkv);
            M[i * n + j] = deriv ? dkv : kv;
        }
    }
}

/* O2, pairwise form, one window: for target rows,
 *   h_i = sum_j v_j sum_{k in I_N} b_k cos(2 pi k.(x~_i - x~_j))
 * (eq. Fourier_sum, real part).  Xs holds the scaled window coordinates
 * (n x d row-major).  O(nrows * n * N^d): tiny inputs only. */
void orc_rf_pairwise(int64_t n, int32_t d, const double *Xs, int32_t N,
                     const double *b, const double *V, int32_t nrhs,
                     const int64_t *rows, int64_t nrows, double *H)
{
    int64_t K = 1;
    for (int q = 0; q < d; ++q) K *= N;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nrows; ++t) {
        const int64_t i = rows[t];
        for (int r = 0; r < nrhs; ++r) H[t * nrhs + r] = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double kappa_rf = 0.0;
            for (int64_t kk = 0; kk < K; ++kk) {
                int64_t rem = kk;
                double phase = 0.0;
                for (int q = d - 1; q >= 0; --q) {
                    int64_t kq = rem % N - N / 2;
                    rem /= N;
                    phase += (double)kq * (Xs[i * d + q] - Xs[j * d + q]);
                }
                kappa_rf += b[kk] * cos(2.0 * ORC_PI * phase);
            }
            for (int r = 0; r < nrhs; ++r) H[t * nrhs + r] += kappa_rf * V[j * nrhs + r];
        }
    }
}

/* Per-dimension exponentials e^{sign 2 pi i k x_q}, k in I_N (index k + N/2),
 * for one point x (d coordinates): ec/es[q * N + k] = cos/sin. */
static void orc_exp_tables(int32_t d, int32_t N, const double *x, double sign, double *ec, double *es)
{
    for (int q = 0; q < d; ++q)
        for (int k = 0; k < N; ++k) {
            double ang = sign * 2.0 * ORC_PI * (double)(k - N / 2) * x[q];
            ec[q * N + k] = cos(ang);
            es[q * N + k] = sin(ang);
        }
}

/* Product of the exponentials of all dimensions but the last, for the
 * row-major index `outer` over those dimensions (the exponential of k.x is
 * the product of the d one-dimensional exponentials). */
static void orc_exp_prefix(int32_t d, int32_t N, int64_t outer, const double *ec, const double *es,
                           double *pr, double *pi)
{
    double er = 1.0, ei = 0.0;
    for (int q = d - 2; q >= 0; --q) {
        int k = (int)(outer % N);
        outer /= N;
        double cr = ec[q * N + k], ci = es[q * N + k];
        double tr = er * cr - ei * ci;
        ei = er * ci + ei * cr;
        er = tr;
    }
    *pr = er;
    *pi = ei;
}

/* Inner sums of eq. Fourier_sum (adjoint non-equispaced DFT), one window:
 *   A[k][r] = sum_j v_j^r e^{-2 pi i k.x~_j},  k in I_N^d,
 * stored interleaved (re, im) as A[(kk * nrhs + r) * 2 + {0,1}], kk row-major
 * over (k_1 + N/2, ..., k_d + N/2), last fastest.
 * Only points with a non-zero row in V contribute, so a sparse V is cheap.
 * The exponential of k.x is formed as the product of the d one-dimensional
 * exponentials e^{-2 pi i k_q x_q}.  Each thread sums a disjoint range of
 * points into a private array; the partial arrays are then added in thread
 * order. */
void orc_ndft_adjoint(int64_t n, int32_t d, const double *Xs, int32_t N,
                      const double *V, int32_t nrhs, double *A)
{
    int64_t K = 1;
    for (int q = 0; q < d; ++q) K *= N;
    const int64_t len = K * nrhs * 2;
    memset(A, 0, sizeof(double) * len);
    int nt = orc_num_threads();
    double *part = (double *)calloc((size_t)nt * len, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *acc = part + (int64_t)tid * len;
        double *ec = (double *)malloc(sizeof(double) * 3 * N);
        double *es = (double *)malloc(sizeof(double) * 3 * N);
        const int last = d - 1;
#pragma omp for schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            const double *v = V + j * nrhs;
            int nz = 0;
            for (int r = 0; r < nrhs; ++r) nz |= (v[r] != 0.0);
            if (!nz) continue;
            orc_exp_tables(d, N, Xs + j * d, -1.0, ec, es);
            for (int64_t outer = 0; outer < K / N; ++outer) {
                double pr, pi;
                orc_exp_prefix(d, N, outer, ec, es, &pr, &pi);
                for (int k = 0; k < N; ++k) {
                    double cr = ec[last * N + k], ci = es[last * N + k];
                    double er = pr * cr - pi * ci, ei = pr * ci + pi * cr;
                    double *a = acc + (outer * N + k) * nrhs * 2;
                    for (int r = 0; r < nrhs; ++r) {
                        a[2 * r + 0] += v[r] * er;
                        a[2 * r + 1] += v[r] * ei;
                    }
                }
            }
        }
        free(ec);
        free(es);
    }
    for (int t = 0; t < nt; ++t)
        for (int64_t e = 0; e < len; ++e) A[e] += part[(int64_t)t * len + e];
    free(part);
}

/* Outer sums of eq. Fourier_sum (real part), one window, target rows:
 *   H[t][r] = Re sum_k b_k A[k][r] e^{2 pi i k.x~_i},  i = rows[t]. */
void orc_ndft_forward(int32_t d, const double *Xs, int32_t N, const double *b,
                      const double *A, int32_t nrhs,
                      const int64_t *rows, int64_t nrows, double *H)
{
    int64_t K = 1;
    for (int q = 0; q < d; ++q) K *= N;
#pragma omp parallel
    {
        double *ec = (double *)malloc(sizeof(double) * 3 * N);
        double *es = (double *)malloc(sizeof(double) * 3 * N);
        const int last = d - 1;
#pragma omp for schedule(dynamic, 4)
        for (int64_t t = 0; t < nrows; ++t) {
            const int64_t i = rows[t];
            double *h = H + t * nrhs;
            orc_exp_tables(d, N, Xs + i * d, 1.0, ec, es);
            for (int r = 0; r < nrhs; ++r) h[r] = 0.0;
            for (int64_t outer = 0; outer < K / N; ++outer) {
                double pr, pi;
                orc_exp_prefix(d, N, outer, ec, es, &pr, &pi);
                for (int k = 0; k < N; ++k) {
                    double cr = ec[last * N + k], ci = es[last * N + k];
                    double er = pr * cr - pi * ci, ei = pr * ci + pi * cr;
                    const int64_t kk = outer * N + k;
                    const double *a = A + kk * nrhs * 2;
                    for (int r = 0; r < nrhs; ++r)
                        h[r] += b[kk] * (a[2 * r + 0] * er - a[2 * r + 1] * ei);
                }
            }
        }
        free(ec);
        free(es);
    }
}
