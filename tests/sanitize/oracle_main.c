/* Drives every function of oracle/oracle.c on small inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py).
 * Besides running clean under the sanitizers it checks two identities the
 * oracle must satisfy: the non-equispaced DFT route of eq. Fourier_sum equals
 * the pairwise definition, and the dense kernel matrix is symmetric with a
 * unit diagonal. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_kernel(int type, double r, double ell, double *val, double *dval);
int orc_num_threads(void);
void orc_set_threads(int t);
void orc_dense_apply(int64_t n, int32_t p, const double *X, int64_t ldx, int32_t P, const int32_t *win_ptr,
                     const int32_t *win_idx, const int32_t *ktype, const double *ell, double sigma_f,
                     double sigma_eps, const double *V, int32_t nrhs, const int64_t *rows, int64_t nrows,
                     double *Y, double *DL, double *KS);
void orc_dense_matrix(int64_t n, const double *X, int64_t ldx, int32_t nfeat, const int32_t *feat,
                      int32_t ktype, double ell, int deriv, double *M);
void orc_rf_pairwise(int64_t n, int32_t d, const double *Xs, int32_t N, const double *b, const double *V,
                     int32_t nrhs, const int64_t *rows, int64_t nrows, double *H);
void orc_ndft_adjoint(int64_t n, int32_t d, const double *Xs, int32_t N, const double *V, int32_t nrhs,
                      double *A);
void orc_ndft_forward(int32_t d, const double *Xs, int32_t N, const double *b, const double *A,
                      int32_t nrhs, const int64_t *rows, int64_t nrows, double *H);

static uint64_t state = 0x9e3779b97f4a7c15ull;
static double unif(void)   /* splitmix64 -> [0, 1) */
{
    uint64_t z = (state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

int main(void)
{
    orc_set_threads(2);
    if (orc_num_threads() < 1) return 1;
    const int64_t n = 37;
    const int32_t p = 6, nrhs = 3, P = 3;
    double *X = malloc(sizeof(double) * n * p), *V = malloc(sizeof(double) * n * nrhs);
    for (int64_t i = 0; i < n * p; ++i) X[i] = 2.0 * unif() - 1.0;
    for (int64_t i = 0; i < n * nrhs; ++i) V[i] = unif() - 0.5;
    for (int t = 0; t < 3; ++t) {
        double v, dv;
        orc_kernel(t, 0.3, 0.7, &v, &dv);
        if (!isfinite(v) || !isfinite(dv)) return 2;
    }
    /* O1 on every row and a subset, three windows of dimension 3, 2, 1 */
    const int32_t win_ptr[4] = {0, 3, 5, 6}, win_idx[6] = {0, 1, 2, 3, 4, 5}, kt[3] = {0, 1, 2};
    const double ell[3] = {0.8, 0.5, 1.1};
    int64_t rows[5] = {0, 3, 17, 25, 36};
    double *Y = malloc(sizeof(double) * n * nrhs), *DL = malloc(sizeof(double) * P * n * nrhs),
           *KS = malloc(sizeof(double) * P * n * nrhs);
    int64_t *all = malloc(sizeof(int64_t) * n);
    for (int64_t i = 0; i < n; ++i) all[i] = i;
    orc_dense_apply(n, p, X, p, P, win_ptr, win_idx, kt, ell, 1.2, 0.3, V, nrhs, all, n, Y, DL, KS);
    orc_dense_apply(n, p, X, p, P, win_ptr, win_idx, kt, ell, 1.2, 0.3, V, nrhs, rows, 5, Y, NULL, NULL);
    /* dense matrix: symmetric, unit diagonal */
    double *M = malloc(sizeof(double) * n * n);
    for (int32_t t = 0; t < 3; ++t) {
        orc_dense_matrix(n, X, p, 3, win_idx, t, 0.6, 0, M);
        for (int64_t i = 0; i < n; ++i) {
            if (fabs(M[i * n + i] - 1.0) > 1e-15) return 3;
            for (int64_t j = 0; j < n; ++j)
                if (M[i * n + j] != M[j * n + i]) return 4;
        }
        orc_dense_matrix(n, X, p, 3, win_idx, t, 0.6, 1, M);
    }
    /* O2: pairwise against the NDFT route, d = 1, 2, 3, N = 8 */
    for (int32_t d = 1; d <= 3; ++d) {
        const int32_t N = 8;
        int64_t K = 1;
        for (int q = 0; q < d; ++q) K *= N;
        double *Xs = malloc(sizeof(double) * n * d), *b = malloc(sizeof(double) * K);
        double *A = malloc(sizeof(double) * K * nrhs * 2);
        double *H1 = malloc(sizeof(double) * n * nrhs), *H2 = malloc(sizeof(double) * n * nrhs);
        for (int64_t i = 0; i < n * d; ++i) Xs[i] = 0.5 * unif() - 0.25;
        for (int64_t k = 0; k < K; ++k) b[k] = unif();
        orc_rf_pairwise(n, d, Xs, N, b, V, nrhs, all, n, H1);
        orc_ndft_adjoint(n, d, Xs, N, V, nrhs, A);
        orc_ndft_forward(d, Xs, N, b, A, nrhs, all, n, H2);
        double scale = 0.0, err = 0.0;
        for (int64_t i = 0; i < n * nrhs; ++i) {
            scale = fmax(scale, fabs(H1[i]));
            err = fmax(err, fabs(H1[i] - H2[i]));
        }
        if (!(err <= 1e-12 * scale)) {
            printf("d=%d NDFT vs pairwise %.3e (scale %.3e)\n", d, err, scale);
            return 5;
        }
        free(Xs); free(b); free(A); free(H1); free(H2);
    }
    free(X); free(V); free(Y); free(DL); free(KS); free(all); free(M);
    printf("oracle sanitizer run ok\n");
    return 0;
}
