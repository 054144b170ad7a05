// Drives the host-side paths of libnfftgp that run without a GPU -- argument
// validation of every entry point, error reporting, and the FP64 Lanczos
// quadrature of nfftgp_slq_logquad -- for a host build with AddressSanitizer
// and UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  The quadrature
// is checked on CG coefficients of a diagonal matrix at full Krylov dimension,
// where e_1^T log(T) e_1 times |b|^2 equals b^T log(A) b exactly.
#include "nfftgp.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

static int fails = 0;
#define EXPECT(cond)                                                        \
    do {                                                                    \
        if (!(cond)) {                                                      \
            std::printf("line %d: expectation failed: %s\n", __LINE__, #cond); \
            ++fails;                                                        \
        }                                                                   \
    } while (0)

static void expect_error(nfftgp_status st)
{
    EXPECT(st != NFFTGP_OK);
    const char *msg = nfftgp_last_error();
    EXPECT(msg != nullptr && std::strlen(msg) > 0);
}

int main()
{
    nfftgp_plan plan = nullptr;
    const int32_t win_ptr[2] = {0, 3}, win_idx[3] = {0, 1, 2}, kern[1] = {NFFTGP_GAUSS}, N[1] = {16};
    double dummy[8] = {0};
    // plan creation: every rejected argument
    expect_error(nfftgp_plan_create(nullptr, dummy, 4, 3, 3, 1, win_ptr, win_idx, kern, N, 4, NFFTGP_F32, 0, 1,
                                    nullptr));
    expect_error(nfftgp_plan_create(&plan, dummy, -1, 3, 3, 1, win_ptr, win_idx, kern, N, 4, NFFTGP_F32, 0, 1,
                                    nullptr));
    expect_error(nfftgp_plan_create(&plan, nullptr, 4, 3, 3, 1, win_ptr, win_idx, kern, N, 4, NFFTGP_F32, 0, 1,
                                    nullptr));
    expect_error(nfftgp_plan_create(&plan, dummy, 4, 3, 2, 1, win_ptr, win_idx, kern, N, 4, NFFTGP_F32, 0, 1,
                                    nullptr));
    expect_error(nfftgp_plan_create(&plan, dummy, 4, 3, 3, 0, win_ptr, win_idx, kern, N, 4, NFFTGP_F32, 0, 1,
                                    nullptr));
    expect_error(nfftgp_plan_create(&plan, dummy, 4, 3, 3, 1, nullptr, win_idx, kern, N, 4, NFFTGP_F32, 0, 1,
                                    nullptr));
    expect_error(nfftgp_plan_create(&plan, dummy, 4, 3, 3, 1, win_ptr, win_idx, kern, N, 4, (nfftgp_prec)7, 0, 1,
                                    nullptr));
    expect_error(nfftgp_plan_create(&plan, dummy, 4, 3, 3, 1, win_ptr, win_idx, kern, N, 4, NFFTGP_F32, 0, 0,
                                    nullptr));
    const int32_t badN[1] = {15};
    expect_error(nfftgp_plan_create(&plan, dummy, 4, 3, 3, 1, win_ptr, win_idx, kern, badN, 4, NFFTGP_F32, 0, 1,
                                    nullptr));
    const int32_t bad_idx[3] = {0, 1, 7};
    expect_error(nfftgp_plan_create(&plan, dummy, 4, 3, 3, 1, win_ptr, bad_idx, kern, N, 4, NFFTGP_F32, 0, 1,
                                    nullptr));
    const double c0[3] = {0, 0, 0}, c_bad[1] = {-1.0};
    expect_error(nfftgp_plan_create_scaled(&plan, dummy, 4, 3, 3, 1, win_ptr, win_idx, kern, N, 4, NFFTGP_F32, c0,
                                           c_bad, 1, nullptr));
    EXPECT(plan == nullptr);
    // entry points on a NULL plan
    const double ell[1] = {0.5};
    expect_error(nfftgp_set_hyper(nullptr, 1.0, ell, 0.1));
    expect_error(nfftgp_apply(nullptr, dummy, 1, 1, dummy, nullptr, nullptr, nullptr));
    int32_t it[2] = {0, 0};
    double ab[8], res[2];
    expect_error(nfftgp_cg(nullptr, dummy, 1, dummy, 1e-6, 10, 1, it, ab, res));
    expect_error(nfftgp_pcg(nullptr, dummy, 1, dummy, 1e-6, 10, 1, it, ab, res));
    expect_error(nfftgp_col_dots(nullptr, dummy, 1, dummy, 1, 1, 0, dummy));
    expect_error(nfftgp_col_dots_noalloc(NFFTGP_F64, dummy, 1, dummy, 1, 1, 65, dummy, nullptr));
    double c0o[3], co, mb[2];
    int32_t dd, NN;
    expect_error(nfftgp_get_window_info(nullptr, 0, c0o, &co, &dd, &NN, &mb[0], &mb[1]));
    size_t bytes = 0;
    expect_error(nfftgp_get_workspace_bytes(nullptr, &bytes));
    char rep[64];
    expect_error(nfftgp_describe(nullptr, 1, rep, sizeof(rep)));
    expect_error(nfftgp_autotune(nullptr, 1, 1, 1, rep, sizeof(rep)));
    expect_error(nfftgp_profile(nullptr, 0));
    expect_error(nfftgp_precond_attach(nullptr, dummy, 3, 4, 8, 8));
    int32_t k = 0, nb = 0;
    double ld = 0.0;
    expect_error(nfftgp_precond_info(nullptr, &k, &nb, &ld, dummy));
    expect_error(nfftgp_precond_apply(nullptr, NFFTGP_PC_MINV, dummy, 1, dummy));
    nfftgp_plan_destroy(nullptr);
    // Lanczos quadrature: CG on A = diag(lambda), b = ones, run to full dimension
    const int n = 6;
    const double lam[n] = {0.5, 1.0, 2.0, 3.5, 7.0, 11.0};
    std::vector<double> x(n, 0.0), r(n, 1.0), p(n, 1.0), hist(2 * n);
    double rr = n;
    for (int j = 0; j < n; ++j) {
        double pap = 0.0;
        for (int i = 0; i < n; ++i) pap += p[i] * lam[i] * p[i];
        const double alpha = rr / pap;
        double rr2 = 0.0;
        for (int i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * lam[i] * p[i];
            rr2 += r[i] * r[i];
        }
        const double beta = rr2 / rr;
        for (int i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rr = rr2;
        hist[2 * j] = alpha;
        hist[2 * j + 1] = beta;
    }
    const int32_t iters[1] = {n};
    const double zn[1] = {(double)n};
    double out[1] = {0.0};
    EXPECT(nfftgp_slq_logquad(hist.data(), iters, 1, n, zn, out) == NFFTGP_OK);
    double exact = 0.0;
    for (int i = 0; i < n; ++i) exact += std::log(lam[i]);
    EXPECT(std::fabs(out[0] - exact) <= 1e-10 * std::fabs(exact));
    const int32_t bad_it[1] = {n + 1};
    expect_error(nfftgp_slq_logquad(hist.data(), bad_it, 1, n, zn, out));
    expect_error(nfftgp_slq_logquad(nullptr, iters, 1, n, zn, out));
    if (fails == 0) std::printf("abi sanitizer run ok (quadrature %.15g, exact %.15g)\n", out[0], exact);
    return fails == 0 ? 0 : 1;
}
