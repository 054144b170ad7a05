// Per-hyper-parameter kernels (FP64): samples of the periodically continued
// kernel and of its ell-derivative on the N^d grid (Sec. 3.1, Sec. 3.2), their
// discrete Fourier coefficients b_k (eq. discrete_fourier_coefficients1), and
// the diagonal applied between the two FFTs of the fast summation:
//
//   D(k) = 1/2 (b(k) + b(-k)) / C(k)^2,   k in [-N/2, N/2]^d,
//
// where b is extended by zero outside I_N = [-N/2, N/2)^d, and C(k) is the
// product over dimensions of the normalised Kaiser-Bessel window coefficient
// I_0(m sqrt(beta^2 - (2 pi k / 2N)^2)) / I_0(m beta) (Appendix A: the window's
// Fourier coefficients are given by the modified Bessel function I_0).  The
// symmetrisation makes the product the real part of the trigonometric sum,
// which is the symmetric matrix sum_k b_k cos(2 pi k.(x_i - x_j)).
#include "nfftgp_impl.h"

namespace nfftgp {
namespace {

// Modified Bessel function I_0 from its power series sum ((z/2)^{2j} / (j!)^2).
__device__ double bessel_i0(double z)
{
    double q = 0.25 * z * z, term = 1.0, sum = 1.0;
    for (int j = 1; j < 500; ++j) {
        term *= q / ((double)j * (double)j);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

__global__ void k_sample(int d, int N, int kernel, double ell, double c, double *__restrict__ coef)
{
    int64_t K = 1;
    for (int q = 0; q < d; ++q) K *= N;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= K) return;
    int64_t rem = idx;
    double r2 = 0.0;
    for (int q = 0; q < d; ++q) {
        int l = (int)(rem % N) - N / 2;
        rem /= N;
        double x = (double)l / (double)N;
        r2 += x * x;
    }
    double r = sqrt(r2) / c;   // distance in caller units
    double v, dv;
    if (kernel == NFFTGP_GAUSS) {
        v = exp(-(r * r) / (2.0 * ell * ell));
        dv = (r * r) / (ell * ell * ell) * v;
    } else {
        v = exp(-r / ell);
        dv = r / (ell * ell) * v;
    }
    coef[2 * idx] = v;
    coef[2 * idx + 1] = 0.0;
    coef[2 * (K + idx)] = dv;
    coef[2 * (K + idx) + 1] = 0.0;
}

// One axis of the d-dimensional DFT, applied to two stacked arrays:
// out[.., k, ..] = sum_l in[.., l, ..] exp(-2 pi i l k / N), l, k in [-N/2, N/2).
__global__ void k_dft_axis(int d, int N, int axis, const double *__restrict__ in,
                           double *__restrict__ out)
{
    int64_t K = 1;
    for (int q = 0; q < d; ++q) K *= N;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 2 * K) return;
    int64_t arr = idx / K, e = idx % K;
    int64_t stride = 1;
    for (int q = d - 1; q > axis; --q) stride *= N;
    int kk = (int)((e / stride) % N);
    int64_t base = arr * K + e - (int64_t)kk * stride;
    int k = kk - N / 2;
    double sr = 0.0, si = 0.0;
    for (int ll = 0; ll < N; ++ll) {
        int l = ll - N / 2;
        int ph = ((l * k) % N + N) % N;               // exp(-2 pi i ph / N)
        double sn, cs;
        sincospi(-2.0 * (double)ph / (double)N, &sn, &cs);
        double ar = in[2 * (base + (int64_t)ll * stride)], ai = in[2 * (base + (int64_t)ll * stride) + 1];
        sr += ar * cs - ai * sn;
        si += ar * sn + ai * cs;
    }
    out[2 * (arr * K + e)] = sr;
    out[2 * (arr * K + e) + 1] = si;
}

// Normalised window coefficient per dimension, c(k) = I_0(m sqrt(beta^2 -
// (2 pi k / 2N)^2)) / I_0(m beta) for k = -N/2..N/2 (index k + N/2), stored as
// 1 / c(k)^2 -- the factor the diagonal applies once per transform.
__global__ void k_window_coef(int N, int m, double beta, double *__restrict__ cinv2)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > N) return;
    const int k = i - N / 2;
    const double w = 2.0 * kPi * k / (2.0 * N);
    const double c = bessel_i0(m * sqrt(beta * beta - w * w)) / bessel_i0(m * beta);
    cinv2[i] = 1.0 / (c * c);
}

template <typename T>
__global__ void k_make_diag(int d, int N, const double *__restrict__ cinv2,
                            const double *__restrict__ B, double *__restrict__ bbar,
                            T *__restrict__ Dk, T *__restrict__ Dder)
{
    int64_t K = 1, KD = 1;
    for (int q = 0; q < d; ++q) {
        K *= N;
        KD *= (N + 1);
    }
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double invK = 1.0 / (double)K;
    if (idx < K) {   // plain coefficients on I_N (for the definiteness report)
        bbar[idx] = B[2 * idx] * invK;
        bbar[K + idx] = B[2 * (K + idx)] * invK;
    }
    if (idx >= KD) return;
    int kv[3] = {0, 0, 0};
    int64_t rem = idx;
    for (int q = d - 1; q >= 0; --q) {
        kv[q] = (int)(rem % (N + 1)) - N / 2;
        rem /= (N + 1);
    }
    bool in_pos = true, in_neg = true;
    int64_t ip = 0, in_ = 0;
    double f = 1.0;
    for (int q = 0; q < d; ++q) {
        in_pos = in_pos && (kv[q] < N / 2);
        in_neg = in_neg && (-kv[q] < N / 2);
        ip = ip * N + (kv[q] + N / 2);
        in_ = in_ * N + (-kv[q] + N / 2);
        f *= cinv2[kv[q] + N / 2];
    }
    double bk = 0.0, bd = 0.0;
    if (in_pos) {
        bk += B[2 * ip] * invK;
        bd += B[2 * (K + ip)] * invK;
    }
    if (in_neg) {
        bk += B[2 * in_] * invK;
        bd += B[2 * (K + in_)] * invK;
    }
    Dk[idx] = (T)(0.5 * bk * f);
    Dder[idx] = (T)(0.5 * bd * f);
}

__global__ void __launch_bounds__(1024)
k_min2(const double *__restrict__ v, int64_t K, double *__restrict__ out)
{
    __shared__ double s0[1024], s1[1024];
    double a = INFINITY, b = INFINITY;
    for (int64_t i = threadIdx.x; i < K; i += 1024) {
        a = fmin(a, v[i]);
        b = fmin(b, v[K + i]);
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            s0[threadIdx.x] = fmin(s0[threadIdx.x], s0[threadIdx.x + off]);
            s1[threadIdx.x] = fmin(s1[threadIdx.x], s1[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s0[0];
        out[1] = s1[0];
    }
}

}  // namespace

hipError_t launch_window_coef(int N, int m, double *cinv2, hipStream_t s)
{
    k_window_coef<<<1, 256, 0, s>>>(N, m, kb_beta(), cinv2);
    return hipGetLastError();
}

hipError_t launch_coefficients(int prec, const WindowGeom &g, int m, int kernel, double ell,
                               double c, const double *cinv2, double *coef, double *bbar, void *Dk,
                               void *Dder, double *minb_out, hipStream_t s)
{
    (void)m;
    int64_t K = 1, KD = 1;
    for (int q = 0; q < g.d; ++q) {
        K *= g.N;
        KD *= (g.N + 1);
    }
    double *a = coef, *b = coef + 4 * K;   // two ping-pong buffers of 2 x K complex
    k_sample<<<(unsigned)((K + 255) / 256), 256, 0, s>>>(g.d, g.N, kernel, ell, c, a);
    for (int q = 0; q < g.d; ++q) {
        k_dft_axis<<<(unsigned)((2 * K + 255) / 256), 256, 0, s>>>(g.d, g.N, q, a, b);
        double *t = a;
        a = b;
        b = t;
    }
    int64_t nthr = KD > K ? KD : K;
    if (prec == NFFTGP_F32)
        k_make_diag<float><<<(unsigned)((nthr + 255) / 256), 256, 0, s>>>(
            g.d, g.N, cinv2, a, bbar, (float *)Dk, (float *)Dder);
    else
        k_make_diag<double><<<(unsigned)((nthr + 255) / 256), 256, 0, s>>>(
            g.d, g.N, cinv2, a, bbar, (double *)Dk, (double *)Dder);
    k_min2<<<1, 1024, 0, s>>>(bbar, K, minb_out);
    return hipGetLastError();
}

}  // namespace nfftgp
