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
#include "nfftgp_dev.h"
#include "nfftgp_coef_sep.h"

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

// Kernel and ell-derivative at distance sqrt(r2) in scaled units (converted to
// caller units by the window's scale c).
// Multiquadric, inverse multiquadric and sinc kernels at distance r >= 0 with
// shape parameter c, and their derivatives in c.
__device__ __forceinline__ void kernel_shape(int type, double r, double c, double &v, double &dv)
{
    if (type == NFFTGP_SINC) {
        // sin(c r) / r = c sin(x) / x, x = c r; d/dc = cos(c r)
        const double x = c * r;
        v = fabs(x) < 1e-4 ? c * (1.0 - x * x / 6.0) : sin(x) / r;
        dv = cos(x);
    } else {
        const double q = sqrt(r * r + c * c);
        if (type == NFFTGP_MQ) {
            v = q;
            dv = c / q;
        } else {
            v = 1.0 / q;
            dv = -c / (q * q * q);
        }
    }
}

__device__ __forceinline__ void sample_pair(const CoefParams &prm, int w, double r2, double &v,
                                            double &dv)
{
    const double ell = prm.ell[w];
    const double r = sqrt(r2) / prm.c[w];
    if (prm.kernel[w] == NFFTGP_GAUSS) {
        v = exp(-(r * r) / (2.0 * ell * ell));
        dv = (r * r) / (ell * ell * ell) * v;
    } else if (prm.kernel[w] == NFFTGP_MATERN32) {
        // (1 + a) e^-a with a = sqrt(3) r / ell; d/d ell = (3 r^2 / ell^3) e^-a
        const double a = 1.7320508075688772 * r / ell, e = exp(-a);
        v = (1.0 + a) * e;
        dv = 3.0 * r * r / (ell * ell * ell) * e;
    } else if (prm.kernel[w] >= NFFTGP_MQ) {
        kernel_shape(prm.kernel[w], r, ell, v, dv);
    } else {
        v = exp(-r / ell);
        dv = r / (ell * ell) * v;
    }
}

constexpr int kMaxH = 65;   // N/2 + 1 for N <= 128

// The samples f(l) = kappa(|l| / N), l in [-N/2, N/2)^d, are real and even in
// every coordinate (l = -N/2 has no partner and enters once), so their DFT is
// real and even; per axis
//
//   sum_l g(l) exp(-2 pi i l k / N) = g(0) + 2 sum_{0<l<N/2} g(l) cos(2 pi l k / N)
//                                     + g(N/2) (-1)^k,
//
// a real transform on the H = N/2 + 1 magnitudes l, k = 0..N/2, applied axis
// by axis.  Then b(k) = N^-d B(|k_1|, .., |k_d|) on I_N, the smallest b_k is
// the smallest of these values, and in D(k) the term b(k) counts when no
// k_q = N/2, the term b(-k) when no k_q = -N/2.
__device__ __forceinline__ double cos_weight(int l, int k, int N)
{
    if (l == 0) return 1.0;
    if (l == N / 2) return (k & 1) ? -1.0 : 1.0;
    return 2.0 * cospi(2.0 * (double)((l * k) & (N - 1)) / (double)N);
}

// Stage 1: samples and the transforms of axes 0..d-2 of one slab (last-axis
// magnitude l = blockIdx.x) of one window (blockIdx.z) and array (blockIdx.y:
// 0 kernel, 1 derivative), in LDS.  Output S[w][arr][k_0..k_{d-2}][l] in the
// scratch (H^d doubles per window and array).
__global__ void __launch_bounds__(256)
k_coef_slab(int d, int N, CoefParams prm, const double *__restrict__ cwg, double *__restrict__ scratch)
{
    __shared__ double cw[kMaxH * kMaxH];
    // a slab holds H^(d-1) values: at most 33^2 (d = 3 needs N <= 64), 65 for d = 2
    __shared__ double A[33 * 33], B[33 * 33];
    const int l_last = blockIdx.x, arr = blockIdx.y, w = blockIdx.z;
    const int H = N / 2 + 1;
    const float invH = 1.0f / (float)H;
    int KS = 1;   // slab size H^(d-1)
    for (int q = 0; q + 1 < d; ++q) KS *= H;
    int KH = KS * H;
    for (int i = threadIdx.x; i < H * H && d > 1; i += 256) cw[i] = cwg[i];
    const double xl = (double)l_last / (double)N;
    for (int i = threadIdx.x; i < KS; i += 256) {
        int rem = i;
        double r2 = xl * xl;
        for (int q = 0; q + 1 < d; ++q) {
            const int qt = fdiv_small(rem, H, invH);
            const double x = (double)(rem - qt * H) / (double)N;
            rem = qt;
            r2 += x * x;
        }
        double v, dv;
        sample_pair(prm, w, r2, v, dv);
        A[i] = arr == 0 ? v : dv;
    }
    __syncthreads();
    double *src = A, *dst = B;
    int stride = KS / H;   // axis q of the slab has stride H^(d-2-q)
    for (int q = 0; q + 1 < d; ++q) {
        const float inv_st = 1.0f / (float)stride;
        for (int i = threadIdx.x; i < KS; i += 256) {
            const int hi = fdiv_small(i, stride, inv_st);
            const int k = hi - fdiv_small(hi, H, invH) * H;
            const int base = i - k * stride;
            double acc = 0.0;
            for (int l = 0; l < H; ++l) acc += cw[l * H + k] * src[base + l * stride];
            dst[i] = acc;
        }
        __syncthreads();
        double *t = src;
        src = dst;
        dst = t;
        stride = stride > 1 ? stride / H : 1;
    }
    double *S = scratch + ((int64_t)w * 2 + arr) * KH;
    for (int i = threadIdx.x; i < KS; i += 256) S[(int64_t)i * H + l_last] = src[i];
}

// Stage 2: transform of the last axis on the fly and the diagonal
// D(k) on [-N/2, N/2]^d; the smallest b over the block goes to
// part[(w * 2 + arr) * gridDim.x + blockIdx.x].  Grid (ceil((N+1)^d / 256), 2, nwin).
template <typename T>
__global__ void __launch_bounds__(256)
k_coef_diag(int d, int N, const double *__restrict__ cinv2, const double *__restrict__ cwg,
            const double *__restrict__ scratch, const WinDesc *__restrict__ wd, double *__restrict__ part)
{
    __shared__ double cw[kMaxH * kMaxH];
    __shared__ double red[256];
    const int arr = blockIdx.y, w = blockIdx.z;
    const int H = N / 2 + 1;
    const float invN1 = 1.0f / (float)(N + 1);
    for (int j = threadIdx.x; j < H * H; j += 256) cw[j] = cwg[j];
    __syncthreads();
    int KH = 1, KD = 1, K = 1;
    for (int q = 0; q < d; ++q) {
        KH *= H;
        KD *= N + 1;
        K *= N;
    }
    const int i = blockIdx.x * 256 + threadIdx.x;
    const double *S = scratch + ((int64_t)w * 2 + arr) * KH;
    double b = INFINITY;
    if (i < KD) {
        int rem = i, ai = 0, astr = H, kl = 0;
        bool in_pos = true, in_neg = true;
        double f = 1.0;
        for (int q = d - 1; q >= 0; --q) {
            const int qt = fdiv_small(rem, N + 1, invN1);
            const int k = rem - qt * (N + 1) - N / 2;
            rem = qt;
            in_pos = in_pos && k < N / 2;
            in_neg = in_neg && k > -N / 2;
            const int ka = k < 0 ? -k : k;
            if (q == d - 1) kl = ka;
            else {
                ai += ka * astr;
                astr *= H;
            }
            f *= cinv2[k + N / 2];
        }
        // S is stored [slab index][last-axis l]; ai = H * slab index
        double acc = 0.0;
        for (int l = 0; l < H; ++l) acc += cw[l * H + kl] * S[ai + l];
        b = acc / (double)K;
        const double c = (in_pos ? 1.0 : 0.0) + (in_neg ? 1.0 : 0.0);
        T *Dout = reinterpret_cast<T *>(const_cast<void *>(arr == 0 ? wd[w].Dk : wd[w].Dder));
        Dout[i] = (T)(0.5 * c * b * f);
    }
    red[threadIdx.x] = b;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[((int64_t)w * 2 + arr) * gridDim.x + blockIdx.x] = red[0];
}

// Separable kernels (every window of the group Gaussian): one launch of
// coef_sep_block (nfftgp_coef_sep.h).  Grid (ceil((N+1)^d / 256), 2, nwin).
template <typename T>
__global__ void __launch_bounds__(256)
k_coef_sep(int d, int N, CoefParams prm, const double *__restrict__ cinv2, const double *__restrict__ cwg,
           const WinDesc *__restrict__ wd, double *__restrict__ part)
{
    __shared__ double lds[4 * kCoefMaxH + 256];
    coef_sep_block<T>(d, N, prm, cinv2, cwg, wd, part, blockIdx.x, gridDim.x, blockIdx.y, blockIdx.z, lds);
}

// Stage 3: smallest coefficient of every window (blockIdx.y) and array
// (blockIdx.x) from the block minima, written to minb[2 * s_global + arr]
// (host-visible memory).
__global__ void __launch_bounds__(256)
k_coef_min(const double *__restrict__ part, int nper, const WinDesc *__restrict__ wd,
           double *__restrict__ minb)
{
    __shared__ double red[256];
    const int arr = blockIdx.x, w = blockIdx.y;
    const double *p = part + ((int64_t)w * 2 + arr) * nper;
    double m = INFINITY;
    for (int j = threadIdx.x; j < nper; j += 256) m = fmin(m, p[j]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) minb[2 * wd[w].s_global + arr] = red[0];
}

// Weights cw[l * H + k] of the real transform on the H = N/2 + 1 magnitudes.
__global__ void k_cos_table(int N, double *__restrict__ cw)
{
    const int H = N / 2 + 1;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < H * H) cw[i] = cos_weight(i / H, i % H, N);
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

}  // namespace

hipError_t launch_window_coef(int N, int m, double *cinv2, double *cw, hipStream_t s)
{
    k_window_coef<<<1, 256, 0, s>>>(N, m, kb_beta(), cinv2);
    const int H = N / 2 + 1;
    k_cos_table<<<(H * H + 255) / 256, 256, 0, s>>>(N, cw);
    return hipGetLastError();
}

int64_t coef_scratch_doubles(const WindowGeom &g, int nwin)
{
    int64_t KH = 1, KD = 1;
    for (int q = 0; q < g.d; ++q) {
        KH *= g.N / 2 + 1;
        KD *= g.N + 1;
    }
    (void)KD;
    return 2 * KH * nwin;   // the slabs of every window and array
}

int64_t coef_part_doubles(const WindowGeom &g, int nwin)
{
    int64_t KD = 1;
    for (int q = 0; q < g.d; ++q) KD *= g.N + 1;
    return 2 * ((KD + 255) / 256) * nwin;
}

hipError_t launch_coefficients(int prec, const Group &G, const CoefParams &prm, const double *cinv2,
                               double *scratch, hipStream_t s)
{
    const int d = G.g.d, N = G.g.N, H = N / 2 + 1;
    int64_t KH = 1, KD = 1;
    for (int q = 0; q < d; ++q) {
        KH *= H;
        KD *= N + 1;
    }
    const unsigned nper = (unsigned)((KD + 255) / 256);
    const dim3 dgrid(nper, 2, (unsigned)G.nwin);
    bool separable = true;
    for (int w = 0; w < prm.nwin; ++w) separable = separable && prm.kernel[w] == NFFTGP_GAUSS;
    if (separable) {
        if (prec == NFFTGP_F32)
            k_coef_sep<float><<<dgrid, 256, 0, s>>>(d, N, prm, cinv2, G.cw, G.desc, G.coef_part);
        else
            k_coef_sep<double><<<dgrid, 256, 0, s>>>(d, N, prm, cinv2, G.cw, G.desc, G.coef_part);
        return hipGetLastError();
    }
    k_coef_slab<<<dim3((unsigned)H, 2, (unsigned)G.nwin), 256, 0, s>>>(d, N, prm, G.cw, scratch);
    if (prec == NFFTGP_F32)
        k_coef_diag<float><<<dgrid, 256, 0, s>>>(d, N, cinv2, G.cw, scratch, G.desc, G.coef_part);
    else
        k_coef_diag<double><<<dgrid, 256, 0, s>>>(d, N, cinv2, G.cw, scratch, G.desc, G.coef_part);
    return hipGetLastError();
}

hipError_t launch_coef_min(const Group &G, double *minb, hipStream_t s)
{
    int64_t KD = 1;
    for (int q = 0; q < G.g.d; ++q) KD *= G.g.N + 1;
    const int nper = (int)((KD + 255) / 256);
    k_coef_min<<<dim3(2, (unsigned)G.nwin), 256, 0, s>>>(G.coef_part, nper, G.desc, minb);
    return hipGetLastError();
}

}  // namespace nfftgp
