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

// Kernel and ell-derivative samples at grid offset l (index set [-N/2, N/2)^d,
// spacing 1/N in scaled units); r is the distance in caller units.
__device__ __forceinline__ void sample_pair(const CoefParams &prm, int w, double r2, double &v,
                                            double &dv)
{
    const double ell = prm.ell[w];
    const double r = sqrt(r2) / prm.c[w];
    if (prm.kernel[w] == NFFTGP_GAUSS) {
        v = exp(-(r * r) / (2.0 * ell * ell));
        dv = (r * r) / (ell * ell * ell) * v;
    } else {
        v = exp(-r / ell);
        dv = r / (ell * ell) * v;
    }
}

// First DFT axis (axis 0) of the samples of every window of a group, with the
// samples evaluated on the fly.  Output arrays [window][2][K] of complex values
// (kernel, then ell-derivative), K = N^d, index l + N/2 per axis:
// out[k, rest] = sum_l f(l, rest) exp(-2 pi i l k / N); tw[j] = exp(-2 pi i j / N).
__global__ void k_dft_first(int d, int N, CoefParams prm, const double2 *__restrict__ tw,
                            double *__restrict__ out)
{
    int64_t K = 1;
    for (int q = 0; q < d; ++q) K *= N;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= K * prm.nwin) return;
    const int w = (int)(idx / K);
    const int64_t e = idx % K;
    const int64_t stride = K / N;                  // axis 0 is the slowest index
    const int k = (int)(e / stride) - N / 2;
    int64_t rem = e % stride;
    double rest2 = 0.0;
    for (int q = 1; q < d; ++q) {
        const int l = (int)(rem % N) - N / 2;      // last axis fastest
        rem /= N;
        const double x = (double)l / (double)N;
        rest2 += x * x;
    }
    double sr = 0.0, si = 0.0, dr = 0.0, di = 0.0;
    for (int ll = 0; ll < N; ++ll) {
        const int l = ll - N / 2;
        const double x = (double)l / (double)N;
        double v, dv;
        sample_pair(prm, w, rest2 + x * x, v, dv);
        const double2 t = tw[(l * k) & (N - 1)];   // N is a power of two
        sr += v * t.x;
        si += v * t.y;
        dr += dv * t.x;
        di += dv * t.y;
    }
    double *base = out + (int64_t)w * 4 * K;
    base[2 * e] = sr;
    base[2 * e + 1] = si;
    base[2 * (K + e)] = dr;
    base[2 * (K + e) + 1] = di;
}

// One further axis of the d-dimensional DFT, applied to all 2 x nwin stacked
// arrays: out[.., k, ..] = sum_l in[.., l, ..] exp(-2 pi i l k / N).
__global__ void k_dft_axis(int d, int N, int axis, int narr, const double2 *__restrict__ tw,
                           const double *__restrict__ in, double *__restrict__ out)
{
    int64_t K = 1;
    for (int q = 0; q < d; ++q) K *= N;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)narr * K) return;
    int64_t arr = idx / K, e = idx % K;
    int64_t stride = 1;
    for (int q = d - 1; q > axis; --q) stride *= N;
    int kk = (int)((e / stride) % N);
    int64_t base = arr * K + e - (int64_t)kk * stride;
    int k = kk - N / 2;
    double sr = 0.0, si = 0.0;
    for (int ll = 0; ll < N; ++ll) {
        int l = ll - N / 2;
        const double2 t = tw[(l * k) & (N - 1)];
        double ar = in[2 * (base + (int64_t)ll * stride)], ai = in[2 * (base + (int64_t)ll * stride) + 1];
        sr += ar * t.x - ai * t.y;
        si += ar * t.y + ai * t.x;
    }
    out[2 * (arr * K + e)] = sr;
    out[2 * (arr * K + e) + 1] = si;
}

__global__ void k_twiddles(int N, double2 *__restrict__ tw)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    double sn, cs;
    sincospi(-2.0 * (double)j / (double)N, &sn, &cs);
    tw[j] = make_double2(cs, sn);
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

// Grid (ceil(span / 256), nwin): block x of window y.  Besides the diagonal,
// every block writes the minima of the plain coefficients b_k, b^der_k it
// visited to part[(y * gridDim.x + x) * 2 + {0, 1}].
template <typename T>
__global__ void __launch_bounds__(256)
k_make_diag(int d, int N, const double *__restrict__ cinv2, const double *__restrict__ coef,
            const WinDesc *__restrict__ wd, double *__restrict__ part)
{
    __shared__ double s0[256], s1[256];
    int64_t K = 1, KD = 1;
    for (int q = 0; q < d; ++q) {
        K *= N;
        KD *= (N + 1);
    }
    const int w = blockIdx.y;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double *B = coef + (int64_t)w * 4 * K;
    const double invK = 1.0 / (double)K;
    double mk = INFINITY, md = INFINITY;
    if (idx < K) {   // plain coefficients on I_N (for the definiteness report)
        mk = B[2 * idx] * invK;
        md = B[2 * (K + idx)] * invK;
    }
    if (idx < KD) {
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
        reinterpret_cast<T *>(const_cast<void *>(wd[w].Dk))[idx] = (T)(0.5 * bk * f);
        reinterpret_cast<T *>(const_cast<void *>(wd[w].Dder))[idx] = (T)(0.5 * bd * f);
    }
    s0[threadIdx.x] = mk;
    s1[threadIdx.x] = md;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            s0[threadIdx.x] = fmin(s0[threadIdx.x], s0[threadIdx.x + off]);
            s1[threadIdx.x] = fmin(s1[threadIdx.x], s1[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t o = ((int64_t)w * gridDim.x + blockIdx.x) * 2;
        part[o] = s0[0];
        part[o + 1] = s1[0];
    }
}

// Smallest b_k and b^der_k of every window of the group (one block per window)
// from the block minima, written to minb[2 * s_global + {0, 1}].
__global__ void __launch_bounds__(256)
k_min2(const double *__restrict__ part, int nper, const WinDesc *__restrict__ wd,
       double *__restrict__ minb)
{
    __shared__ double s0[256], s1[256];
    const int w = blockIdx.x;
    const double *v = part + (int64_t)w * nper * 2;
    double a = INFINITY, b = INFINITY;
    for (int i = threadIdx.x; i < nper; i += 256) {
        a = fmin(a, v[2 * i]);
        b = fmin(b, v[2 * i + 1]);
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            s0[threadIdx.x] = fmin(s0[threadIdx.x], s0[threadIdx.x + off]);
            s1[threadIdx.x] = fmin(s1[threadIdx.x], s1[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        minb[2 * wd[w].s_global] = s0[0];
        minb[2 * wd[w].s_global + 1] = s1[0];
    }
}

}  // namespace

hipError_t launch_window_coef(int N, int m, double *cinv2, hipStream_t s)
{
    k_window_coef<<<1, 256, 0, s>>>(N, m, kb_beta(), cinv2);
    return hipGetLastError();
}

hipError_t launch_twiddles(int N, double2 *tw, hipStream_t s)
{
    k_twiddles<<<(N + 255) / 256, 256, 0, s>>>(N, tw);
    return hipGetLastError();
}

hipError_t launch_coefficients(int prec, const Group &G, const CoefParams &prm, const double *cinv2,
                               const double2 *tw, double *coef, double *bbar, double *minb,
                               hipStream_t s)
{
    const WindowGeom &g = G.g;
    int64_t K = 1, KD = 1;
    for (int q = 0; q < g.d; ++q) {
        K *= g.N;
        KD *= (g.N + 1);
    }
    const int nw = G.nwin;
    double *a = coef, *b = coef + (int64_t)nw * 4 * K;   // ping-pong: [window][2][K] complex each
    k_dft_first<<<(unsigned)((nw * K + 255) / 256), 256, 0, s>>>(g.d, g.N, prm, tw, a);
    for (int q = 1; q < g.d; ++q) {
        k_dft_axis<<<(unsigned)((2 * nw * K + 255) / 256), 256, 0, s>>>(g.d, g.N, q, 2 * nw, tw, a, b);
        double *t = a;
        a = b;
        b = t;
    }
    const unsigned nper = (unsigned)(((KD > K ? KD : K) + 255) / 256);
    const dim3 grid(nper, (unsigned)nw);
    if (prec == NFFTGP_F32)
        k_make_diag<float><<<grid, 256, 0, s>>>(g.d, g.N, cinv2, a, G.desc, bbar);
    else
        k_make_diag<double><<<grid, 256, 0, s>>>(g.d, g.N, cinv2, a, G.desc, bbar);
    k_min2<<<nw, 256, 0, s>>>(bbar, (int)nper, G.desc, minb);
    return hipGetLastError();
}

}  // namespace nfftgp
