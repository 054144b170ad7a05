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

constexpr int kMaxH = 65;   // N/2 + 1 for N <= 128

// All per-hyper-parameter work of one window and one array (kernel or
// ell-derivative) in one work-group.  The samples f(l) = kappa(|l| / N),
// l in [-N/2, N/2)^d, are real and even in every coordinate (l = -N/2 has no
// partner and enters once), so their DFT is real and even; per axis
//
//   sum_l g(l) exp(-2 pi i l k / N) = g(0) + 2 sum_{0<l<N/2} g(l) cos(2 pi l k / N)
//                                     + g(N/2) (-1)^k,
//
// a real transform on the H = N/2 + 1 magnitudes l, k = 0..N/2, applied axis
// by axis (scratch: two arrays of H^d doubles per window and array).  Then
// b(k) = N^-d B(|k_1|, .., |k_d|) on I_N, the smallest b_k is the smallest of
// these values, and in D(k) the term b(k) counts when no k_q = N/2, the term
// b(-k) when no k_q = -N/2.  Grid (2, nwin): x = array (0: K, 1: derivative),
// y = window of the group; the smallest coefficient goes to
// minb[2 * s_global + x] (host-visible memory) and the transformed array to
// the start of the block's scratch, where k_coef_diag reads it.
// With INLDS the two H^d arrays live in LDS (dynamic shared memory, used when
// they fit); otherwise in the global scratch.
template <bool INLDS>
__global__ void __launch_bounds__(1024)
k_coef_all(int d, int N, CoefParams prm, double *__restrict__ scratch, const WinDesc *__restrict__ wd,
           double *__restrict__ minb)
{
    __shared__ double cw[kMaxH * kMaxH];
    __shared__ double red[1024];
    extern __shared__ double dyn[];
    const int arr = blockIdx.x, w = blockIdx.y;
    const int H = N / 2 + 1;
    const float invH = 1.0f / (float)H;
    int KH = 1, K = 1;   // at most 65^3
    for (int q = 0; q < d; ++q) {
        KH *= H;
        K *= N;
    }
    double *A = INLDS ? dyn : scratch + ((int64_t)w * 2 + arr) * 2 * KH;
    double *B = A + KH;
    for (int i = threadIdx.x; i < H * H; i += blockDim.x) {
        const int l = i / H, k = i % H;
        double c;
        if (l == 0) c = 1.0;
        else if (l == N / 2) c = (k & 1) ? -1.0 : 1.0;
        else c = 2.0 * cospi(2.0 * (double)((l * k) & (N - 1)) / (double)N);
        cw[i] = c;
    }
    // samples at magnitudes l_q = 0..N/2 (l_q = N/2 stands for the offset -N/2)
    for (int i = threadIdx.x; i < KH; i += blockDim.x) {
        int rem = i;
        double r2 = 0.0;
        for (int q = 0; q < d; ++q) {
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
    // axis passes (axis q has stride H^(d-1-q))
    int stride = KH / H;
    for (int q = 0; q < d; ++q) {
        const float inv_st = 1.0f / (float)stride;
        for (int i = threadIdx.x; i < KH; i += blockDim.x) {
            const int hi = fdiv_small(i, stride, inv_st);   // i / stride
            const int k = hi - fdiv_small(hi, H, invH) * H;
            const int base = i - k * stride;
            double acc = 0.0;
            for (int l = 0; l < H; ++l) acc += cw[l * H + k] * A[base + l * stride];
            B[i] = acc;
        }
        __syncthreads();
        double *t = A;
        A = B;
        B = t;
        stride /= H;
    }
    const double invK = 1.0 / (double)K;
    double mn = INFINITY;
    for (int i = threadIdx.x; i < KH; i += blockDim.x) mn = fmin(mn, A[i] * invK);
    red[threadIdx.x] = mn;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) minb[2 * wd[w].s_global + arr] = red[0];
    // transformed array for the diagonal kernel
    double *out = scratch + ((int64_t)w * 2 + arr) * 2 * KH;
    if (INLDS || out != A)
        for (int i = threadIdx.x; i < KH; i += blockDim.x) out[i] = A[i];
}

// Diagonal D(k) on [-N/2, N/2]^d of every window and array of the group from
// the transformed arrays (scratch layout of k_coef_all).  Grid
// (ceil((N+1)^d / 256), 2, nwin).
template <typename T>
__global__ void __launch_bounds__(256)
k_coef_diag(int d, int N, const double *__restrict__ cinv2, const double *__restrict__ scratch,
            const WinDesc *__restrict__ wd)
{
    const int arr = blockIdx.y, w = blockIdx.z;
    const int H = N / 2 + 1;
    const float invN1 = 1.0f / (float)(N + 1);
    int KH = 1, KD = 1, K = 1;
    for (int q = 0; q < d; ++q) {
        KH *= H;
        KD *= N + 1;
        K *= N;
    }
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= KD) return;
    const double *A = scratch + ((int64_t)w * 2 + arr) * 2 * KH;
    int rem = i, ai = 0, astr = 1;
    bool in_pos = true, in_neg = true;
    double f = 1.0;
    for (int q = d - 1; q >= 0; --q) {
        const int qt = fdiv_small(rem, N + 1, invN1);
        const int k = rem - qt * (N + 1) - N / 2;
        rem = qt;
        in_pos = in_pos && k < N / 2;
        in_neg = in_neg && k > -N / 2;
        ai += (k < 0 ? -k : k) * astr;
        astr *= H;
        f *= cinv2[k + N / 2];
    }
    const double cnt = (in_pos ? 1.0 : 0.0) + (in_neg ? 1.0 : 0.0);
    T *Dout = reinterpret_cast<T *>(const_cast<void *>(arr == 0 ? wd[w].Dk : wd[w].Dder));
    Dout[i] = (T)(0.5 * cnt * A[ai] / (double)K * f);
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

hipError_t launch_window_coef(int N, int m, double *cinv2, hipStream_t s)
{
    k_window_coef<<<1, 256, 0, s>>>(N, m, kb_beta(), cinv2);
    return hipGetLastError();
}

int64_t coef_scratch_doubles(const WindowGeom &g, int nwin)
{
    int64_t KH = 1;
    for (int q = 0; q < g.d; ++q) KH *= g.N / 2 + 1;
    return 4 * KH * nwin;
}

hipError_t launch_coefficients(int prec, const Group &G, const CoefParams &prm, const double *cinv2,
                               double *scratch, double *minb, hipStream_t s)
{
    const dim3 grid(2, (unsigned)G.nwin);
    int64_t KH = 1, KD = 1;
    for (int q = 0; q < G.g.d; ++q) {
        KH *= G.g.N / 2 + 1;
        KD *= G.g.N + 1;
    }
    const size_t lds = (size_t)2 * KH * sizeof(double);
    if (lds <= 96 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k_coef_all<true>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        k_coef_all<true><<<grid, 1024, lds, s>>>(G.g.d, G.g.N, prm, scratch, G.desc, minb);
    } else {
        k_coef_all<false><<<grid, 1024, 0, s>>>(G.g.d, G.g.N, prm, scratch, G.desc, minb);
    }
    const dim3 dgrid((unsigned)((KD + 255) / 256), 2, (unsigned)G.nwin);
    if (prec == NFFTGP_F32)
        k_coef_diag<float><<<dgrid, 256, 0, s>>>(G.g.d, G.g.N, cinv2, scratch, G.desc);
    else
        k_coef_diag<double><<<dgrid, 256, 0, s>>>(G.g.d, G.g.N, cinv2, scratch, G.desc);
    return hipGetLastError();
}

}  // namespace nfftgp
