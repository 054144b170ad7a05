// Separable (Gaussian) coefficients of one block: shared by the
// coefficient kernel and by the fold kernel, which carries this work in
// extra work-groups when an apply follows a set_hyper (one launch fewer).
#pragma once

#include "nfftgp_impl.h"
#include "nfftgp_dev.h"

namespace nfftgp {

constexpr int kCoefMaxH = 65;   // N/2 + 1 for N <= 128

// Every window of the group Gaussian.  The samples are a product over
// dimensions, g(x_0) ... g(x_{d-1}) with g(x) = exp(-(x/c)^2 / (2 ell^2)), so
// b(k) = prod_q B1(|k_q|) / N^d with B1 the real transform of g on the H
// magnitudes (weights cwg[l * H + k]), and the ell-derivative, whose samples
// are sum_q g'(x_q) prod_{p != q} g(x_p) with g'(x) = (x/c)^2 / ell^3 g(x), has
// b^der(k) = sum_q B1'(|k_q|) prod_{p != q} B1(|k_p|) / N^d -- the same
// coefficients as the transform of all d axes.  Block `blk` of `nblk` (256
// threads) of array `arr` (0 kernel, 1 derivative) of window `w` builds the
// 1-D transforms in LDS (lds: 4 kCoefMaxH + 256 doubles), fills its 256
// entries of D(k) = 1/2 (b(k) + b(-k)) / C(k)^2 on [-N/2, N/2]^d and writes
// its minimum of b to part[(w * 2 + arr) * nblk + blk].
template <typename T>
__device__ __forceinline__ void coef_sep_block(int d, int N, const CoefParams &prm, const double *cinv2,
                                               const double *cwg, const WinDesc *wd, double *part,
                                               int blk, int nblk, int arr, int w, double *lds)
{
    double *g1 = lds, *gd1 = lds + kCoefMaxH, *B1 = lds + 2 * kCoefMaxH, *Bd1 = lds + 3 * kCoefMaxH;
    double *red = lds + 4 * kCoefMaxH;
    const int H = N / 2 + 1;
    const float invN1 = 1.0f / (float)(N + 1);
    const double ell = prm.ell[w], cs = prm.c[w];
    for (int l = threadIdx.x; l < H; l += 256) {
        const double x = (double)l / (double)N / cs;
        const double v = exp(-(x * x) / (2.0 * ell * ell));
        g1[l] = v;
        gd1[l] = (x * x) / (ell * ell * ell) * v;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < H; k += 256) {
        double a = 0.0, ad = 0.0;
        for (int l = 0; l < H; ++l) {
            const double c = cwg[l * H + k];
            a += c * g1[l];
            ad += c * gd1[l];
        }
        B1[k] = a / (double)N;
        Bd1[k] = ad / (double)N;
    }
    __syncthreads();
    int KD = 1;
    for (int q = 0; q < d; ++q) KD *= N + 1;
    const int i = blk * 256 + threadIdx.x;
    double b = INFINITY;
    if (i < KD) {
        int rem = i;
        bool in_pos = true, in_neg = true;
        double f = 1.0, prod = 1.0, dsum = 0.0;
        for (int q = d - 1; q >= 0; --q) {
            const int qt = fdiv_small(rem, N + 1, invN1);
            const int k = rem - qt * (N + 1) - N / 2;
            rem = qt;
            in_pos = in_pos && k < N / 2;
            in_neg = in_neg && k > -N / 2;
            const int ka = k < 0 ? -k : k;
            // derivative: product rule over the factors taken so far
            dsum = dsum * B1[ka] + prod * Bd1[ka];
            prod *= B1[ka];
            f *= cinv2[k + N / 2];
        }
        b = arr == 0 ? prod : dsum;
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
    if (threadIdx.x == 0) part[((int64_t)w * 2 + arr) * nblk + blk] = red[0];
}

}  // namespace nfftgp
