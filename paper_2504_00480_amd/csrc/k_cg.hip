// Conjugate gradients on the regularised additive kernel matrix (Sec. 1: CG
// approximates Khat^-1 Y and, through its coefficients, the Lanczos matrices
// of stochastic Lanczos quadrature).  Vectors are in the plan precision; every
// dot product, step length and residual norm is accumulated in FP64.  Dot
// products reduce in a fixed order (per-block partials, then one block), so
// repeated runs give identical results.
#include "nfftgp_impl.h"

namespace nfftgp {
namespace {

template <typename T>
__global__ void __launch_bounds__(256)
k_dot_part(const T *__restrict__ A, int64_t lda, const T *__restrict__ B, int64_t ldb, int64_t n,
           double *__restrict__ part)
{
    __shared__ double s[256];
    const int c = blockIdx.y;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        acc += (double)A[i * lda + c] * (double)B[i * ldb + c];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)c * gridDim.x + blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(128)
k_dot_final(const double *__restrict__ part, int nblk, double *__restrict__ out)
{
    __shared__ double s[128];
    const int c = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 128) acc += part[(int64_t)c * nblk + b];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 64; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = s[0];
}

template <typename T>
__global__ void k_cg_init(int64_t total, const T *__restrict__ B, T *__restrict__ X,
                          T *__restrict__ R, T *__restrict__ P)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    T b = B[i];
    X[i] = T(0);
    R[i] = b;
    P[i] = b;
}

__global__ void k_cg_start(int nrhs, double *__restrict__ sc)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nrhs) return;
    double rr = sc[kRR * nrhs + c];
    sc[kRR0 * nrhs + c] = rr;
    sc[kActive * nrhs + c] = rr > 0.0 ? 1.0 : 0.0;
    sc[kIters * nrhs + c] = 0.0;
    sc[kNotPD * nrhs + c] = 0.0;
    sc[kAlpha * nrhs + c] = 0.0;
    sc[kBeta * nrhs + c] = 0.0;
    sc[kStep * nrhs + c] = -1.0;   // advanced at the start of every iteration
}

// x += alpha p, r -= alpha Khat p over the flat n x nrhs array (coalesced);
// used with a separate pass for the r^T r partials when nrhs > 2.
template <typename T>
__global__ void k_cg_xr(int64_t total, int nrhs, const double *__restrict__ sc, T *__restrict__ X,
                        T *__restrict__ R, const T *__restrict__ P, const T *__restrict__ AP)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int c = (int)(i % nrhs);
    const double a = sc[kAlpha * nrhs + c];
    if (a == 0.0) return;
    X[i] = (T)((double)X[i] + a * (double)P[i]);
    R[i] = (T)((double)R[i] - a * (double)AP[i]);
}

template <typename T>
__global__ void k_cg_p(int64_t total, int nrhs, const double *__restrict__ sc,
                       const T *__restrict__ R, T *__restrict__ P)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int c = (int)(i % nrhs);
    if (sc[kActive * nrhs + c] == 0.0) {
        P[i] = T(0);
        return;
    }
    P[i] = (T)((double)R[i] + sc[kBeta * nrhs + c] * (double)P[i]);
}

// ---- fused forms of the iteration (five launches besides the apply)

// Column c = blockIdx.x: p^T Khat p from the partials (the reduction of
// k_dot_final), then alpha as k_cg_alpha.  Block 0 also advances the
// iteration index (no other kernel of this launch reads it).
__global__ void __launch_bounds__(128)
k_dot_final_alpha(const double *__restrict__ part, int nblk, int nrhs, double *__restrict__ sc)
{
    __shared__ double s[128];
    const int c = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 128) acc += part[(int64_t)c * nblk + b];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 64; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double pap = s[0];
        sc[kPAP * nrhs + c] = pap;
        double alpha = 0.0;
        if (sc[kActive * nrhs + c] != 0.0) {
            if (!(pap > 0.0)) {
                sc[kNotPD * nrhs + c] = 1.0;
                sc[kActive * nrhs + c] = 0.0;
            } else {
                alpha = sc[kRR * nrhs + c] / pap;
            }
        }
        sc[kAlpha * nrhs + c] = alpha;
        if (c == 0) sc[kStep * nrhs] += 1.0;
    }
}

// x += alpha p, r -= alpha Khat p for column blockIdx.y (as k_cg_xr), and the
// partials of the new r^T r (the loop and reduction of k_dot_part).
template <typename T>
__global__ void __launch_bounds__(256)
k_cg_xr_dot(int64_t n, int nrhs, const double *__restrict__ sc, T *__restrict__ X, T *__restrict__ R,
            const T *__restrict__ P, const T *__restrict__ AP, double *__restrict__ part)
{
    __shared__ double s[256];
    const int c = blockIdx.y;
    const double a = sc[kAlpha * nrhs + c];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int64_t e = i * nrhs + c;
        T r = R[e];
        if (a != 0.0) {
            X[e] = (T)((double)X[e] + a * (double)P[e]);
            r = (T)((double)r - a * (double)AP[e]);
            R[e] = r;
        }
        acc += (double)r * (double)r;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)c * gridDim.x + blockIdx.x] = s[0];
}

// Column c = blockIdx.x: the new r^T r from the partials, then beta, the
// convergence test and the Lanczos history entry (as k_cg_beta).
__global__ void __launch_bounds__(128)
k_dot_final_beta(const double *__restrict__ part, int nblk, int nrhs, double *__restrict__ sc, double tol,
                 double *__restrict__ hist)
{
    __shared__ double s[128];
    const int c = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 128) acc += part[(int64_t)c * nblk + b];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 64; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int it = (int)sc[kStep * nrhs];
        const double rrn = s[0];
        sc[kRRNew * nrhs + c] = rrn;
        double beta = 0.0;
        if (sc[kActive * nrhs + c] != 0.0) {
            const double rr = sc[kRR * nrhs + c];
            beta = rrn / rr;
            if (hist) {
                hist[((int64_t)it * nrhs + c) * 2] = sc[kAlpha * nrhs + c];
                hist[((int64_t)it * nrhs + c) * 2 + 1] = beta;
            }
            sc[kRR * nrhs + c] = rrn;
            sc[kIters * nrhs + c] = (double)(it + 1);
            if (sqrt(rrn) <= tol * sqrt(sc[kRR0 * nrhs + c])) sc[kActive * nrhs + c] = 0.0;
        }
        sc[kBeta * nrhs + c] = beta;
    }
}

inline unsigned blocks(int64_t total) { return (unsigned)((total + 255) / 256); }

}  // namespace

hipError_t launch_coldots(int prec, const void *A, int64_t lda, const void *B, int64_t ldb,
                          int64_t n, int ncol, double *part, double *out, hipStream_t s)
{
    dim3 g(kDotBlocks, (unsigned)ncol);
    if (prec == NFFTGP_F32)
        k_dot_part<float><<<g, 256, 0, s>>>((const float *)A, lda, (const float *)B, ldb, n, part);
    else
        k_dot_part<double><<<g, 256, 0, s>>>((const double *)A, lda, (const double *)B, ldb, n, part);
    k_dot_final<<<(unsigned)ncol, 128, 0, s>>>(part, kDotBlocks, out);
    return hipGetLastError();
}

hipError_t launch_dot_part(int prec, const void *A, int64_t lda, const void *B, int64_t ldb, int64_t n,
                           int ncol, double *part, hipStream_t s)
{
    dim3 g(kDotBlocks, (unsigned)ncol);
    if (prec == NFFTGP_F32)
        k_dot_part<float><<<g, 256, 0, s>>>((const float *)A, lda, (const float *)B, ldb, n, part);
    else
        k_dot_part<double><<<g, 256, 0, s>>>((const double *)A, lda, (const double *)B, ldb, n, part);
    return hipGetLastError();
}

hipError_t launch_cg_init(int prec, int64_t n, int nrhs, const void *B, void *X, void *R, void *Pv,
                          hipStream_t s)
{
    int64_t tot = n * nrhs;
    if (tot == 0) return hipSuccess;
    if (prec == NFFTGP_F32)
        k_cg_init<float><<<blocks(tot), 256, 0, s>>>(tot, (const float *)B, (float *)X, (float *)R,
                                                      (float *)Pv);
    else
        k_cg_init<double><<<blocks(tot), 256, 0, s>>>(tot, (const double *)B, (double *)X,
                                                       (double *)R, (double *)Pv);
    return hipGetLastError();
}

hipError_t launch_cg_start(int nrhs, double *scal, hipStream_t s)
{
    k_cg_start<<<1, 64, 0, s>>>(nrhs, scal);
    return hipGetLastError();
}

hipError_t launch_cg_alpha(int nrhs, const double *part, double *scal, hipStream_t s)
{
    k_dot_final_alpha<<<(unsigned)nrhs, 128, 0, s>>>(part, kDotBlocks, nrhs, scal);
    return hipGetLastError();
}

hipError_t launch_cg_xr(int prec, int64_t n, int nrhs, const double *scal, void *X, void *R,
                        const void *Pv, const void *AP, double *part, hipStream_t s)
{
    if (n * nrhs == 0) return hipSuccess;
    if (nrhs > 2) {
        // column-strided updates would waste the coalescing of the flat form:
        // flat update, then the partials as a separate pass (same values)
        const int64_t tot = n * nrhs;
        if (prec == NFFTGP_F32)
            k_cg_xr<float><<<blocks(tot), 256, 0, s>>>(tot, nrhs, scal, (float *)X, (float *)R,
                                                        (const float *)Pv, (const float *)AP);
        else
            k_cg_xr<double><<<blocks(tot), 256, 0, s>>>(tot, nrhs, scal, (double *)X, (double *)R,
                                                         (const double *)Pv, (const double *)AP);
        return launch_dot_part(prec, R, nrhs, R, nrhs, n, nrhs, part, s);
    }
    const dim3 g(kDotBlocks, (unsigned)nrhs);
    if (prec == NFFTGP_F32)
        k_cg_xr_dot<float><<<g, 256, 0, s>>>(n, nrhs, scal, (float *)X, (float *)R, (const float *)Pv,
                                              (const float *)AP, part);
    else
        k_cg_xr_dot<double><<<g, 256, 0, s>>>(n, nrhs, scal, (double *)X, (double *)R, (const double *)Pv,
                                               (const double *)AP, part);
    return hipGetLastError();
}

hipError_t launch_cg_beta(int nrhs, const double *part, double *scal, double tol, double *hist, hipStream_t s)
{
    k_dot_final_beta<<<(unsigned)nrhs, 128, 0, s>>>(part, kDotBlocks, nrhs, scal, tol, hist);
    return hipGetLastError();
}

hipError_t launch_cg_p(int prec, int64_t n, int nrhs, const double *scal, const void *R, void *Pv,
                       hipStream_t s)
{
    int64_t tot = n * nrhs;
    if (tot == 0) return hipSuccess;
    if (prec == NFFTGP_F32)
        k_cg_p<float><<<blocks(tot), 256, 0, s>>>(tot, nrhs, scal, (const float *)R, (float *)Pv);
    else
        k_cg_p<double><<<blocks(tot), 256, 0, s>>>(tot, nrhs, scal, (const double *)R,
                                                    (double *)Pv);
    return hipGetLastError();
}

}  // namespace nfftgp
