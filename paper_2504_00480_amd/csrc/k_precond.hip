// Additive AFN preconditioner (Sec. 2.3): landmarks by farthest point
// sampling per feature window, merged into the (1,1) block of the
// regularised kernel matrix; Cholesky factor of that block; the Schur
// complement of the other points replaced by its diagonal blocks over runs
// of at most f spatially close points (a factorised approximate inverse with
// the pattern "lower triangle of the block").  With the landmarks first,
//
//   M = [[K11, K12], [K21, K21 K11^-1 K12 + blockdiag(S_BB)]] = F F^T,
//   F = [[L11, 0], [V, blockdiag(L_B)]],  V = K21 L11^-T,
//   S_BB = Khat_BB - V_B V_B^T = L_B L_B^T.
//
// Kernel entries are those of the exact kernel (caller units), computed in
// FP64 from a copy of the window features.  Everything here is FP64; the
// vectors the application kernels read and write have the plan precision.
#include <cmath>

#include "nfftgp_dev.h"
#include "nfftgp_impl.h"

namespace nfftgp {
namespace {

constexpr int kWG = 256;

// Exact regularised additive kernel between two points (rows of the feature
// copy) and its derivatives: v[0] = Khat_ij, v[1 + j] = dKhat_ij / dtheta_j,
// theta = (sigma_f, ell_1..ell_P, sigma_eps) (Sec. 1, eq. kernel_definition;
// Sec. 2.1, eq. def_der_additive_kernels).  `same` marks the diagonal.
template <bool DER>
__device__ __forceinline__ void pc_pair(const double *__restrict__ xi, const double *__restrict__ xj,
                                        bool same, const PcKer &kp, double *v)
{
    double ks = 0.0;
#pragma unroll
    for (int s = 0; s < kPcMaxWin; ++s) {
        if (s >= kp.P) continue;
        const int o = kp.off[s];
        double r2 = 0.0;
        for (int q = 0; q < kp.d[s]; ++q) {
            const double df = xi[o + q] - xj[o + q];
            r2 += df * df;
        }
        const double l = kp.ell[s];
        double e, de;
        if (kp.type[s] == NFFTGP_GAUSS) {
            e = exp(-r2 / (2.0 * l * l));
            de = r2 / (l * l * l) * e;
        } else if (kp.type[s] == NFFTGP_MATERN32) {
            const double r = sqrt(r2), a = 1.7320508075688772 * r / l, ea = exp(-a);
            e = (1.0 + a) * ea;
            de = 3.0 * r2 / (l * l * l) * ea;
        } else if (kp.type[s] == NFFTGP_SINC) {
            const double r = sqrt(r2), x = l * r;
            e = fabs(x) < 1e-4 ? l * (1.0 - x * x / 6.0) : sin(x) / r;
            de = cos(x);
        } else if (kp.type[s] == NFFTGP_MQ || kp.type[s] == NFFTGP_IMQ) {
            const double q = sqrt(r2 + l * l);
            e = kp.type[s] == NFFTGP_MQ ? q : 1.0 / q;
            de = kp.type[s] == NFFTGP_MQ ? l / q : -l / (q * q * q);
        } else {
            const double r = sqrt(r2);
            e = exp(-r / l);
            de = r / (l * l) * e;
        }
        ks += e;
        if (DER) v[2 + s] = kp.sf * kp.sf * de;
    }
    v[0] = kp.sf * kp.sf * ks + (same ? kp.se * kp.se : 0.0);
    if (DER) {
        v[1] = 2.0 * kp.sf * ks;
#pragma unroll
        for (int s = 0; s <= kPcMaxWin; ++s)
            if (s == kp.P) v[2 + s] = same ? 2.0 * kp.se : 0.0;
    }
}

// Work-group sums of the first np2 entries of acc (compile-time indices),
// written to out[0 .. np2) by thread 0.
__device__ __forceinline__ void wg_sums(const double (&acc)[kPcMaxWin + 2], int np2, double *red, double *out)
{
#pragma unroll
    for (int j = 0; j < kPcMaxWin + 2; ++j) {
        if (j >= np2) continue;
        red[threadIdx.x] = acc[j];
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[j] = red[0];
        __syncthreads();
    }
}

// Sum over the 256 threads of a work-group (tree in LDS, fixed order).
__device__ double wg_sum(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = kWG / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- attach time
// FP64 copy of the window features: Xw[i][q] = X[i][feat[q]].
template <typename T>
__global__ void k_pc_gather(const T *__restrict__ X, int64_t ldx, int64_t n, int ptot, const int *__restrict__ feat,
                            double *__restrict__ Xw)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * ptot) return;
    const int64_t i = e / ptot;
    const int q = (int)(e % ptot);
    Xw[e] = (double)X[i * ldx + feat[q]];
}

// Farthest point sampling in window s (one work-group per window): the
// first point is the one farthest from the window centre, every further one
// maximises the distance to the points chosen so far; ties go to the
// smallest index.  Squared distances are sums over the window's features in
// order, each term a rounded product then a rounded sum (as the oracle
// evaluates them), so both sides take the same decisions.
__global__ void __launch_bounds__(1024)
k_pc_fps(const double *__restrict__ X, int64_t n, int ptot, PcKer kp, const double *__restrict__ centre,
         int kw, double *__restrict__ mind_all, int *__restrict__ sel)
{
    __shared__ double bv[1024];
    __shared__ int bi[1024];
    __shared__ int cur;
    const int s = blockIdx.x;
    const int o = kp.off[s], d = kp.d[s];
    double *mind = mind_all + (int64_t)s * n;
    const double *ref = centre + o;   // first pass: distances to the centre
    for (int t = 0; t < kw; ++t) {
        double best = -1.0;
        int bidx = 0x7fffffff;
        for (int64_t i = threadIdx.x; i < n; i += 1024) {
            const double *xi = X + i * ptot + o;
            double r2 = 0.0;
            for (int q = 0; q < d; ++q) {
                const double df = __dsub_rn(xi[q], ref[q]);
                r2 = __dadd_rn(r2, __dmul_rn(df, df));
            }
            double m = r2;   // t = 0: distance to the centre
            if (t > 0) {
                m = t == 1 ? r2 : fmin(mind[i], r2);
                mind[i] = m;
            }
            if (m > best) {   // indices rise within a thread: the first maximum is kept
                best = m;
                bidx = (int)i;
            }
        }
        bv[threadIdx.x] = best;
        bi[threadIdx.x] = bidx;
        __syncthreads();
        for (int w = 512; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) {
                const double a = bv[threadIdx.x], b = bv[threadIdx.x + w];
                const int ia = bi[threadIdx.x], ib = bi[threadIdx.x + w];
                if (b > a || (b == a && ib < ia)) {
                    bv[threadIdx.x] = b;
                    bi[threadIdx.x] = ib;
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            // every remaining point coincides with a chosen one: stop
            cur = (t > 0 && !(bv[0] > 0.0)) ? -1 : bi[0];
            sel[s * kw + t] = cur;
        }
        __syncthreads();
        if (cur < 0) {
            for (int u = t + 1 + (int)threadIdx.x; u < kw; u += 1024) sel[s * kw + u] = -1;
            return;
        }
        ref = X + (int64_t)cur * ptot + o;
        __syncthreads();
    }
}

// Window-0 cell order keys of the points (FP64, t = 2N c (x - c0) + N,
// cells by tile then inside the tile, row-major).
__global__ void k_pc_keys(const double *__restrict__ X, int64_t n, int ptot, int d, int N, int tb,
                          double c, const double *__restrict__ c0, int64_t *__restrict__ key)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ng = 2 * N, nb = ng / tb;
    int64_t tile = 0, loc = 0, tbd = 1;
    for (int q = 0; q < d; ++q) {
        const double t = __dadd_rn(__dmul_rn(__dmul_rn(c, __dsub_rn(X[i * ptot + q], c0[q])), (double)ng), (double)N);
        int64_t cell = (int64_t)floor(t);
        cell = cell < 0 ? 0 : (cell > ng - 1 ? ng - 1 : cell);
        tile = tile * nb + cell / tb;
        loc = loc * tb + cell % tb;
        tbd *= tb;
    }
    key[i] = tile * tbd + loc;
}

// ---------------------------------------------------------------- per theta
// Landmark block K11 and its derivatives.
__global__ void k_pc_k11(const double *__restrict__ X, int ptot, const int *__restrict__ lm, int k, PcKer kp,
                         double *__restrict__ K11, double *__restrict__ dK11)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)k * k) return;
    const int a = (int)(e / k), b = (int)(e % k);
    double v[kPcMaxWin + 3];
    pc_pair<true>(X + (int64_t)lm[a] * ptot, X + (int64_t)lm[b] * ptot, a == b, kp, v);
    K11[e] = v[0];
#pragma unroll
    for (int j = 0; j < kPcMaxWin + 2; ++j)
        if (j < kp.P + 2) dK11[(int64_t)j * k * k + e] = v[1 + j];
}

// One work-group: L11 (Cholesky of K11, right-looking, in place in L),
// L11^-1 (columns by forward substitution) and K11^-1 = L11^-T L11^-1, and
// log det K11 into acc[0].  flag[0] is set when a pivot is not positive.
__global__ void __launch_bounds__(1024)
k_pc_chol11(const double *__restrict__ K11, int k, double *__restrict__ L, double *__restrict__ Li,
            double *__restrict__ Ki, double *__restrict__ acc, int *__restrict__ flag)
{
    __shared__ double piv;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int64_t e = tid; e < (int64_t)k * k; e += nt) L[e] = K11[e];
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        if (tid == 0) {
            const double dj = L[(int64_t)j * k + j];
            if (!(dj > 0.0)) flag[0] = 1;
            piv = dj > 0.0 ? sqrt(dj) : 1.0;
            L[(int64_t)j * k + j] = piv;
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < k; i += nt) L[(int64_t)i * k + j] /= piv;
        __syncthreads();
        const int m = k - j - 1;
        for (int64_t e = tid; e < (int64_t)m * m; e += nt) {
            const int i = j + 1 + (int)(e / m), l = j + 1 + (int)(e % m);
            if (l <= i) L[(int64_t)i * k + l] -= L[(int64_t)i * k + j] * L[(int64_t)l * k + j];
        }
        __syncthreads();
    }
    for (int64_t e = tid; e < (int64_t)k * k; e += nt) {
        const int i = (int)(e / k), l = (int)(e % k);
        if (l > i) L[e] = 0.0;
    }
    __syncthreads();
    // L^-1, one column per thread
    for (int c = tid; c < k; c += nt) {
        for (int i = 0; i < k; ++i) {
            double x = 0.0;
            if (i >= c) {
                double acc = i == c ? 1.0 : 0.0;
                for (int l = c; l < i; ++l) acc -= L[(int64_t)i * k + l] * Li[(int64_t)l * k + c];
                x = acc / L[(int64_t)i * k + i];
            }
            Li[(int64_t)i * k + c] = x;
        }
    }
    __syncthreads();
    for (int64_t e = tid; e < (int64_t)k * k; e += nt) {
        const int a = (int)(e / k), b = (int)(e % k);
        double s = 0.0;
        for (int m2 = (a > b ? a : b); m2 < k; ++m2) s += Li[(int64_t)m2 * k + a] * Li[(int64_t)m2 * k + b];
        Ki[e] = s;
    }
    if (tid == 0) {
        double ld = 0.0;
        for (int j = 0; j < k; ++j) ld += log(L[(int64_t)j * k + j]);
        acc[0] = 2.0 * ld;
    }
}

// V rows: V[i] = L11^-1 Khat(x_ord[i], x_lm), 16 points per work-group.
constexpr int kVP = 16;
__global__ void __launch_bounds__(256)
k_pc_v(const double *__restrict__ X, int ptot, const int *__restrict__ lm, int k, const int *__restrict__ ord,
       int64_t np, PcKer kp, const double *__restrict__ Li, double *__restrict__ V)
{
    extern __shared__ double cs[];   // kVP x k kernel values
    const int64_t p0 = (int64_t)blockIdx.x * kVP;
    const int npt = (int)(np - p0 < kVP ? np - p0 : kVP);
    for (int e = threadIdx.x; e < npt * k; e += 256) {
        const int p = e / k, a = e % k;
        double v[kPcMaxWin + 3];
        pc_pair<false>(X + (int64_t)ord[p0 + p] * ptot, X + (int64_t)lm[a] * ptot, false, kp, v);
        cs[e] = v[0];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < npt * k; e += 256) {
        const int p = e / k, a = e % k;
        double s = 0.0;
        for (int b = 0; b <= a; ++b) s += Li[(int64_t)a * k + b] * cs[p * k + b];
        V[(p0 + p) * k + a] = s;
    }
}

// One work-group per Schur-complement block: S = Khat_BB - V_B V_B^T in LDS,
// its Cholesky factor L_B and L_B^-1 (global), Y_B = L_B^-1 V_B,
// W_B = L_B^-T Y_B (= S^-1 V_B) and G_B = -2 W_B L11^-1, then this block's
// share of tr(M^-1 dM/dtheta_j):
//   sum_{i in B} G_B[i] . dKhat(x_i, x_lm)/dtheta_j + <S^-1, dKhat_BB/dtheta_j>,
// and 2 log det L_B, into part[b * (P + 3) + ...].
__global__ void __launch_bounds__(256)
k_pc_block(const double *__restrict__ X, int ptot, const int *__restrict__ lm, int k,
           const int *__restrict__ ord, int64_t np, int f, PcKer kp, const double *__restrict__ V,
           const double *__restrict__ Li, double *__restrict__ LB, double *__restrict__ LBi,
           double *__restrict__ Y, double *__restrict__ Wt, double *__restrict__ G,
           double *__restrict__ part, int *__restrict__ flag)
{
    extern __shared__ double S[];   // f x f
    __shared__ double red[kWG];
    __shared__ double piv;
    const int b = blockIdx.x, tid = threadIdx.x;
    const int64_t base = (int64_t)b * f;
    const int nb = (int)(np - base < f ? np - base : f);
    double *Lb = LB + (int64_t)b * f * f;
    double *Lbi = LBi + (int64_t)b * f * f;
    const double *Vb = V + base * k;
    // S = Khat_BB - V_B V_B^T
    for (int e = tid; e < nb * nb; e += kWG) {
        const int i = e / nb, l = e % nb;
        double v[kPcMaxWin + 3];
        pc_pair<false>(X + (int64_t)ord[base + i] * ptot, X + (int64_t)ord[base + l] * ptot, i == l, kp, v);
        double s = v[0];
        for (int a = 0; a < k; ++a) s -= Vb[(int64_t)i * k + a] * Vb[(int64_t)l * k + a];
        S[i * f + l] = s;
    }
    __syncthreads();
    // Cholesky (lower, right-looking)
    for (int j = 0; j < nb; ++j) {
        if (tid == 0) {
            const double dj = S[j * f + j];
            if (!(dj > 0.0)) flag[0] = 1;
            piv = dj > 0.0 ? sqrt(dj) : 1.0;
            S[j * f + j] = piv;
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < nb; i += kWG) S[i * f + j] /= piv;
        __syncthreads();
        const int m = nb - j - 1;
        for (int e = tid; e < m * m; e += kWG) {
            const int i = j + 1 + e / m, l = j + 1 + e % m;
            if (l <= i) S[i * f + l] -= S[i * f + j] * S[l * f + j];
        }
        __syncthreads();
    }
    for (int e = tid; e < f * f; e += kWG) {
        const int i = e / f, l = e % f;
        Lb[e] = (i < nb && l <= i) ? S[i * f + l] : 0.0;
    }
    // L_B^-1, one column per thread
    for (int c = tid; c < nb; c += kWG) {
        for (int i = 0; i < nb; ++i) {
            double x = 0.0;
            if (i == c) {
                x = 1.0 / S[i * f + i];
            } else if (i > c) {
                double acc = 0.0;
                for (int l = c; l < i; ++l) acc += S[i * f + l] * Lbi[(int64_t)l * f + c];
                x = -acc / S[i * f + i];
            }
            Lbi[(int64_t)i * f + c] = x;
        }
    }
    for (int e = tid; e < f * f; e += kWG) {
        const int i = e / f, c = e % f;
        if (i >= nb || c >= nb) Lbi[e] = 0.0;
    }
    double ldpart = 0.0;
    for (int i = tid; i < nb; i += kWG) ldpart += log(S[i * f + i]);
    __threadfence_block();
    __syncthreads();
    const double logdet_b = 2.0 * wg_sum(ldpart, red);
    // Y_B = L_B^-1 V_B, W_B = L_B^-T Y_B, G_B = -2 W_B L11^-1
    double *Yb = Y + base * k;
    double *Wb = Wt + base * k;
    double *Gb = G + base * k;
    for (int e = tid; e < nb * k; e += kWG) {
        const int i = e / k, a = e % k;
        double s = 0.0;
        for (int l = 0; l <= i; ++l) s += Lbi[(int64_t)i * f + l] * Vb[(int64_t)l * k + a];
        Yb[e] = s;
    }
    __threadfence_block();
    __syncthreads();
    for (int e = tid; e < nb * k; e += kWG) {
        const int i = e / k, a = e % k;
        double s = 0.0;
        for (int l = i; l < nb; ++l) s += Lbi[(int64_t)l * f + i] * Yb[(int64_t)l * k + a];
        Wb[e] = s;
    }
    __threadfence_block();
    __syncthreads();
    for (int e = tid; e < nb * k; e += kWG) {
        const int i = e / k, a = e % k;
        double s = 0.0;
        for (int c = a; c < k; ++c) s += Wb[(int64_t)i * k + c] * Li[(int64_t)c * k + a];
        Gb[e] = -2.0 * s;
    }
    __threadfence_block();
    __syncthreads();
    // contraction with the derivative kernels
    const int np2 = kp.P + 2;
    double acc[kPcMaxWin + 2];
#pragma unroll
    for (int j = 0; j < kPcMaxWin + 2; ++j) acc[j] = 0.0;
    for (int e = tid; e < nb * k; e += kWG) {
        const int i = e / k, a = e % k;
        double v[kPcMaxWin + 3];
        pc_pair<true>(X + (int64_t)ord[base + i] * ptot, X + (int64_t)lm[a] * ptot, false, kp, v);
        const double g = Gb[e];
#pragma unroll
        for (int j = 0; j < kPcMaxWin + 2; ++j)
            if (j < np2) acc[j] += g * v[1 + j];
    }
    for (int e = tid; e < nb * nb; e += kWG) {
        const int i = e / nb, l = e % nb;
        // (S^-1)_il = sum_{m >= max(i, l)} (L_B^-1)_mi (L_B^-1)_ml
        double si = 0.0;
        for (int m2 = (i > l ? i : l); m2 < nb; ++m2) si += Lbi[(int64_t)m2 * f + i] * Lbi[(int64_t)m2 * f + l];
        double v[kPcMaxWin + 3];
        pc_pair<true>(X + (int64_t)ord[base + i] * ptot, X + (int64_t)ord[base + l] * ptot, i == l, kp, v);
#pragma unroll
        for (int j = 0; j < kPcMaxWin + 2; ++j)
            if (j < np2) acc[j] += si * v[1 + j];
    }
    double *pb = part + (int64_t)b * (np2 + 1);
    wg_sums(acc, np2, red, pb + 1);
    if (tid == 0) pb[0] = logdet_b;
}

// Z = Y^T Y over all non-landmark rows: partial sums over chunks of rows,
// one work-group per chunk (upper triangle a <= c).
__global__ void __launch_bounds__(256)
k_pc_z(const double *__restrict__ Y, int64_t np, int k, int64_t rows, double *__restrict__ zpart)
{
    const int64_t r0 = (int64_t)blockIdx.x * rows;
    const int64_t r1 = r0 + rows < np ? r0 + rows : np;
    double *zp = zpart + (int64_t)blockIdx.x * k * k;
    for (int64_t e = threadIdx.x; e < (int64_t)k * k; e += 256) {
        const int a = (int)(e / k), c = (int)(e % k);
        if (c < a) continue;
        double s = 0.0;
        for (int64_t r = r0; r < r1; ++r) s += Y[r * k + a] * Y[r * k + c];
        zp[e] = s;
    }
}

// One work-group: Z from its partials, Gk = K11^-1 + L11^-T Z L11^-1, the
// traces <Gk, dK11/dtheta_j>, the blocks' shares, and the results:
// out[0] = log det M, out[1 + j] = tr(M^-1 dM/dtheta_j).
__global__ void __launch_bounds__(1024)
k_pc_final(const double *__restrict__ zpart, int nz, int k, const double *__restrict__ Li,
           const double *__restrict__ Ki, const double *__restrict__ dK11, const double *__restrict__ part,
           int nblk, int np2, const double *__restrict__ acc, double *__restrict__ Z, double *__restrict__ T,
           double *__restrict__ out)
{
    __shared__ double red[1024];
    const int tid = threadIdx.x;
    for (int64_t e = tid; e < (int64_t)k * k; e += 1024) {
        const int a = (int)(e / k), c = (int)(e % k);
        const int64_t u = a <= c ? (int64_t)a * k + c : (int64_t)c * k + a;
        double s = 0.0;
        for (int z = 0; z < nz; ++z) s += zpart[(int64_t)z * k * k + u];
        Z[e] = s;
    }
    __syncthreads();
    // T = Z L11^-1
    for (int64_t e = tid; e < (int64_t)k * k; e += 1024) {
        const int a = (int)(e / k), c = (int)(e % k);
        double s = 0.0;
        for (int m2 = c; m2 < k; ++m2) s += Z[(int64_t)a * k + m2] * Li[(int64_t)m2 * k + c];
        T[e] = s;
    }
    __syncthreads();
    // Gk = K11^-1 + L11^-T T, stored in Z
    for (int64_t e = tid; e < (int64_t)k * k; e += 1024) {
        const int a = (int)(e / k), c = (int)(e % k);
        double s = Ki[e];
        for (int m2 = a; m2 < k; ++m2) s += Li[(int64_t)m2 * k + a] * T[(int64_t)m2 * k + c];
        Z[e] = s;
    }
    __syncthreads();
    for (int j = 0; j < np2; ++j) {
        double s = 0.0;
        for (int64_t e = tid; e < (int64_t)k * k; e += 1024) s += Z[e] * dK11[(int64_t)j * k * k + e];
        red[tid] = s;
        __syncthreads();
        for (int o = 512; o > 0; o >>= 1) {
            if (tid < o) red[tid] += red[tid + o];
            __syncthreads();
        }
        if (tid == 0) {
            double t = red[0];
            for (int b = 0; b < nblk; ++b) t += part[(int64_t)b * (np2 + 1) + 1 + j];
            out[1 + j] = t;
        }
        __syncthreads();
    }
    if (tid == 0) {
        double ld = acc[0];
        for (int b = 0; b < nblk; ++b) ld += part[(int64_t)b * (np2 + 1)];
        out[0] = ld;
    }
}

// ---------------------------------------------------------------- application
// Landmark part before the blocks, one work-group per vector c:
//   MINV: T1 = L11^-1 v1;  FINVT, FAC: T1 = v1 (and FAC writes L11 v1 to out).
template <typename T>
__global__ void __launch_bounds__(256)
k_pc_lm_pre(int op, const T *__restrict__ v, int nrhs, const int *__restrict__ lm, int k,
            const double *__restrict__ L, const double *__restrict__ Li, double *__restrict__ T1,
            T *__restrict__ out)
{
    const int c = blockIdx.x;
    for (int a = threadIdx.x; a < k; a += 256) {
        if (op == kPcMinv) {
            double s = 0.0;
            for (int b = 0; b <= a; ++b) s += Li[(int64_t)a * k + b] * (double)v[(int64_t)lm[b] * nrhs + c];
            T1[(int64_t)c * k + a] = s;
        } else {
            T1[(int64_t)c * k + a] = (double)v[(int64_t)lm[a] * nrhs + c];
            if (op == kPcFac) {
                double s = 0.0;
                for (int b = 0; b <= a; ++b) s += L[(int64_t)a * k + b] * (double)v[(int64_t)lm[b] * nrhs + c];
                out[(int64_t)lm[a] * nrhs + c] = (T)s;
            }
        }
    }
}

// One work-group per (block b, vector c):
//   MINV:  u = v_B - V_B T1, t2 = L_B^-1 u, s2 = L_B^-T t2 -> out_B; Q_b = V_B^T s2
//   FINVT: s2 = L_B^-T v_B -> out_B; Q_b = V_B^T s2
//   FAC:   out_B = V_B T1 + L_B v_B
template <typename T>
__global__ void __launch_bounds__(256)
k_pc_blk(int op, const T *__restrict__ v, int nrhs, const int *__restrict__ ord, int64_t np, int f, int k,
         const double *__restrict__ V, const double *__restrict__ LB, const double *__restrict__ LBi,
         const double *__restrict__ T1, double *__restrict__ Q, T *__restrict__ out)
{
    extern __shared__ double sm[];
    double *u = sm;           // f
    double *t2 = sm + f;      // f
    const int b = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
    const int64_t base = (int64_t)b * f;
    const int nb = (int)(np - base < f ? np - base : f);
    const double *Vb = V + base * k;
    const double *Lb = LB + (int64_t)b * f * f;
    const double *Lbi = LBi + (int64_t)b * f * f;
    const double *t1 = T1 + (int64_t)c * k;
    for (int i = tid; i < nb; i += 256) {
        const double vi = (double)v[(int64_t)ord[base + i] * nrhs + c];
        if (op == kPcFac) {
            double s = 0.0;
            for (int a = 0; a < k; ++a) s += Vb[(int64_t)i * k + a] * t1[a];
            for (int l = 0; l <= i; ++l) s += Lb[(int64_t)i * f + l] * (double)v[(int64_t)ord[base + l] * nrhs + c];
            out[(int64_t)ord[base + i] * nrhs + c] = (T)s;
        } else if (op == kPcMinv) {
            double s = vi;
            for (int a = 0; a < k; ++a) s -= Vb[(int64_t)i * k + a] * t1[a];
            u[i] = s;
        } else {
            t2[i] = vi;
        }
    }
    if (op == kPcFac) return;
    __syncthreads();
    if (op == kPcMinv) {
        for (int i = tid; i < nb; i += 256) {
            double s = 0.0;
            for (int l = 0; l <= i; ++l) s += Lbi[(int64_t)i * f + l] * u[l];
            t2[i] = s;
        }
        __syncthreads();
    }
    for (int i = tid; i < nb; i += 256) {
        double s = 0.0;
        for (int l = i; l < nb; ++l) s += Lbi[(int64_t)l * f + i] * t2[l];
        u[i] = s;   // s2
    }
    __syncthreads();
    for (int i = tid; i < nb; i += 256) out[(int64_t)ord[base + i] * nrhs + c] = (T)u[i];
    for (int a = tid; a < k; a += 256) {
        double s = 0.0;
        for (int i = 0; i < nb; ++i) s += Vb[(int64_t)i * k + a] * u[i];
        Q[((int64_t)b * nrhs + c) * k + a] = s;
    }
}

// Landmark part after the blocks (MINV, FINVT), one work-group per vector:
//   s1 = L11^-T (T1 - sum_b Q_b) -> out at the landmarks.
template <typename T>
__global__ void __launch_bounds__(256)
k_pc_lm_post(const double *__restrict__ Q, int nblk, int nrhs, const int *__restrict__ lm, int k,
             const double *__restrict__ Li, const double *__restrict__ T1, double *__restrict__ R,
             T *__restrict__ out)
{
    const int c = blockIdx.x;
    double *r = R + (int64_t)c * k;
    for (int a = threadIdx.x; a < k; a += 256) {
        double s = T1[(int64_t)c * k + a];
        for (int b = 0; b < nblk; ++b) s -= Q[((int64_t)b * nrhs + c) * k + a];
        r[a] = s;
    }
    __syncthreads();
    for (int a = threadIdx.x; a < k; a += 256) {
        double s = 0.0;
        for (int m2 = a; m2 < k; ++m2) s += Li[(int64_t)m2 * k + a] * r[m2];
        out[(int64_t)lm[a] * nrhs + c] = (T)s;
    }
}

// ---------------------------------------------------------------- w^T dM w
// nu_B = V_B^T w_B per (block, vector), into Q.
template <typename T>
__global__ void __launch_bounds__(256)
k_pc_nu(const T *__restrict__ w, int nrhs, const int *__restrict__ ord, int64_t np, int f, int k,
        const double *__restrict__ V, double *__restrict__ Q)
{
    const int b = blockIdx.x, c = blockIdx.y;
    const int64_t base = (int64_t)b * f;
    const int nb = (int)(np - base < f ? np - base : f);
    const double *Vb = V + base * k;
    for (int a = threadIdx.x; a < k; a += 256) {
        double s = 0.0;
        for (int i = 0; i < nb; ++i) s += Vb[(int64_t)i * k + a] * (double)w[(int64_t)ord[base + i] * nrhs + c];
        Q[((int64_t)b * nrhs + c) * k + a] = s;
    }
}

// Per vector: abar = L11^-T sum_b nu_b, w1 = w at the landmarks, and the
// landmark terms w1^T dK11_j w1 - abar^T dK11_j abar into lmt[c * np2 + j].
template <typename T>
__global__ void __launch_bounds__(256)
k_pc_dq_lm(const T *__restrict__ w, int nrhs, const double *__restrict__ Q, int nblk, const int *__restrict__ lm,
           int k, const double *__restrict__ Li, const double *__restrict__ dK11, int np2,
           double *__restrict__ ABAR, double *__restrict__ W1, double *__restrict__ NUS, double *__restrict__ lmt)
{
    __shared__ double red[kWG];
    const int c = blockIdx.x;
    double *ab = ABAR + (int64_t)c * k;
    double *w1 = W1 + (int64_t)c * k;
    double *nu = NUS + (int64_t)c * k;
    for (int a = threadIdx.x; a < k; a += 256) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += Q[((int64_t)b * nrhs + c) * k + a];
        nu[a] = s;
        w1[a] = (double)w[(int64_t)lm[a] * nrhs + c];
    }
    __syncthreads();
    for (int a = threadIdx.x; a < k; a += 256) {
        double s = 0.0;
        for (int m2 = a; m2 < k; ++m2) s += Li[(int64_t)m2 * k + a] * nu[m2];
        ab[a] = s;
    }
    __syncthreads();
    for (int j = 0; j < np2; ++j) {
        const double *D = dK11 + (int64_t)j * k * k;
        double s = 0.0;
        for (int64_t e = threadIdx.x; e < (int64_t)k * k; e += 256) {
            const int a = (int)(e / k), b2 = (int)(e % k);
            s += D[e] * (w1[a] * w1[b2] - ab[a] * ab[b2]);
        }
        const double t = wg_sum(s, red);
        if (threadIdx.x == 0) lmt[(int64_t)c * np2 + j] = t;
    }
}

// Per (block, vector): abar_B = L11^-T nu_B, h = w1 + abar - abar_B, and the
// block's share of w^T dM_j w:
//   abar_B^T dK11_j abar_B + sum_{i in B} 2 w_i h . dKhat(x_i, x_lm)/dtheta_j
//   + w_B^T dKhat_BB/dtheta_j w_B   -> dqp[(b * nrhs + c) * np2 + j].
template <typename T>
__global__ void __launch_bounds__(256)
k_pc_dq_blk(const T *__restrict__ w, int nrhs, const double *__restrict__ X, int ptot, const int *__restrict__ lm,
            int k, const int *__restrict__ ord, int64_t np, int f, PcKer kp, const double *__restrict__ Li,
            const double *__restrict__ dK11, const double *__restrict__ Q, const double *__restrict__ ABAR,
            const double *__restrict__ W1, double *__restrict__ dqp)
{
    extern __shared__ double sm[];
    double *abB = sm;        // k
    double *h = sm + k;      // k
    double *wb = sm + 2 * k; // f
    __shared__ double red[kWG];
    const int b = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
    const int64_t base = (int64_t)b * f;
    const int nb = (int)(np - base < f ? np - base : f);
    const int np2 = kp.P + 2;
    const double *nu = Q + ((int64_t)b * nrhs + c) * k;
    for (int a = tid; a < k; a += 256) {
        double s = 0.0;
        for (int m2 = a; m2 < k; ++m2) s += Li[(int64_t)m2 * k + a] * nu[m2];
        abB[a] = s;
    }
    for (int i = tid; i < nb; i += 256) wb[i] = (double)w[(int64_t)ord[base + i] * nrhs + c];
    __syncthreads();
    for (int a = tid; a < k; a += 256) h[a] = W1[(int64_t)c * k + a] + ABAR[(int64_t)c * k + a] - abB[a];
    __syncthreads();
    double acc[kPcMaxWin + 2];
#pragma unroll
    for (int j = 0; j < kPcMaxWin + 2; ++j) acc[j] = 0.0;
#pragma unroll
    for (int j = 0; j < kPcMaxWin + 2; ++j) {
        if (j >= np2) continue;
        const double *D = dK11 + (int64_t)j * k * k;
        double s = 0.0;
        for (int64_t e = tid; e < (int64_t)k * k; e += 256) s += abB[e / k] * D[e] * abB[e % k];
        acc[j] += s;
    }
    for (int e = tid; e < nb * k; e += 256) {
        const int i = e / k, a = e % k;
        double v[kPcMaxWin + 3];
        pc_pair<true>(X + (int64_t)ord[base + i] * ptot, X + (int64_t)lm[a] * ptot, false, kp, v);
        const double g = 2.0 * wb[i] * h[a];
#pragma unroll
        for (int j = 0; j < kPcMaxWin + 2; ++j)
            if (j < np2) acc[j] += g * v[1 + j];
    }
    for (int e = tid; e < nb * nb; e += 256) {
        const int i = e / nb, l = e % nb;
        double v[kPcMaxWin + 3];
        pc_pair<true>(X + (int64_t)ord[base + i] * ptot, X + (int64_t)ord[base + l] * ptot, i == l, kp, v);
        const double g = wb[i] * wb[l];
#pragma unroll
        for (int j = 0; j < kPcMaxWin + 2; ++j)
            if (j < np2) acc[j] += g * v[1 + j];
    }
    wg_sums(acc, np2, red, dqp + ((int64_t)b * nrhs + c) * np2);
}

// out[j * nrhs + c] = lmt[c][j] + sum_b dqp[b][c][j] (fixed order).
__global__ void k_pc_dq_final(const double *__restrict__ dqp, int nblk, int nrhs, int np2,
                              const double *__restrict__ lmt, double *__restrict__ out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nrhs * np2) return;
    const int c = e / np2, j = e % np2;
    double s = lmt[(int64_t)c * np2 + j];
    for (int b = 0; b < nblk; ++b) s += dqp[((int64_t)b * nrhs + c) * np2 + j];
    out[(int64_t)j * nrhs + c] = s;
}

// ---------------------------------------------------------------- PCG scalars
// Start of preconditioned CG: kRR0 = b^T b (held in kRRNew by the caller's
// dot launch), kRR = r^T z.
__global__ void k_pcg_start(int nrhs, double *__restrict__ sc)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nrhs) return;
    const double rr = sc[kRRNew * nrhs + c];
    sc[kRR0 * nrhs + c] = rr;
    sc[kActive * nrhs + c] = rr > 0.0 ? 1.0 : 0.0;
    sc[kIters * nrhs + c] = 0.0;
    sc[kNotPD * nrhs + c] = 0.0;
    sc[kAlpha * nrhs + c] = 0.0;
    sc[kBeta * nrhs + c] = 0.0;
    sc[kStep * nrhs + c] = -1.0;
}

// Column c: r^T r (convergence) and r^T z (beta) from their partials, the
// Lanczos history entry, and beta = (r^T z)_new / (r^T z)_old.
__global__ void __launch_bounds__(128)
k_pcg_beta(const double *__restrict__ prr, const double *__restrict__ prz, int nblk, int nrhs,
           double *__restrict__ sc, double tol, double *__restrict__ hist)
{
    __shared__ double s1[128], s2[128];
    const int c = blockIdx.x;
    double a1 = 0.0, a2 = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 128) {
        a1 += prr[(int64_t)c * nblk + b];
        a2 += prz[(int64_t)c * nblk + b];
    }
    s1[threadIdx.x] = a1;
    s2[threadIdx.x] = a2;
    __syncthreads();
    for (int o = 64; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s1[threadIdx.x] += s1[threadIdx.x + o];
            s2[threadIdx.x] += s2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int it = (int)sc[kStep * nrhs];
        const double rr = s1[0], rz = s2[0];
        sc[kRRNew * nrhs + c] = rr;
        double beta = 0.0;
        if (sc[kActive * nrhs + c] != 0.0) {
            beta = rz / sc[kRR * nrhs + c];
            if (hist) {
                hist[((int64_t)it * nrhs + c) * 2] = sc[kAlpha * nrhs + c];
                hist[((int64_t)it * nrhs + c) * 2 + 1] = beta;
            }
            sc[kRR * nrhs + c] = rz;
            sc[kIters * nrhs + c] = (double)(it + 1);
            if (sqrt(rr) <= tol * sqrt(sc[kRR0 * nrhs + c])) sc[kActive * nrhs + c] = 0.0;
        }
        sc[kBeta * nrhs + c] = beta;
    }
}

inline unsigned nblocks(int64_t total, int bs) { return (unsigned)((total + bs - 1) / bs); }

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_pc_gather(int prec, const void *X, int64_t ldx, int64_t n, int ptot, const int *feat, double *Xw,
                            hipStream_t s)
{
    const int64_t tot = n * ptot;
    if (tot == 0) return hipSuccess;
    if (prec == NFFTGP_F32)
        k_pc_gather<float><<<nblocks(tot, 256), 256, 0, s>>>((const float *)X, ldx, n, ptot, feat, Xw);
    else
        k_pc_gather<double><<<nblocks(tot, 256), 256, 0, s>>>((const double *)X, ldx, n, ptot, feat, Xw);
    return hipGetLastError();
}

hipError_t launch_pc_fps(const double *X, int64_t n, int ptot, const PcKer &kp, const double *centre, int kw,
                         double *mind, int *sel, hipStream_t s)
{
    k_pc_fps<<<(unsigned)kp.P, 1024, 0, s>>>(X, n, ptot, kp, centre, kw, mind, sel);
    return hipGetLastError();
}

hipError_t launch_pc_keys(const double *X, int64_t n, int ptot, int d, int N, int tb, double c, const double *c0,
                          int64_t *key, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    k_pc_keys<<<nblocks(n, 256), 256, 0, s>>>(X, n, ptot, d, N, tb, c, c0, key);
    return hipGetLastError();
}

hipError_t launch_pc_setup(const Precond &pc, const PcKer &kp, hipStream_t s)
{
    const int k = pc.k, np2 = kp.P + 2;
    k_pc_k11<<<nblocks((int64_t)k * k, 256), 256, 0, s>>>(pc.X, pc.ptot, pc.lm, k, kp, pc.K11, pc.dK11);
    k_pc_chol11<<<1, 1024, 0, s>>>(pc.K11, k, pc.L11, pc.L11inv, pc.K11inv, pc.acc, pc.flag);
    if (pc.np > 0) {
        k_pc_v<<<nblocks(pc.np, kVP), 256, (size_t)kVP * k * sizeof(double), s>>>(
            pc.X, pc.ptot, pc.lm, k, pc.ord, pc.np, kp, pc.L11inv, pc.V);
        const size_t shb = (size_t)pc.f * pc.f * sizeof(double);
        if (shb > 64 * 1024) {
            const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_pc_block),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shb);
            if (e != hipSuccess) return e;
        }
        k_pc_block<<<(unsigned)pc.nblk, kWG, shb, s>>>(
            pc.X, pc.ptot, pc.lm, k, pc.ord, pc.np, pc.f, kp, pc.V, pc.L11inv, pc.LB, pc.LBinv, pc.Y, pc.Wt,
            pc.G, pc.part, pc.flag);
        k_pc_z<<<(unsigned)pc.nzpart, 256, 0, s>>>(pc.Y, pc.np, k, pc.zrows, pc.zpart);
    }
    k_pc_final<<<1, 1024, 0, s>>>(pc.zpart, pc.np > 0 ? pc.nzpart : 0, k, pc.L11inv, pc.K11inv, pc.dK11, pc.part,
                                  pc.np > 0 ? pc.nblk : 0, np2, pc.acc, pc.Zk, pc.Tk, pc.out_dev);
    return hipGetLastError();
}

hipError_t launch_pc_apply(int prec, const Precond &pc, int op, const void *v, int nrhs, void *out, hipStream_t s)
{
    const int k = pc.k;
    const dim3 gb((unsigned)pc.nblk, (unsigned)nrhs);
    const size_t shb = (size_t)2 * pc.f * sizeof(double);
    if (prec == NFFTGP_F32) {
        const float *vi = (const float *)v;
        float *o = (float *)out;
        k_pc_lm_pre<float><<<(unsigned)nrhs, 256, 0, s>>>(op, vi, nrhs, pc.lm, k, pc.L11, pc.L11inv, pc.T1, o);
        if (pc.np > 0)
            k_pc_blk<float><<<gb, 256, shb, s>>>(op, vi, nrhs, pc.ord, pc.np, pc.f, k, pc.V, pc.LB, pc.LBinv, pc.T1,
                                                pc.Q, o);
        if (op != kPcFac)
            k_pc_lm_post<float><<<(unsigned)nrhs, 256, 0, s>>>(pc.Q, pc.np > 0 ? pc.nblk : 0, nrhs, pc.lm, k,
                                                                pc.L11inv, pc.T1, pc.R1, o);
    } else {
        const double *vi = (const double *)v;
        double *o = (double *)out;
        k_pc_lm_pre<double><<<(unsigned)nrhs, 256, 0, s>>>(op, vi, nrhs, pc.lm, k, pc.L11, pc.L11inv, pc.T1, o);
        if (pc.np > 0)
            k_pc_blk<double><<<gb, 256, shb, s>>>(op, vi, nrhs, pc.ord, pc.np, pc.f, k, pc.V, pc.LB, pc.LBinv,
                                                 pc.T1, pc.Q, o);
        if (op != kPcFac)
            k_pc_lm_post<double><<<(unsigned)nrhs, 256, 0, s>>>(pc.Q, pc.np > 0 ? pc.nblk : 0, nrhs, pc.lm, k,
                                                                 pc.L11inv, pc.T1, pc.R1, o);
    }
    return hipGetLastError();
}

hipError_t launch_pc_dquad(int prec, const Precond &pc, const PcKer &kp, const void *w, int nrhs, double *out,
                           hipStream_t s)
{
    const int k = pc.k, np2 = kp.P + 2;
    const dim3 gb((unsigned)pc.nblk, (unsigned)nrhs);
    const size_t sh = (size_t)(2 * k + pc.f) * sizeof(double);
    const int nblk = pc.np > 0 ? pc.nblk : 0;
    if (prec == NFFTGP_F32) {
        const float *wi = (const float *)w;
        if (pc.np > 0) k_pc_nu<float><<<gb, 256, 0, s>>>(wi, nrhs, pc.ord, pc.np, pc.f, k, pc.V, pc.Q);
        k_pc_dq_lm<float><<<(unsigned)nrhs, 256, 0, s>>>(wi, nrhs, pc.Q, nblk, pc.lm, k, pc.L11inv, pc.dK11, np2,
                                                        pc.ABAR, pc.W1, pc.R1, pc.lmt);
        if (pc.np > 0)
            k_pc_dq_blk<float><<<gb, 256, sh, s>>>(wi, nrhs, pc.X, pc.ptot, pc.lm, k, pc.ord, pc.np, pc.f, kp,
                                                  pc.L11inv, pc.dK11, pc.Q, pc.ABAR, pc.W1, pc.dqp);
    } else {
        const double *wi = (const double *)w;
        if (pc.np > 0) k_pc_nu<double><<<gb, 256, 0, s>>>(wi, nrhs, pc.ord, pc.np, pc.f, k, pc.V, pc.Q);
        k_pc_dq_lm<double><<<(unsigned)nrhs, 256, 0, s>>>(wi, nrhs, pc.Q, nblk, pc.lm, k, pc.L11inv, pc.dK11, np2,
                                                         pc.ABAR, pc.W1, pc.R1, pc.lmt);
        if (pc.np > 0)
            k_pc_dq_blk<double><<<gb, 256, sh, s>>>(wi, nrhs, pc.X, pc.ptot, pc.lm, k, pc.ord, pc.np, pc.f, kp,
                                                   pc.L11inv, pc.dK11, pc.Q, pc.ABAR, pc.W1, pc.dqp);
    }
    k_pc_dq_final<<<nblocks((int64_t)nrhs * np2, 64), 64, 0, s>>>(pc.dqp, nblk, nrhs, np2, pc.lmt, out);
    return hipGetLastError();
}

hipError_t launch_pcg_start(int nrhs, double *scal, hipStream_t s)
{
    k_pcg_start<<<1, 64, 0, s>>>(nrhs, scal);
    return hipGetLastError();
}

hipError_t launch_pcg_beta(int nrhs, const double *prr, const double *prz, double *scal, double tol, double *hist,
                           hipStream_t s)
{
    k_pcg_beta<<<(unsigned)nrhs, 128, 0, s>>>(prr, prz, kDotBlocks, nrhs, scal, tol, hist);
    return hipGetLastError();
}

}  // namespace nfftgp
