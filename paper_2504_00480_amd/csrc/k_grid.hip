// Grid kernels of the fast summation (Sec. 3.1 eq. Fourier_sum; Appendix A):
//
//   spreading      g_l = sum_j v_j psi(t_j - l)          (adjoint NFFT, gridding)
//   fold           deterministic sum of the per-tile partial grids
//   interpolation  h_i = sum_l G_l psi(t_i - l)          (NFFT, sparse window sums)
//   assembly       sigma_f^2 sum_s h^(s) + sigma_eps^2 v and derivative blocks
//
// Coordinates t are in grid units (t = 2N x~ + N, x~ in [-1/4, 1/4)), so a
// point touches the 2m cells floor(t)-m+1 .. floor(t)+m per dimension.  psi is
// the Kaiser-Bessel window of Appendix A in grid units, normalised so that
// its Fourier coefficient at frequency 0 is 1 / (2N):
//   psi(t) = sinh(b sqrt(m^2 - t^2)) / (pi sqrt(m^2 - t^2) I_0(m b)),  |t| <= m.
//
// Points are sorted by tile ("bin", tb cells per dimension); a subproblem is a
// run of at most kMaxSubPoints points of one bin.  Spreading accumulates one
// subproblem into an LDS copy of its padded tile ((tb + 2m)^d cells) and writes
// the tile out; no global atomics are used and the result does not depend on
// scheduling: each wave owns one LDS copy and adds one point at a time, and
// the copies and tiles are summed in a fixed order.
#include "nfftgp_impl.h"

namespace nfftgp {
namespace {

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

template <typename T, int M>
__device__ __forceinline__ T kb_psi(T t, T beta, T knorm)
{
    T s2 = T(M * M) - t * t;
    s2 = s2 > T(0) ? s2 : T(0);
    T s = sqrt(s2);
    T z = beta * s;
    T r;
    if (z < T(1e-3)) {
        r = beta * (T(1) + z * z * T(1.0 / 6.0));
    } else {
        r = T(0.5) * (expm1(z) - expm1(-z)) / s;
    }
    return r * knorm;
}

__device__ __forceinline__ float rdlane(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double rdlane(double v, int l)
{
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ int rdlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ float bperm(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(l << 2, __float_as_int(v)));
}
__device__ __forceinline__ double bperm(double v, int l)
{
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_ds_bpermute(l << 2, (int)(b & 0xffffffffLL));
    int hi = __builtin_amdgcn_ds_bpermute(l << 2, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int D>
__device__ __forceinline__ void bin_origin(int bin, int nb, int tb, int *org)
{
    int rem = bin;
    for (int q = D - 1; q >= 0; --q) {
        org[q] = (rem % nb) * tb;
        rem /= nb;
    }
}

// ---------------------------------------------------------------- spreading
template <typename T, int D, int M, int W>
__global__ void __launch_bounds__(W * 64)
k_spread(const T *__restrict__ ts, int64_t n, const int *__restrict__ perm,
         const T *__restrict__ V, int64_t ldv, int nrhs, const int *__restrict__ sub_bin,
         const int *__restrict__ sub_start, const int *__restrict__ sub_count, int tb, int nb,
         T beta, T knorm, T *__restrict__ tilebuf)
{
    constexpr int TW = 2 * M;
    constexpr int PW = 64 / TW;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tiles = reinterpret_cast<T *>(smem_raw);
    const int pd = tb + 2 * M;
    int pc = pd;
    for (int q = 1; q < D; ++q) pc *= pd;
    const int sq = blockIdx.x, r = blockIdx.y;
    const int start = sub_start[sq], cnt = sub_count[sq];
    int org[3] = {0, 0, 0};
    bin_origin<D>(sub_bin[sq], nb, tb, org);
    for (int i = threadIdx.x; i < W * pc; i += blockDim.x) tiles[i] = T(0);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    T *my = tiles + wave * pc;
    const int pt = lane / TW, a = lane % TW;
    for (int base = wave * PW; base < cnt; base += W * PW) {
        const bool valid = (pt < PW) && (base + pt < cnt);
        T w[D];
        int anc[D];
        T v = T(0);
#pragma unroll
        for (int q = 0; q < D; ++q) {
            w[q] = T(0);
            anc[q] = 0;
        }
        if (valid) {
            const int64_t j = start + base + pt;
#pragma unroll
            for (int q = 0; q < D; ++q) {
                T t = ts[(int64_t)q * n + j];
                T fl = floor(t);
                anc[q] = (int)fl - org[q] + 1;   // local index of the first tap
                w[q] = kb_psi<T, M>(t - (fl - T(M - 1) + T(a)), beta, knorm);
            }
            v = V[(int64_t)perm[j] * ldv + r];
        }
        if (D == 1) {
            if (valid) atomicAdd(my + anc[0] + a, w[0] * v);
            continue;
        }
        const int npts = min(PW, cnt - base);
        for (int p = 0; p < npts; ++p) {
            const int src = p * TW;
            const int A0 = rdlane(anc[0], src);
            const int A1 = rdlane(anc[D > 1 ? 1 : 0], src);
            const int A2 = rdlane(anc[D > 2 ? 2 : 0], src);
            const T vp = rdlane(v, src);
            if (D == 2) {
#pragma unroll
                for (int it = 0; it < (TW * TW + 63) / 64; ++it) {
                    const int tau = lane + 64 * it;
                    const int ta = min(tau / TW, TW - 1), tbb = tau % TW;
                    const T w0 = bperm(w[0], src + ta);
                    const T w1 = bperm(w[D > 1 ? 1 : 0], src + tbb);
                    if (tau < TW * TW) atomicAdd(my + (A0 + ta) * pd + (A1 + tbb), w0 * w1 * vp);
                }
            } else {
#pragma unroll
                for (int it = 0; it < (TW * TW + 63) / 64; ++it) {
                    const int pi = lane + 64 * it;
                    const int tbb = min(pi / TW, TW - 1), tc = pi % TW;
                    const T w1 = bperm(w[D > 1 ? 1 : 0], src + tbb);
                    const T w2 = bperm(w[D > 2 ? 2 : 0], src + tc);
                    const T wbc = w1 * w2 * vp;
                    if (pi < TW * TW) {
                        T *col = my + (A1 + tbb) * pd + (A2 + tc) + A0 * pd * pd;
#pragma unroll
                        for (int aa = 0; aa < TW; ++aa) {
                            const T w0 = rdlane(w[0], src + aa);
                            atomicAdd(col + aa * pd * pd, w0 * wbc);
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    T *out = tilebuf + ((int64_t)sq * nrhs + r) * pc;
    for (int i = threadIdx.x; i < pc; i += blockDim.x) {
        T s = tiles[i];
        for (int c = 1; c < W; ++c) s += tiles[c * pc + i];
        out[i] = s;
    }
}

// ---------------------------------------------------------------- fold
template <typename T, int D>
__global__ void __launch_bounds__(256)
k_fold(const T *__restrict__ tilebuf, const int *__restrict__ bin_sub_ptr, int nrhs, int tb,
       int nb, int ng, int m, int pd, int pc, int64_t cells,
       typename Cplx<T>::type *__restrict__ grid)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nrhs * cells) return;
    const int r = (int)(idx / cells);
    const int64_t cell = idx % cells;
    int l[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    int64_t rem = cell;
    for (int q = D - 1; q >= 0; --q) {
        l[q] = (int)(rem % ng);
        rem /= ng;
        // bins b with b*tb - m <= l <= b*tb - m + pd - 1
        int num = l[q] + m - pd + 1;
        int blo = num >= 0 ? (num + tb - 1) / tb : -((-num) / tb);
        int bhi = (l[q] + m) / tb;
        lo[q] = blo < 0 ? 0 : blo;
        hi[q] = bhi > nb - 1 ? nb - 1 : bhi;
    }
    T sum = T(0);
    for (int b0 = lo[0]; b0 <= hi[0]; ++b0)
        for (int b1 = (D > 1 ? lo[1] : 0); b1 <= (D > 1 ? hi[1] : 0); ++b1)
            for (int b2 = (D > 2 ? lo[2] : 0); b2 <= (D > 2 ? hi[2] : 0); ++b2) {
                int bin = b0, li = l[0] - b0 * tb + m;
                if (D > 1) {
                    bin = bin * nb + b1;
                    li = li * pd + (l[1] - b1 * tb + m);
                }
                if (D > 2) {
                    bin = bin * nb + b2;
                    li = li * pd + (l[2] - b2 * tb + m);
                }
                for (int s = bin_sub_ptr[bin]; s < bin_sub_ptr[bin + 1]; ++s)
                    sum += tilebuf[((int64_t)s * nrhs + r) * pc + li];
            }
    typename Cplx<T>::type o;
    o.x = sum;
    o.y = T(0);
    grid[idx] = o;
}

// ---------------------------------------------------------------- interpolation
template <typename T, int D, int M, bool DER>
__global__ void __launch_bounds__(256)
k_interp(const T *__restrict__ ts, int64_t n, const int *__restrict__ perm,
         const int *__restrict__ sub_bin, const int *__restrict__ sub_start,
         const int *__restrict__ sub_count, int tb, int nb, int ng, T beta, T knorm,
         const typename Cplx<T>::type *__restrict__ gridK,
         const typename Cplx<T>::type *__restrict__ gridD, int64_t cells, int nrhs,
         T *__restrict__ acc, T *__restrict__ comp, T *__restrict__ dout, T dscale)
{
    constexpr int TW = 2 * M;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tK = reinterpret_cast<T *>(smem_raw);
    const int pd = tb + 2 * M;
    int pc = pd;
    for (int q = 1; q < D; ++q) pc *= pd;
    T *tD = tK + pc;
    const int sq = blockIdx.x, r = blockIdx.y;
    const int start = sub_start[sq], cnt = sub_count[sq];
    int org[3] = {0, 0, 0};
    bin_origin<D>(sub_bin[sq], nb, tb, org);
    const typename Cplx<T>::type *gK = gridK + (int64_t)r * cells;
    const typename Cplx<T>::type *gD = DER ? gridD + (int64_t)r * cells : nullptr;
    for (int i = threadIdx.x; i < pc; i += blockDim.x) {
        int rem = i, loc[3] = {0, 0, 0};
        for (int q = D - 1; q >= 0; --q) {
            loc[q] = rem % pd;
            rem /= pd;
        }
        bool in = true;
        int64_t g = 0;
        for (int q = 0; q < D; ++q) {
            int l = org[q] - M + loc[q];
            in = in && (l >= 0) && (l < ng);
            g = g * ng + l;
        }
        tK[i] = in ? gK[g].x : T(0);
        if (DER) tD[i] = in ? gD[g].x : T(0);
    }
    __syncthreads();
    for (int p = threadIdx.x; p < cnt; p += blockDim.x) {
        const int64_t j = start + p;
        // per-dimension window weights; for d = 3 the first dimension's weights
        // are evaluated inside its loop so that no register array is indexed
        // by a loop variable
        T w[D][TW];
        T t0 = T(0), fl0 = T(0);
        int A[3] = {0, 0, 0};
#pragma unroll
        for (int q = 0; q < D; ++q) {
            T t = ts[(int64_t)q * n + j];
            T fl = floor(t);
            A[q] = (int)fl - org[q] + 1;
            if (q == 0) {
                t0 = t;
                fl0 = fl;
            }
            if (D < 3 || q > 0) {
#pragma unroll
                for (int aa = 0; aa < TW; ++aa)
                    w[q][aa] = kb_psi<T, M>(t - (fl - T(M - 1) + T(aa)), beta, knorm);
            }
        }
        T hK = T(0), hD = T(0);
        if (D == 1) {
#pragma unroll
            for (int aa = 0; aa < TW; ++aa) {
                hK += tK[A[0] + aa] * w[0][aa];
                if (DER) hD += tD[A[0] + aa] * w[0][aa];
            }
        } else if (D == 2) {
#pragma unroll
            for (int aa = 0; aa < TW; ++aa) {
                T sK = T(0), sD = T(0);
                const int row = (A[0] + aa) * pd + A[1];
#pragma unroll
                for (int bb = 0; bb < TW; ++bb) {
                    sK += tK[row + bb] * w[D > 1 ? 1 : 0][bb];
                    if (DER) sD += tD[row + bb] * w[D > 1 ? 1 : 0][bb];
                }
                hK += sK * w[0][aa];
                if (DER) hD += sD * w[0][aa];
            }
        } else {
#pragma unroll 1
            for (int aa = 0; aa < TW; ++aa) {
                const T w0 = kb_psi<T, M>(t0 - (fl0 - T(M - 1) + T(aa)), beta, knorm);
                T sK = T(0), sD = T(0);
#pragma unroll
                for (int bb = 0; bb < TW; ++bb) {
                    const int row = ((A[0] + aa) * pd + (A[1] + bb)) * pd + A[2];
                    T cK = T(0), cD = T(0);
#pragma unroll
                    for (int cc = 0; cc < TW; ++cc) {
                        cK += tK[row + cc] * w[D > 2 ? 2 : 0][cc];
                        if (DER) cD += tD[row + cc] * w[D > 2 ? 2 : 0][cc];
                    }
                    sK += cK * w[D > 1 ? 1 : 0][bb];
                    if (DER) sD += cD * w[D > 1 ? 1 : 0][bb];
                }
                hK += sK * w0;
                if (DER) hD += sD * w0;
            }
        }
        const int64_t o = (int64_t)perm[j] * nrhs + r;
        // compensated sum over windows (Kahan)
        T s0 = acc[o];
        T y = hK - comp[o];
        T s1 = s0 + y;
        comp[o] = (s1 - s0) - y;
        acc[o] = s1;
        if (DER) dout[o] = dscale * hD;
    }
}

template <typename T>
__global__ void k_fill(T *__restrict__ p, int64_t count)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = T(0);
}

template <typename T>
__global__ void k_assemble(int64_t n, int nrhs, const T *__restrict__ V, int64_t ldv,
                           const T *__restrict__ acc, const T *__restrict__ comp, T sf2, T se2,
                           T two_sf, T two_se, T *__restrict__ KV, T *__restrict__ dsf,
                           T *__restrict__ dse)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * nrhs) return;
    int64_t i = idx / nrhs;
    int r = (int)(idx % nrhs);
    T s = acc[idx] - comp[idx];
    T v = V[i * ldv + r];
    KV[idx] = sf2 * s + se2 * v;
    if (dsf) dsf[idx] = two_sf * s;
    if (dse) dse[idx] = two_se * v;
}

// Normalisation 1 / (pi I_0(m b)) of psi, evaluated on the host in FP64.
double kb_knorm(int m)
{
    double z = m * kb_beta(), q = 0.25 * z * z, term = 1.0, sum = 1.0;
    for (int j = 1; j < 500; ++j) {
        term *= q / ((double)j * (double)j);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return 1.0 / (kPi * sum);
}

// Kernels that need more than 64 KiB of dynamic LDS must say so before launch.
template <typename K>
hipError_t allow_lds(K kernel, size_t bytes)
{
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename T, int D, int M>
hipError_t spread_dm(const Window &w, int64_t n, const void *V, int64_t ldv, int nrhs,
                     void *tilebuf, hipStream_t s)
{
    const WindowGeom &g = w.g;
    size_t tile_bytes = (size_t)g.pc * sizeof(T);
    dim3 grid((unsigned)w.nsub, (unsigned)nrhs);
    T beta = (T)kb_beta(), knorm = (T)kb_knorm(M);
    if (4 * tile_bytes <= 64 * 1024) {
        k_spread<T, D, M, 4><<<grid, 256, 4 * tile_bytes, s>>>(
            (const T *)w.t_sorted, n, w.perm, (const T *)V, ldv, nrhs, w.sub_bin, w.sub_start,
            w.sub_count, g.tb, g.nb, beta, knorm, (T *)tilebuf);
    } else if (2 * tile_bytes <= 64 * 1024) {
        k_spread<T, D, M, 2><<<grid, 128, 2 * tile_bytes, s>>>(
            (const T *)w.t_sorted, n, w.perm, (const T *)V, ldv, nrhs, w.sub_bin, w.sub_start,
            w.sub_count, g.tb, g.nb, beta, knorm, (T *)tilebuf);
    } else {
        hipError_t e = allow_lds(k_spread<T, D, M, 1>, tile_bytes);
        if (e != hipSuccess) return e;
        k_spread<T, D, M, 1><<<grid, 64, tile_bytes, s>>>(
            (const T *)w.t_sorted, n, w.perm, (const T *)V, ldv, nrhs, w.sub_bin, w.sub_start,
            w.sub_count, g.tb, g.nb, beta, knorm, (T *)tilebuf);
    }
    return hipGetLastError();
}

template <typename T, int D, int M>
hipError_t interp_dm(const Window &w, int64_t n, int nrhs, const void *grid, bool with_der,
                     void *acc, void *comp, void *dout, double dscale, hipStream_t s)
{
    const WindowGeom &g = w.g;
    using C = typename Cplx<T>::type;
    const C *gK = (const C *)grid;
    const C *gD = gK + (int64_t)nrhs * g.cells;
    dim3 grd((unsigned)w.nsub, (unsigned)nrhs);
    T beta = (T)kb_beta(), knorm = (T)kb_knorm(M);
    size_t shm = (size_t)g.pc * sizeof(T) * (with_der ? 2 : 1);
    hipError_t e = with_der ? allow_lds(k_interp<T, D, M, true>, shm) : allow_lds(k_interp<T, D, M, false>, shm);
    if (e != hipSuccess) return e;
    if (with_der)
        k_interp<T, D, M, true><<<grd, 256, shm, s>>>(
            (const T *)w.t_sorted, n, w.perm, w.sub_bin, w.sub_start, w.sub_count, g.tb, g.nb, g.ng,
            beta, knorm, gK, gD, g.cells, nrhs, (T *)acc, (T *)comp, (T *)dout, (T)dscale);
    else
        k_interp<T, D, M, false><<<grd, 256, shm, s>>>(
            (const T *)w.t_sorted, n, w.perm, w.sub_bin, w.sub_start, w.sub_count, g.tb, g.nb, g.ng,
            beta, knorm, gK, nullptr, g.cells, nrhs, (T *)acc, (T *)comp, nullptr, (T)dscale);
    return hipGetLastError();
}

#define NFFTGP_DISPATCH_DM(FN, T, D, M, ...)                         \
    switch (M) {                                                     \
    case 2: return FN<T, D, 2>(__VA_ARGS__);                         \
    case 4: return FN<T, D, 4>(__VA_ARGS__);                         \
    case 6: return FN<T, D, 6>(__VA_ARGS__);                         \
    case 8: return FN<T, D, 8>(__VA_ARGS__);                         \
    default: return hipErrorInvalidValue;                            \
    }

template <typename T>
hipError_t spread_t(const Window &w, int m, int64_t n, const void *V, int64_t ldv, int nrhs,
                    void *tilebuf, hipStream_t s)
{
    switch (w.g.d) {
    case 1: NFFTGP_DISPATCH_DM(spread_dm, T, 1, m, w, n, V, ldv, nrhs, tilebuf, s)
    case 2: NFFTGP_DISPATCH_DM(spread_dm, T, 2, m, w, n, V, ldv, nrhs, tilebuf, s)
    case 3: NFFTGP_DISPATCH_DM(spread_dm, T, 3, m, w, n, V, ldv, nrhs, tilebuf, s)
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t interp_t(const Window &w, int m, int64_t n, int nrhs, const void *grid, bool with_der,
                    void *acc, void *comp, void *dout, double dscale, hipStream_t s)
{
    switch (w.g.d) {
    case 1: NFFTGP_DISPATCH_DM(interp_dm, T, 1, m, w, n, nrhs, grid, with_der, acc, comp, dout, dscale, s)
    case 2: NFFTGP_DISPATCH_DM(interp_dm, T, 2, m, w, n, nrhs, grid, with_der, acc, comp, dout, dscale, s)
    case 3: NFFTGP_DISPATCH_DM(interp_dm, T, 3, m, w, n, nrhs, grid, with_der, acc, comp, dout, dscale, s)
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t fold_t(const Window &w, int m, int nrhs, const void *tilebuf, void *grid, hipStream_t s)
{
    const WindowGeom &g = w.g;
    using C = typename Cplx<T>::type;
    int64_t tot = (int64_t)nrhs * g.cells;
    unsigned nblk = (unsigned)((tot + 255) / 256);
    switch (g.d) {
    case 1: k_fold<T, 1><<<nblk, 256, 0, s>>>((const T *)tilebuf, w.bin_sub_ptr, nrhs, g.tb, g.nb, g.ng, m, g.pd, g.pc, g.cells, (C *)grid); break;
    case 2: k_fold<T, 2><<<nblk, 256, 0, s>>>((const T *)tilebuf, w.bin_sub_ptr, nrhs, g.tb, g.nb, g.ng, m, g.pd, g.pc, g.cells, (C *)grid); break;
    case 3: k_fold<T, 3><<<nblk, 256, 0, s>>>((const T *)tilebuf, w.bin_sub_ptr, nrhs, g.tb, g.nb, g.ng, m, g.pd, g.pc, g.cells, (C *)grid); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fill(int prec, void *p, int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    unsigned nblk = (unsigned)((count + 255) / 256);
    if (prec == NFFTGP_F32)
        k_fill<float><<<nblk, 256, 0, s>>>((float *)p, count);
    else
        k_fill<double><<<nblk, 256, 0, s>>>((double *)p, count);
    return hipGetLastError();
}

hipError_t launch_spread(int prec, const Window &w, int m, int64_t n, const void *V, int64_t ldv,
                         int nrhs, void *tilebuf, hipStream_t s)
{
    if (w.nsub == 0) return hipSuccess;
    return prec == NFFTGP_F32 ? spread_t<float>(w, m, n, V, ldv, nrhs, tilebuf, s)
                              : spread_t<double>(w, m, n, V, ldv, nrhs, tilebuf, s);
}

hipError_t launch_fold(int prec, const Window &w, int m, int nrhs, const void *tilebuf, void *grid,
                       hipStream_t s)
{
    return prec == NFFTGP_F32 ? fold_t<float>(w, m, nrhs, tilebuf, grid, s)
                              : fold_t<double>(w, m, nrhs, tilebuf, grid, s);
}

hipError_t launch_interp(int prec, const Window &w, int m, int64_t n, int nrhs, const void *grid,
                         bool with_der, void *acc, void *comp, void *dout, double dscale,
                         hipStream_t s)
{
    if (w.nsub == 0) return hipSuccess;
    return prec == NFFTGP_F32
               ? interp_t<float>(w, m, n, nrhs, grid, with_der, acc, comp, dout, dscale, s)
               : interp_t<double>(w, m, n, nrhs, grid, with_der, acc, comp, dout, dscale, s);
}

hipError_t launch_assemble(int prec, int64_t n, int nrhs, const void *V, int64_t ldv,
                           const void *acc, const void *comp, double sf, double se, void *KV,
                           void *dsf, void *dse, hipStream_t s)
{
    int64_t tot = n * nrhs;
    if (tot == 0) return hipSuccess;
    unsigned nblk = (unsigned)((tot + 255) / 256);
    if (prec == NFFTGP_F32)
        k_assemble<float><<<nblk, 256, 0, s>>>(n, nrhs, (const float *)V, ldv, (const float *)acc,
                                               (const float *)comp, (float)(sf * sf),
                                               (float)(se * se), (float)(2 * sf), (float)(2 * se),
                                               (float *)KV, (float *)dsf, (float *)dse);
    else
        k_assemble<double><<<nblk, 256, 0, s>>>(n, nrhs, (const double *)V, ldv,
                                                (const double *)acc, (const double *)comp, sf * sf,
                                                se * se, 2 * sf, 2 * se, (double *)KV,
                                                (double *)dsf, (double *)dse);
    return hipGetLastError();
}

}  // namespace nfftgp
