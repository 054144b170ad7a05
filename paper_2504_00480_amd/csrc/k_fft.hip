// FFT over the oversampled (2N)^d grid and the diagonal multiply between the
// forward and inverse transforms (Appendix A steps 1-2 and their adjoint).
//
// The grid is stored [batch][l_0][l_1]...[l_{d-1}] (last index fastest) as
// interleaved complex values.  The forward transform uses
// exp(-2 pi i k l / n_g), the inverse exp(+2 pi i k l / n_g) without scaling.
// Grid index l corresponds to the spatial offset l - N; the sign factor
// (-1)^k this introduces in both transforms cancels in the product, so the
// diagonal is applied at the plain signed frequency k.
//
// Pruning.  Every point has t in [N/2, 3N/2], so spreading only reaches the
// cells Omega = [N/2 - m + 1, 3N/2 + m] of each axis and interpolation only
// reads them; the diagonal is zero outside the frequencies
// F = [-N/2, N/2] (indices 0..N/2 and 2N - N/2..2N-1).  Axis by axis, the
// forward transform of axis q reads Omega and keeps F, the inverse reads F and
// writes Omega, and a line of axis q only exists for the positions its other
// axes hold at that stage: Omega for the axes before q, F for those after
// (the axes are transformed from the last to the first and back).  Cells and
// frequencies outside these ranges are never read, so they need not be
// cleared.  The first axis is transformed forward, multiplied by the diagonal
// (and by the derivative diagonal) and transformed back in one pass.
//
// A work-group transforms LPB lines of one axis in LDS (iterative radix-2
// after a bit-reversed load).  Lines are numbered with the fastest other axis
// varying fastest, so for strided axes consecutive lines of a group read
// consecutive addresses.
#include "nfftgp_impl.h"
#include "nfftgp_dev.h"

namespace nfftgp {
namespace {

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

// Position j of a cyclic range (start, len) on a grid of edge ng (power of 2).
__device__ __forceinline__ int cyc_pos(int start, int j, int ng) { return (start + j) & (ng - 1); }
__device__ __forceinline__ bool cyc_has(int start, int len, int k, int ng)
{
    return ((k - start) & (ng - 1)) < len;
}

struct PruneGeom {
    int d, ng, N;
    int olo, on;   // Omega: cells olo .. olo + on - 1
    int flo, fn;   // F: indices flo .. flo + fn - 1 modulo ng
    int64_t cells;
};

template <typename T, int LOGN, int LPB>
__device__ __forceinline__ void fft_stages(typename Cplx<T>::type (*buf)[(1 << LOGN) + 1],
                                           const typename Cplx<T>::type *tw)
{
    using C = typename Cplx<T>::type;
    constexpr int NG = 1 << LOGN;
#pragma unroll
    for (int s = 1; s <= LOGN; ++s) {
        const int len = 1 << s, half = len >> 1;
        for (int bfi = threadIdx.x; bfi < LPB * NG / 2; bfi += 256) {
            const int li = bfi / (NG / 2), rest = bfi % (NG / 2);
            const int grp = rest / half, j = rest % half;
            const int i0 = grp * len + j, i1 = i0 + half;
            const C w = tw[j * (NG / len)];
            const C u = buf[li][i0], x = buf[li][i1];
            C v;
            v.x = x.x * w.x - x.y * w.y;
            v.y = x.x * w.y + x.y * w.x;
            C o0, o1;
            o0.x = u.x + v.x;
            o0.y = u.y + v.y;
            o1.x = u.x - v.x;
            o1.y = u.y - v.y;
            buf[li][i0] = o0;
            buf[li][i1] = o1;
        }
        __syncthreads();
    }
}

// Radix-2 stages over `nl` lines of a buffer with row pitch NG + 1.
template <typename T, int LOGN>
__device__ __forceinline__ void fft_stages_n(typename Cplx<T>::type *buf, int nl,
                                             const typename Cplx<T>::type *tw)
{
    using C = typename Cplx<T>::type;
    constexpr int NG = 1 << LOGN;
#pragma unroll
    for (int s = 1; s <= LOGN; ++s) {
        const int len = 1 << s, half = len >> 1;
        for (int bfi = threadIdx.x; bfi < nl * NG / 2; bfi += 256) {
            const int li = bfi / (NG / 2), rest = bfi % (NG / 2);
            const int grp = rest / half, j = rest % half;
            const int i0 = grp * len + j, i1 = i0 + half;
            C *row = buf + li * (NG + 1);
            const C w = tw[j * (NG / len)];
            const C u = row[i0], x = row[i1];
            C v;
            v.x = x.x * w.x - x.y * w.y;
            v.y = x.x * w.y + x.y * w.x;
            C o0, o1;
            o0.x = u.x + v.x;
            o0.y = u.y + v.y;
            o1.x = u.x - v.x;
            o1.y = u.y - v.y;
            row[i0] = o0;
            row[i1] = o1;
        }
        __syncthreads();
    }
}

// 3-D grids with 2N <= 64: axes 2 and 1 of one slab (batch b, first index l0)
// in one work-group.  Forward (INV false): rows l1 in Omega are transformed
// along axis 2 (input Omega, kept F), then columns K2 in F along axis 1
// (input Omega, written F).  Inverse: columns K2 in F along axis 1 (input F,
// kept Omega), then rows l1 in Omega along axis 2 (input F, written Omega).
// Grid (on, batch); LDS rows[on][NG + 1] and cols[fn][NG + 1].
template <typename T, int LOGN, bool INV>
__global__ void __launch_bounds__(256)
k_fft_slab(typename Cplx<T>::type *__restrict__ data, PruneGeom pg)
{
    using C = typename Cplx<T>::type;
    constexpr int NG = 1 << LOGN;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *rows = reinterpret_cast<C *>(smem_raw);            // [on][NG + 1]
    C *cols = rows + pg.on * (NG + 1);                     // [fn][NG + 1]
    __shared__ C tw[NG / 2];
    for (int t = threadIdx.x; t < NG / 2; t += 256) {
        double sn, cs;
        sincospi((INV ? 2.0 : -2.0) * (double)t / (double)NG, &sn, &cs);
        tw[t].x = (T)cs;
        tw[t].y = (T)sn;
    }
    const int l0 = pg.olo + blockIdx.x;
    C *slab = data + (int64_t)blockIdx.y * pg.cells + (int64_t)l0 * NG * NG;
    const int on = pg.on, fn = pg.fn;
    C zero;
    zero.x = T(0);
    zero.y = T(0);
    if (!INV) {
        // rows: l1 = olo + j, input along axis 2 at Omega
        for (int idx = threadIdx.x; idx < on * NG; idx += 256) {
            const int j = idx / NG, k = idx % NG;
            C v = zero;
            if (cyc_has(pg.olo, on, k, NG)) v = slab[(pg.olo + j) * NG + k];
            rows[j * (NG + 1) + (__brev((unsigned)k) >> (32 - LOGN))] = v;
        }
        __syncthreads();
        fft_stages_n<T, LOGN>(rows, on, tw);
        // columns K2 in F: bit-reversed along l1 (rows outside Omega are zero)
        for (int idx = threadIdx.x; idx < fn * NG; idx += 256) {
            const int c = idx / NG, l1 = idx % NG;
            const int k2 = cyc_pos(pg.flo, c, NG);
            C v = zero;
            if (cyc_has(pg.olo, on, l1, NG)) v = rows[(l1 - pg.olo) * (NG + 1) + k2];
            cols[c * (NG + 1) + (__brev((unsigned)l1) >> (32 - LOGN))] = v;
        }
        __syncthreads();
        fft_stages_n<T, LOGN>(cols, fn, tw);
        // write (K1 in F, K2 in F)
        for (int idx = threadIdx.x; idx < fn * fn; idx += 256) {
            const int a = idx / fn, c = idx % fn;
            const int k1 = cyc_pos(pg.flo, a, NG), k2 = cyc_pos(pg.flo, c, NG);
            slab[k1 * NG + k2] = cols[c * (NG + 1) + k1];
        }
    } else {
        // columns K2 in F along axis 1: input K1 in F
        for (int idx = threadIdx.x; idx < fn * NG; idx += 256) {
            const int c = idx / NG, k1 = idx % NG;
            const int k2 = cyc_pos(pg.flo, c, NG);
            C v = zero;
            if (cyc_has(pg.flo, fn, k1, NG)) v = slab[k1 * NG + k2];
            cols[c * (NG + 1) + (__brev((unsigned)k1) >> (32 - LOGN))] = v;
        }
        __syncthreads();
        fft_stages_n<T, LOGN>(cols, fn, tw);
        // rows l1 in Omega along axis 2: input K2 in F (others zero)
        for (int idx = threadIdx.x; idx < on * NG; idx += 256) {
            const int j = idx / NG, k2 = idx % NG;
            C v = zero;
            if (cyc_has(pg.flo, fn, k2, NG)) {
                const int c = (k2 - pg.flo) & (NG - 1);
                v = cols[c * (NG + 1) + pg.olo + j];
            }
            rows[j * (NG + 1) + (__brev((unsigned)k2) >> (32 - LOGN))] = v;
        }
        __syncthreads();
        fft_stages_n<T, LOGN>(rows, on, tw);
        for (int idx = threadIdx.x; idx < on * on; idx += 256) {
            const int j = idx / on, c = idx % on;
            slab[(pg.olo + j) * NG + pg.olo + c] = rows[j * (NG + 1) + pg.olo + c];
        }
    }
}

// MODE 0: forward transform of axis ax (reads Omega, writes F);
// MODE 1: inverse transform of axis ax (reads F, writes Omega);
// MODE 2: axis 0 forward, diagonal, inverse (reads Omega, writes Omega of the
//         K block and, with DER, of the derivative block der_off batches on).
template <typename T, int LOGN, int LPB, int MODE, bool DER>
__global__ void __launch_bounds__(256)
k_fft_pruned(typename Cplx<T>::type *__restrict__ data, PruneGeom pg, int ax, int64_t nlines,
             int64_t lines_per_batch, const WinDesc *__restrict__ wd, int nrhs, int64_t der_off)
{
    using C = typename Cplx<T>::type;
    constexpr int NG = 1 << LOGN;
    __shared__ C buf[LPB][NG + 1];
    __shared__ C buf2[MODE == 2 ? LPB : 1][MODE == 2 ? NG + 1 : 1];
    __shared__ C twf[NG / 2];
    __shared__ C twi[MODE == 2 ? NG / 2 : 1];
    __shared__ int64_t s_base[LPB];
    __shared__ int s_ok[LPB];
    __shared__ int s_di[LPB];
    __shared__ int s_win[LPB];
    for (int t = threadIdx.x; t < NG / 2; t += blockDim.x) {
        double sn, cs;
        sincospi((MODE == 1 ? 2.0 : -2.0) * (double)t / (double)NG, &sn, &cs);
        twf[t].x = (T)cs;
        twf[t].y = (T)sn;
        if (MODE == 2) {
            twi[t].x = (T)cs;
            twi[t].y = (T)(-sn);
        }
    }
    const int ng = NG;
    int64_t S = 1;
    for (int q = ax + 1; q < pg.d; ++q) S *= ng;
    // line bases: other axes before ax hold Omega, after ax hold F
    if ((int)threadIdx.x < LPB) {
        const int li = threadIdx.x;
        const int64_t L = (int64_t)blockIdx.x * LPB + li;
        const bool ok = L < nlines;
        const int64_t Lc = ok ? L : 0;
        // lines of one batch entry: at most 257^2, so 32-bit index math below
        const int64_t b = Lc / lines_per_batch;
        int rem = (int)(Lc - b * lines_per_batch);
        int64_t base = b * pg.cells;
        int di = 0, dstride = 1;   // offset in the (N+1)^d diagonal of the F axes
        int64_t stride = 1;
        for (int q = pg.d - 1; q >= 0; --q) {
            if (q != ax) {
                const bool om = q < ax;
                const int len = om ? pg.on : pg.fn;
                const int qt = fdiv_small(rem, len, 1.0f / (float)len);
                const int j = rem - qt * len;
                rem = qt;
                const int pos = cyc_pos(om ? pg.olo : pg.flo, j, ng);
                base += (int64_t)pos * stride;
                if (!om) {
                    const int f = pos < pg.N ? pos : pos - ng;
                    di += (f + pg.N / 2) * dstride;
                }
            }
            dstride *= pg.N + 1;
            stride *= ng;
        }
        s_base[li] = base;
        s_ok[li] = ok;
        s_di[li] = di;
        s_win[li] = (int)(b / nrhs);
    }
    __syncthreads();
    const bool in_om = MODE != 1;                    // input set: Omega or F
    const int ilo = in_om ? pg.olo : pg.flo, ilen = in_om ? pg.on : pg.fn;
    for (int idx = threadIdx.x; idx < LPB * NG; idx += 256) {
        int li, k;
        if (S == 1) {
            li = idx / NG;
            k = idx % NG;
        } else {
            k = idx / LPB;
            li = idx % LPB;
        }
        C v;
        v.x = T(0);
        v.y = T(0);
        if (s_ok[li] && cyc_has(ilo, ilen, k, ng)) v = data[s_base[li] + (int64_t)k * S];
        buf[li][__brev((unsigned)k) >> (32 - LOGN)] = v;
    }
    __syncthreads();
    fft_stages<T, LOGN, LPB>(buf, twf);
    if constexpr (MODE != 2) {
        const int olo2 = MODE == 0 ? pg.flo : pg.olo, olen = MODE == 0 ? pg.fn : pg.on;
        for (int idx = threadIdx.x; idx < LPB * NG; idx += 256) {
            int li, k;
            if (S == 1) {
                li = idx / NG;
                k = idx % NG;
            } else {
                k = idx / LPB;
                li = idx % LPB;
            }
            if (s_ok[li] && cyc_has(olo2, olen, k, ng)) data[s_base[li] + (int64_t)k * S] = buf[li][k];
        }
    } else {
    // MODE 2 (ax == 0, stride S): diagonal of axis 0 frequency k times the
    // line's offset in the (N+1)^d diagonal, then the inverse transform
    int64_t dstr0 = 1;
    for (int q = 1; q < pg.d; ++q) dstr0 *= (pg.N + 1);
#pragma unroll 1
    for (int pass = 0; pass < (DER ? 2 : 1); ++pass) {
        for (int idx = threadIdx.x; idx < LPB * NG; idx += 256) {
            const int k = S == 1 ? idx % NG : idx / LPB, li = S == 1 ? idx / NG : idx % LPB;
            const int f = k < pg.N ? k : k - ng;
            T dv = T(0);
            if (s_ok[li] && f >= -pg.N / 2 && f <= pg.N / 2) {
                const WinDesc &w = wd[s_win[li]];
                const T *D = reinterpret_cast<const T *>(pass == 0 ? w.Dk : w.Dder);
                dv = D[(int64_t)(f + pg.N / 2) * dstr0 + s_di[li]];
            }
            C v = buf[li][k];
            v.x *= dv;
            v.y *= dv;
            buf2[li][__brev((unsigned)k) >> (32 - LOGN)] = v;
        }
        __syncthreads();
        fft_stages<T, LOGN, LPB>(buf2, twi);
        const int64_t off = pass == 0 ? 0 : der_off * pg.cells;
        for (int idx = threadIdx.x; idx < LPB * NG; idx += 256) {
            const int k = S == 1 ? idx % NG : idx / LPB, li = S == 1 ? idx / NG : idx % LPB;
            if (s_ok[li] && cyc_has(pg.olo, pg.on, k, ng)) data[off + s_base[li] + (int64_t)k * S] = buf2[li][k];
        }
        __syncthreads();
    }
    }
}

PruneGeom prune_geom(const WindowGeom &g, int m)
{
    PruneGeom pg;
    pg.d = g.d;
    pg.ng = g.ng;
    pg.N = g.N;
    pg.olo = g.N / 2 - m + 1;
    pg.on = g.N + 2 * m;
    pg.flo = g.ng - g.N / 2;
    pg.fn = g.N + 1;
    pg.cells = g.cells;
    return pg;
}

int64_t lines_of(const PruneGeom &pg, int ax)
{
    int64_t l = 1;
    for (int q = 0; q < pg.d; ++q)
        if (q != ax) l *= q < ax ? pg.on : pg.fn;
    return l;
}

template <typename T, int LOGN, int MODE, bool DER>
hipError_t fft_launch(void *grid, const PruneGeom &pg, int ax, int64_t batch, const WinDesc *wd,
                      int nrhs, int64_t der_off, hipStream_t s)
{
    constexpr int LPB = (1 << LOGN) >= 256 ? 4 : ((1 << LOGN) >= 128 ? 8 : 16);
    const int64_t lpb = lines_of(pg, ax);
    const int64_t nlines = batch * lpb;
    const unsigned nblk = (unsigned)((nlines + LPB - 1) / LPB);
    if (nblk == 0) return hipSuccess;
    k_fft_pruned<T, LOGN, LPB, MODE, DER><<<nblk, 256, 0, s>>>(
        (typename Cplx<T>::type *)grid, pg, ax, nlines, lpb, wd, nrhs, der_off);
    return hipGetLastError();
}

template <typename T, int MODE, bool DER>
hipError_t fft_dispatch(int logn, void *grid, const PruneGeom &pg, int ax, int64_t batch,
                        const WinDesc *wd, int nrhs, int64_t der_off, hipStream_t s)
{
    switch (logn) {
    case 4: return fft_launch<T, 4, MODE, DER>(grid, pg, ax, batch, wd, nrhs, der_off, s);
    case 5: return fft_launch<T, 5, MODE, DER>(grid, pg, ax, batch, wd, nrhs, der_off, s);
    case 6: return fft_launch<T, 6, MODE, DER>(grid, pg, ax, batch, wd, nrhs, der_off, s);
    case 7: return fft_launch<T, 7, MODE, DER>(grid, pg, ax, batch, wd, nrhs, der_off, s);
    case 8: return fft_launch<T, 8, MODE, DER>(grid, pg, ax, batch, wd, nrhs, der_off, s);
    default: return hipErrorInvalidValue;
    }
}

int log2i(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// Slab pass of a 3-D group (2N <= 64): one launch for axes 2 and 1.
template <typename T, bool INV>
hipError_t slab_t(const Group &G, const PruneGeom &pg, void *grid, int64_t batch, hipStream_t s)
{
    using C = typename Cplx<T>::type;
    const size_t shm = (size_t)(pg.on + pg.fn) * (G.g.ng + 1) * sizeof(C);
    const dim3 grd((unsigned)pg.on, (unsigned)batch);
    hipError_t e;
    switch (G.g.ng) {
    case 16:
        e = hipFuncSetAttribute((const void *)k_fft_slab<T, 4, INV>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        k_fft_slab<T, 4, INV><<<grd, 256, shm, s>>>((C *)grid, pg);
        break;
    case 32:
        e = hipFuncSetAttribute((const void *)k_fft_slab<T, 5, INV>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        k_fft_slab<T, 5, INV><<<grd, 256, shm, s>>>((C *)grid, pg);
        break;
    case 64:
        e = hipFuncSetAttribute((const void *)k_fft_slab<T, 6, INV>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        k_fft_slab<T, 6, INV><<<grd, 256, shm, s>>>((C *)grid, pg);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool use_slab(const Group &G) { return G.g.d == 3 && G.g.ng <= 64; }

template <typename T>
hipError_t fwd_t(const Group &G, int m, void *grid, int nrhs, hipStream_t s)
{
    const PruneGeom pg = prune_geom(G.g, m);
    const int64_t batch = (int64_t)G.nwin * nrhs;
    if (use_slab(G)) return slab_t<T, false>(G, pg, grid, batch, s);
    for (int ax = G.g.d - 1; ax >= 1; --ax) {
        hipError_t e = fft_dispatch<T, 0, false>(log2i(G.g.ng), grid, pg, ax, batch, G.desc, nrhs, 0, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t inv_t(const Group &G, int m, void *grid, int nrhs, bool with_der, hipStream_t s)
{
    const PruneGeom pg = prune_geom(G.g, m);
    const int64_t batch = (int64_t)G.nwin * nrhs * (with_der ? 2 : 1);
    if (use_slab(G)) return slab_t<T, true>(G, pg, grid, batch, s);
    for (int ax = 1; ax < G.g.d; ++ax) {
        hipError_t e = fft_dispatch<T, 1, false>(log2i(G.g.ng), grid, pg, ax, batch, G.desc, nrhs, 0, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t fused_t(const Group &G, int m, void *grid, int nrhs, bool with_der, hipStream_t s)
{
    const PruneGeom pg = prune_geom(G.g, m);
    const int64_t batch = (int64_t)G.nwin * nrhs;
    if (with_der)
        return fft_dispatch<T, 2, true>(log2i(G.g.ng), grid, pg, 0, batch, G.desc, nrhs, batch, s);
    return fft_dispatch<T, 2, false>(log2i(G.g.ng), grid, pg, 0, batch, G.desc, nrhs, batch, s);
}

}  // namespace

hipError_t launch_fft_fwd(int prec, const Group &G, int m, void *grid, int nrhs, hipStream_t s)
{
    return prec == NFFTGP_F32 ? fwd_t<float>(G, m, grid, nrhs, s) : fwd_t<double>(G, m, grid, nrhs, s);
}

hipError_t launch_fft_diag(int prec, const Group &G, int m, void *grid, int nrhs, bool with_der,
                           hipStream_t s)
{
    return prec == NFFTGP_F32 ? fused_t<float>(G, m, grid, nrhs, with_der, s)
                              : fused_t<double>(G, m, grid, nrhs, with_der, s);
}

hipError_t launch_fft_inv(int prec, const Group &G, int m, void *grid, int nrhs, bool with_der,
                          hipStream_t s)
{
    return prec == NFFTGP_F32 ? inv_t<float>(G, m, grid, nrhs, with_der, s)
                              : inv_t<double>(G, m, grid, nrhs, with_der, s);
}

}  // namespace nfftgp
