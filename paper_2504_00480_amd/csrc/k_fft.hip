// FFT over the oversampled (2N)^d grid and the diagonal multiply between the
// forward and inverse transforms (Appendix A steps 1-2 and their adjoint).
//
// The grid is stored [batch][l_0][l_1]...[l_{d-1}] (last index fastest) as
// interleaved complex values.  A work-group transforms 16 lines along one axis
// in LDS (iterative radix-2 after a bit-reversed load); for strided axes the
// 16 lines are adjacent in the fastest index, so every global access is a
// contiguous run of 16 complex values.  The forward transform uses
// exp(-2 pi i k l / n_g), the inverse exp(+2 pi i k l / n_g) without scaling.
//
// Grid index l corresponds to the spatial offset l - N; the sign factor
// (-1)^k this introduces in both transforms cancels in the product, so the
// diagonal is applied at the plain signed frequency k.
#include "nfftgp_impl.h"

namespace nfftgp {
namespace {

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

constexpr int kLines = 16;

template <typename T, int LOGN, bool INV>
__global__ void __launch_bounds__(256)
k_fft_lines(typename Cplx<T>::type *__restrict__ data, int64_t S, int64_t nlines)
{
    using C = typename Cplx<T>::type;
    constexpr int NG = 1 << LOGN;
    __shared__ C buf[kLines][NG + 1];
    __shared__ C tw[NG / 2];
    for (int t = threadIdx.x; t < NG / 2; t += blockDim.x) {
        double sn, cs;
        sincospi((INV ? 2.0 : -2.0) * (double)t / (double)NG, &sn, &cs);
        tw[t].x = (T)cs;
        tw[t].y = (T)sn;
    }
    const int64_t b = blockIdx.x;
    int64_t outer0 = 0, outer = 0, inner0 = 0;
    if (S == 1) {
        outer0 = b * kLines;
    } else {
        const int64_t nib = S / kLines;
        outer = b / nib;
        inner0 = (b % nib) * kLines;
    }
    for (int idx = threadIdx.x; idx < kLines * NG; idx += blockDim.x) {
        int li, k;
        int64_t addr;
        bool ok = true;
        if (S == 1) {
            li = idx / NG;
            k = idx % NG;
            ok = outer0 + li < nlines;
            addr = (outer0 + li) * NG + k;
        } else {
            k = idx / kLines;
            li = idx % kLines;
            addr = outer * NG * S + (int64_t)k * S + inner0 + li;
        }
        const int rk = (int)(__brev((unsigned)k) >> (32 - LOGN));
        C v;
        v.x = T(0);
        v.y = T(0);
        if (ok) v = data[addr];
        buf[li][rk] = v;
    }
    __syncthreads();
#pragma unroll
    for (int s = 1; s <= LOGN; ++s) {
        const int len = 1 << s, half = len >> 1;
        for (int bfi = threadIdx.x; bfi < kLines * NG / 2; bfi += blockDim.x) {
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
    for (int idx = threadIdx.x; idx < kLines * NG; idx += blockDim.x) {
        int li, k;
        int64_t addr;
        bool ok = true;
        if (S == 1) {
            li = idx / NG;
            k = idx % NG;
            ok = outer0 + li < nlines;
            addr = (outer0 + li) * NG + k;
        } else {
            k = idx / kLines;
            li = idx % kLines;
            addr = outer * NG * S + (int64_t)k * S + inner0 + li;
        }
        if (ok) data[addr] = buf[li][k];
    }
}

// Multiply the spectrum by the symmetrised diagonal on [-N/2, N/2]^d and clear
// every other frequency.  The spectra of a group are stored [window][vector]
// [cell]; with DER the same input also gives the derivative spectrum, written
// one group-block further on.
template <typename T, int D, bool DER>
__global__ void __launch_bounds__(256)
k_diag(typename Cplx<T>::type *__restrict__ spec, const WinDesc *__restrict__ wd, int N,
       int nrhs, int64_t cells, int64_t total)
{
    using C = typename Cplx<T>::type;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const WinDesc &win = wd[idx / ((int64_t)nrhs * cells)];
    int64_t rem = idx % cells;
    const int ng = 2 * N;
    bool in = true;
    int64_t di = 0, stride = 1;
    for (int q = D - 1; q >= 0; --q) {
        int K = (int)(rem % ng);
        rem /= ng;
        int f = K < N ? K : K - ng;
        in = in && (f >= -N / 2) && (f <= N / 2);
        di += (int64_t)(f + N / 2) * stride;
        stride *= (N + 1);
    }
    C v = spec[idx];
    C ok, od;
    if (in) {
        T dk = reinterpret_cast<const T *>(win.Dk)[di];
        ok.x = v.x * dk;
        ok.y = v.y * dk;
        if (DER) {
            T dd = reinterpret_cast<const T *>(win.Dder)[di];
            od.x = v.x * dd;
            od.y = v.y * dd;
        }
    } else {
        ok.x = ok.y = T(0);
        od.x = od.y = T(0);
    }
    spec[idx] = ok;
    if (DER) spec[total + idx] = od;
}

template <typename T, bool INV>
hipError_t fft_t(const WindowGeom &g, void *grid, int batch, hipStream_t s)
{
    using C = typename Cplx<T>::type;
    int logn = 0;
    while ((1 << logn) < g.ng) ++logn;
    for (int ax = 0; ax < g.d; ++ax) {
        int64_t S = 1;
        for (int q = ax + 1; q < g.d; ++q) S *= g.ng;
        int64_t nouter = batch;
        for (int q = 0; q < ax; ++q) nouter *= g.ng;
        int64_t nblk, nlines;
        if (S == 1) {
            nlines = nouter;
            nblk = (nlines + kLines - 1) / kLines;
        } else {
            nlines = nouter * S;
            nblk = nouter * (S / kLines);
        }
        C *p = (C *)grid;
        switch (logn) {
        case 4: k_fft_lines<T, 4, INV><<<(unsigned)nblk, 256, 0, s>>>(p, S, nlines); break;
        case 5: k_fft_lines<T, 5, INV><<<(unsigned)nblk, 256, 0, s>>>(p, S, nlines); break;
        case 6: k_fft_lines<T, 6, INV><<<(unsigned)nblk, 256, 0, s>>>(p, S, nlines); break;
        case 7: k_fft_lines<T, 7, INV><<<(unsigned)nblk, 256, 0, s>>>(p, S, nlines); break;
        case 8: k_fft_lines<T, 8, INV><<<(unsigned)nblk, 256, 0, s>>>(p, S, nlines); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

template <typename T>
hipError_t diag_t(const Group &G, int nrhs, void *grid, bool with_der, hipStream_t s)
{
    using C = typename Cplx<T>::type;
    const WindowGeom &g = G.g;
    int64_t total = (int64_t)G.nwin * nrhs * g.cells;
    unsigned nblk = (unsigned)((total + 255) / 256);
    C *spec = (C *)grid;
#define NFFTGP_DIAG(DD)                                                                        \
    if (with_der)                                                                              \
        k_diag<T, DD, true><<<nblk, 256, 0, s>>>(spec, G.desc, g.N, nrhs, g.cells, total);     \
    else                                                                                       \
        k_diag<T, DD, false><<<nblk, 256, 0, s>>>(spec, G.desc, g.N, nrhs, g.cells, total);
    switch (g.d) {
    case 1: NFFTGP_DIAG(1) break;
    case 2: NFFTGP_DIAG(2) break;
    case 3: NFFTGP_DIAG(3) break;
    default: return hipErrorInvalidValue;
    }
#undef NFFTGP_DIAG
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fft(int prec, const WindowGeom &g, void *grid, int batch, bool inverse,
                      hipStream_t s)
{
    if (prec == NFFTGP_F32)
        return inverse ? fft_t<float, true>(g, grid, batch, s) : fft_t<float, false>(g, grid, batch, s);
    return inverse ? fft_t<double, true>(g, grid, batch, s) : fft_t<double, false>(g, grid, batch, s);
}

hipError_t launch_diag(int prec, const Group &G, int nrhs, void *grid, bool with_der,
                       hipStream_t s)
{
    return prec == NFFTGP_F32 ? diag_t<float>(G, nrhs, grid, with_der, s)
                              : diag_t<double>(G, nrhs, grid, with_der, s);
}

}  // namespace nfftgp
