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
// Line transforms.  A line of n_g = P * Q points is transformed in two passes
// (the four-step factorisation n = Q n1 + n2, k = k1 + P k2): pass 1 takes,
// for each n2, the P-point DFT over n1 in registers and multiplies by
// w^(n2 k1); pass 2 takes, for each k1, the Q-point DFT over n2 in registers.
// One LDS exchange (padded rows) and one barrier separate the passes; the
// small DFTs are radix-2 in registers with constant twiddles.
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

// cos and sin of 2 pi e / 16
constexpr double kCos16[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                               0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                               -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                               0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
constexpr double kSin16[16] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                               1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                               0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                               -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};

// d * exp(-+ 2 pi i e / 16) (minus: forward, plus: INV); e is a constant after unrolling
template <typename T, bool INV>
__device__ __forceinline__ typename Cplx<T>::type rot16(typename Cplx<T>::type d, int e)
{
    using C = typename Cplx<T>::type;
    const T sg = INV ? T(1) : T(-1);
    C o;
    if (e == 0) return d;
    if (e == 8) {
        o.x = -d.x;
        o.y = -d.y;
        return o;
    }
    if (e == 4 || e == 12) {   // times sg * i (e = 4) or -sg * i (e = 12)
        const T s = e == 4 ? sg : -sg;
        o.x = -s * d.y;
        o.y = s * d.x;
        return o;
    }
    const T c = (T)kCos16[e], s = sg * (T)kSin16[e];
    o.x = d.x * c - d.y * s;
    o.y = d.x * s + d.y * c;
    return o;
}

constexpr int brev_c(int k, int bits)
{
    int r = 0;
    for (int i = 0; i < bits; ++i) r |= ((k >> i) & 1) << (bits - 1 - i);
    return r;
}

constexpr int log2c(int v) { return v <= 1 ? 0 : 1 + log2c(v / 2); }

// In-register DFT of P <= 16 points, natural order in and out (radix-2
// decimation in frequency, then the bit-reversal permutation by renaming).
template <typename T, int P, bool INV>
__device__ __forceinline__ void dft_reg(typename Cplx<T>::type (&x)[P])
{
    using C = typename Cplx<T>::type;
#pragma unroll
    for (int half = P / 2; half >= 1; half >>= 1) {
#pragma unroll
        for (int b = 0; b < P; b += 2 * half) {
#pragma unroll
            for (int j = 0; j < half; ++j) {
                const C u = x[b + j], v = x[b + j + half];
                C s, d;
                s.x = u.x + v.x;
                s.y = u.y + v.y;
                d.x = u.x - v.x;
                d.y = u.y - v.y;
                x[b + j] = s;
                x[b + j + half] = rot16<T, INV>(d, j * (8 / half));
            }
        }
    }
    C y[P];
#pragma unroll
    for (int k = 0; k < P; ++k) y[k] = x[brev_c(k, log2c(P))];
#pragma unroll
    for (int k = 0; k < P; ++k) x[k] = y[k];
}

template <int LOGN> struct Split {
    static constexpr int NG = 1 << LOGN;
    static constexpr int P = 1 << ((LOGN + 1) / 2);
    static constexpr int Q = NG / P;
    static constexpr int YP = P * (Q + 1) + 1;   // padded row of the exchange buffer
};

// Twiddles w^t = exp(-+ 2 pi i t / n_g), t < n_g / 2, evaluated in FP64.
template <typename T, int LOGN, bool INV>
__device__ __forceinline__ void make_tw(typename Cplx<T>::type *tw)
{
    constexpr int NG = 1 << LOGN;
    for (int t = threadIdx.x; t < NG / 2; t += blockDim.x) {
        double sn, cs;
        sincospi((INV ? 2.0 : -2.0) * (double)t / (double)NG, &sn, &cs);
        tw[t].x = (T)cs;
        tw[t].y = (T)sn;
    }
}

// Pass 1 for line ln, column n2: x[Q n1 + n2] from load(ln, n), P-point DFT,
// times w^(n2 k1), into the exchange row at (Q + 1) k1 + n2.
template <typename T, int LOGN, bool INV, typename Load>
__device__ __forceinline__ void pass1(int ln, int n2, Load &&load, typename Cplx<T>::type *ybuf,
                                      const typename Cplx<T>::type *tw)
{
    using C = typename Cplx<T>::type;
    using S = Split<LOGN>;
    C x[S::P];
#pragma unroll
    for (int n1 = 0; n1 < S::P; ++n1) x[n1] = load(ln, S::Q * n1 + n2, n1);
    dft_reg<T, S::P, INV>(x);
#pragma unroll
    for (int k1 = 1; k1 < S::P; ++k1) {
        const int e = (n2 * k1) & (S::NG - 1);
        C w = tw[e & (S::NG / 2 - 1)];
        if (e >= S::NG / 2) {
            w.x = -w.x;
            w.y = -w.y;
        }
        const C v = x[k1];
        x[k1].x = v.x * w.x - v.y * w.y;
        x[k1].y = v.x * w.y + v.y * w.x;
    }
    C *row = ybuf + ln * S::YP + n2;
#pragma unroll
    for (int k1 = 0; k1 < S::P; ++k1) row[(S::Q + 1) * k1] = x[k1];
}

// Pass 2 for line ln, row k1: Q-point DFT over n2; emit(ln, k1 + P k2, value).
template <typename T, int LOGN, bool INV, typename Emit>
__device__ __forceinline__ void pass2(int ln, int k1, const typename Cplx<T>::type *ybuf, Emit &&emit)
{
    using C = typename Cplx<T>::type;
    using S = Split<LOGN>;
    C y[S::Q];
    const C *row = ybuf + ln * S::YP + (S::Q + 1) * k1;
#pragma unroll
    for (int n2 = 0; n2 < S::Q; ++n2) y[n2] = row[n2];
    dft_reg<T, S::Q, INV>(y);
#pragma unroll
    for (int k2 = 0; k2 < S::Q; ++k2) emit(ln, k1 + S::P * k2, y[k2]);
}

// Both passes over nl lines (work-group-wide; contains barriers).  With
// LINE_FAST the thread index runs over lines first (strided axes, whose
// adjacent lines are adjacent in memory), otherwise over the column / row.
template <typename T, int LOGN, bool INV, bool LINE_FAST, typename Load, typename Emit>
__device__ __forceinline__ void fft_lines(int nl, Load &&load, Emit &&emit, typename Cplx<T>::type *ybuf,
                                          const typename Cplx<T>::type *tw)
{
    using S = Split<LOGN>;
    const int nt = blockDim.x;
    for (int t = threadIdx.x; t < nl * S::Q; t += nt) {
        const int ln = LINE_FAST ? t % nl : t / S::Q, c = LINE_FAST ? t / nl : t % S::Q;
        pass1<T, LOGN, INV>(ln, c, load, ybuf, tw);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nl * S::P; t += nt) {
        const int ln = LINE_FAST ? t % nl : t / S::P, r = LINE_FAST ? t / nl : t % S::P;
        pass2<T, LOGN, INV>(ln, r, ybuf, emit);
    }
    __syncthreads();
}

// 3-D grids with 2N <= 64: axes 2 and 1 of one slab (batch b, first index l0)
// in one work-group.  Forward (INV false): rows l1 in Omega are transformed
// along axis 2 (input Omega, kept F), then columns K2 in F along axis 1
// (input Omega, written F).  Inverse: columns K2 in F along axis 1 (input F,
// kept Omega), then rows l1 in Omega along axis 2 (input F, written Omega).
// Grid (on, batch); LDS: exchange rows [on][YP] and a natural-order buffer
// nat[on][NG + 1] (columns of the intermediate result, then the output).
template <typename T, int LOGN, bool INV>
__global__ void __launch_bounds__(512)
k_fft_slab(typename Cplx<T>::type *__restrict__ data, PruneGeom pg)
{
    using C = typename Cplx<T>::type;
    using S = Split<LOGN>;
    constexpr int NG = S::NG, NP = NG + 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *ybuf = reinterpret_cast<C *>(smem_raw);            // [on][YP]
    C *nat = ybuf + pg.on * S::YP;                         // [on][NG + 1]
    __shared__ C tw[NG / 2];
    make_tw<T, LOGN, INV>(tw);
    const int l0 = pg.olo + blockIdx.x;
    C *slab = data + (int64_t)blockIdx.y * pg.cells + (int64_t)l0 * NG * NG;
    const int on = pg.on, fn = pg.fn, olo = pg.olo, flo = pg.flo;
    C zero;
    zero.x = T(0);
    zero.y = T(0);
    if (!INV) {
        __syncthreads();   // twiddles
        // rows l1 = olo + j along axis 2: Omega in, F kept -> nat[c][l1]
        fft_lines<T, LOGN, false, false>(
            on,
            [&](int j, int k, int) { return cyc_has(olo, on, k, NG) ? slab[(olo + j) * NG + k] : zero; },
            [&](int j, int k2, C v) {
                if (cyc_has(flo, fn, k2, NG)) nat[((k2 - flo) & (NG - 1)) * NP + olo + j] = v;
            },
            ybuf, tw);
        // columns c (K2 in F) along axis 1: Omega in (zero elsewhere), F kept
        fft_lines<T, LOGN, false, false>(
            fn, [&](int c, int l1, int) { return cyc_has(olo, on, l1, NG) ? nat[c * NP + l1] : zero; },
            [&](int c, int k1, C v) {
                if (cyc_has(flo, fn, k1, NG)) nat[c * NP + k1] = v;
            },
            ybuf, tw);
        for (int idx = threadIdx.x; idx < fn * fn; idx += blockDim.x) {
            const int a = idx / fn, c = idx % fn;
            const int k1 = cyc_pos(flo, a, NG), k2 = cyc_pos(flo, c, NG);
            slab[k1 * NG + k2] = nat[c * NP + k1];
        }
    } else {
        // coalesced load of (K1 in F, K2 in F) into nat[c][k1]
        for (int idx = threadIdx.x; idx < fn * fn; idx += blockDim.x) {
            const int a = idx / fn, c = idx % fn;
            const int k1 = cyc_pos(flo, a, NG), k2 = cyc_pos(flo, c, NG);
            nat[c * NP + k1] = slab[k1 * NG + k2];
        }
        __syncthreads();
        // columns c along axis 1: F in, Omega kept -> nat[c][l1]
        fft_lines<T, LOGN, true, false>(
            fn, [&](int c, int k1, int) { return cyc_has(flo, fn, k1, NG) ? nat[c * NP + k1] : zero; },
            [&](int c, int l1, C v) {
                if (cyc_has(olo, on, l1, NG)) nat[c * NP + l1] = v;
            },
            ybuf, tw);
        // rows l1 = olo + j along axis 2: F in (from nat[c][l1]), Omega kept -> nat[j][l2]
        // (the row pass reads nat only in its first pass, which a barrier
        // separates from the writes of its second)
        fft_lines<T, LOGN, true, false>(
            on,
            [&](int j, int k2, int) {
                return cyc_has(flo, fn, k2, NG) ? nat[((k2 - flo) & (NG - 1)) * NP + olo + j] : zero;
            },
            [&](int j, int l2, C v) {
                if (cyc_has(olo, on, l2, NG)) nat[j * NP + l2] = v;
            },
            ybuf, tw);
        for (int idx = threadIdx.x; idx < on * on; idx += blockDim.x) {
            const int j = idx / on, c = idx % on;
            slab[(olo + j) * NG + olo + c] = nat[j * NP + olo + c];
        }
    }
}

// MODE 0: forward transform of axis ax (reads Omega, writes F);
// MODE 1: inverse transform of axis ax (reads F, writes Omega);
// MODE 2: axis 0 forward, diagonal, inverse (reads Omega, writes Omega; with
//         DER the diagonal is D + i D^der, so the kernel and derivative grids
//         come out as the real and imaginary parts).
// LPB lines per work-group of LPB * Q threads; the first pass reads the grid
// and the last writes it directly.
template <typename T, int LOGN, int LPB, int MODE, bool DER>
__global__ void __launch_bounds__(LPB * Split<LOGN>::Q)
k_fft_pruned(typename Cplx<T>::type *__restrict__ data, PruneGeom pg, int ax, int64_t nlines,
             int64_t lines_per_batch, const WinDesc *__restrict__ wd, int nrhs, int64_t der_off)
{
    using C = typename Cplx<T>::type;
    using Sp = Split<LOGN>;
    constexpr int NG = Sp::NG;
    __shared__ C ybuf[LPB * Sp::YP];
    __shared__ C spec[MODE == 2 ? LPB : 1][MODE == 2 ? NG + 1 : 1];
    __shared__ C twf[NG / 2];
    __shared__ C twi[MODE == 2 ? NG / 2 : 1];
    __shared__ int64_t s_base[LPB];
    __shared__ int s_ok[LPB];
    __shared__ int s_di[LPB];
    __shared__ int s_win[LPB];
    make_tw<T, LOGN, MODE == 1>(twf);
    if (MODE == 2) make_tw<T, LOGN, true>(twi);
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
    C zero;
    zero.x = T(0);
    zero.y = T(0);
    const bool in_om = MODE != 1;                    // input set: Omega or F
    const int ilo = in_om ? pg.olo : pg.flo, ilen = in_om ? pg.on : pg.fn;
    auto load = [&](int li, int k, int) {
        return (s_ok[li] && cyc_has(ilo, ilen, k, ng)) ? data[s_base[li] + (int64_t)k * S] : zero;
    };
    if constexpr (MODE != 2) {
        const int olo2 = MODE == 0 ? pg.flo : pg.olo, olen = MODE == 0 ? pg.fn : pg.on;
        auto emit = [&](int li, int k, C v) {
            if (s_ok[li] && cyc_has(olo2, olen, k, ng)) data[s_base[li] + (int64_t)k * S] = v;
        };
        if (S == 1)
            fft_lines<T, LOGN, MODE == 1, false>(LPB, load, emit, ybuf, twf);
        else
            fft_lines<T, LOGN, MODE == 1, true>(LPB, load, emit, ybuf, twf);
    } else {
        // MODE 2 (ax == 0, stride S): forward spectrum into spec, then per
        // block the diagonal at axis-0 frequency k times the line's offset in
        // the (N+1)^d diagonal, and the inverse transform
        // the diagonal values this thread's inverse first pass needs (one
        // task per thread: line li, column n2, frequencies Q n1 + n2) are
        // loaded before the forward transform, so their latency is hidden
        static_assert(LPB * Sp::Q >= 1, "");
        int64_t dstr0 = 1;
        for (int q = 1; q < pg.d; ++q) dstr0 *= (pg.N + 1);
        const int tli = S == 1 ? (int)threadIdx.x / Sp::Q : (int)threadIdx.x % LPB;
        const int tn2 = S == 1 ? (int)threadIdx.x % Sp::Q : (int)threadIdx.x / LPB;
        T dpre[DER ? 2 : 1][Sp::P];
#pragma unroll
        for (int pass = 0; pass < (DER ? 2 : 1); ++pass) {
            const WinDesc &w = wd[s_win[tli]];
            gmem<T> *D = (gmem<T> *)(pass == 0 ? w.Dk : w.Dder);
#pragma unroll
            for (int n1 = 0; n1 < Sp::P; ++n1) {
                const int k = Sp::Q * n1 + tn2;
                const int f = k < pg.N ? k : k - ng;
                const bool in = s_ok[tli] && f >= -pg.N / 2 && f <= pg.N / 2;
                dpre[pass][n1] = in ? D[(int64_t)(f + pg.N / 2) * dstr0 + s_di[tli]] : T(0);
            }
        }
        auto keep = [&](int li, int k, C v) { spec[li][k] = v; };
        if (S == 1)
            fft_lines<T, LOGN, false, false>(LPB, load, keep, ybuf, twf);
        else
            fft_lines<T, LOGN, false, true>(LPB, load, keep, ybuf, twf);
        // the spectrum of a real grid is Hermitian and D, D^der are real and
        // even, so D G^ and D^der G^ transform back to real grids: one inverse
        // of (D + i D^der) G^ gives the kernel grid in the real parts and the
        // derivative grid in the imaginary parts
        auto dload = [&](int li, int k, int n1) {
            const C v = spec[li][k];
            const T dv = dpre[0][n1];
            C o;
            if constexpr (DER) {
                const T dd = dpre[DER ? 1 : 0][n1];
                o.x = dv * v.x - dd * v.y;
                o.y = dv * v.y + dd * v.x;
            } else {
                o.x = dv * v.x;
                o.y = dv * v.y;
            }
            return o;
        };
        auto emit = [&](int li, int k, C v) {
            if (s_ok[li] && cyc_has(pg.olo, pg.on, k, ng)) data[s_base[li] + (int64_t)k * S] = v;
        };
        if (S == 1)
            fft_lines<T, LOGN, true, false>(LPB, dload, emit, ybuf, twi);
        else
            fft_lines<T, LOGN, true, true>(LPB, dload, emit, ybuf, twi);
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

// Lines per work-group: enough for 128 threads in the first pass; halved for
// FP64 at n_g >= 128 to stay within the static LDS limit.
template <typename T, int LOGN>
constexpr int lines_per_group()
{
    constexpr int NG = 1 << LOGN;
    constexpr int base = NG <= 32 ? 32 : (NG <= 128 ? 16 : 8);
    return (sizeof(T) == 8 && NG >= 128) ? base / 2 : base;
}

template <typename T, int LOGN, int MODE, bool DER>
hipError_t fft_launch(void *grid, const PruneGeom &pg, int ax, int64_t batch, const WinDesc *wd,
                      int nrhs, int64_t der_off, hipStream_t s)
{
    constexpr int LPB = lines_per_group<T, LOGN>();
    const int64_t lpb = lines_of(pg, ax);
    const int64_t nlines = batch * lpb;
    const unsigned nblk = (unsigned)((nlines + LPB - 1) / LPB);
    if (nblk == 0) return hipSuccess;
    k_fft_pruned<T, LOGN, LPB, MODE, DER><<<nblk, LPB * Split<LOGN>::Q, 0, s>>>(
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
template <typename T, int LOGN, bool INV>
hipError_t slab_go(const PruneGeom &pg, void *grid, int64_t batch, hipStream_t s)
{
    using C = typename Cplx<T>::type;
    using S = Split<LOGN>;
    const size_t shm = (size_t)pg.on * (S::YP + S::NG + 1) * sizeof(C);
    // one thread per (line, column) of the larger pass, whole waves, <= 512
    int nt = pg.on * (S::P > S::Q ? S::P : S::Q);
    nt = ((nt + 63) / 64) * 64;
    nt = nt > 512 ? 512 : nt;
    hipError_t e = hipFuncSetAttribute((const void *)k_fft_slab<T, LOGN, INV>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    k_fft_slab<T, LOGN, INV><<<dim3((unsigned)pg.on, (unsigned)batch), nt, shm, s>>>((C *)grid, pg);
    return hipGetLastError();
}

template <typename T, bool INV>
hipError_t slab_t(const Group &G, const PruneGeom &pg, void *grid, int64_t batch, hipStream_t s)
{
    switch (G.g.ng) {
    case 16: return slab_go<T, 4, INV>(pg, grid, batch, s);
    case 32: return slab_go<T, 5, INV>(pg, grid, batch, s);
    case 64: return slab_go<T, 6, INV>(pg, grid, batch, s);
    default: return hipErrorInvalidValue;
    }
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
    // one complex grid per window and vector: kernel and derivative grids in
    // its real and imaginary parts
    (void)with_der;
    const int64_t batch = (int64_t)G.nwin * nrhs;
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
