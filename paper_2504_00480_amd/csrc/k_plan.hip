// Plan-time kernels: per-window extent of the points, scaling into the box
// [-1/4, 1/4)^d (Sec. 3.1), grid coordinates, and a stable counting sort of
// the points by grid tile so that spreading and interpolation read them
// coalesced and tile by tile.
#include "nfftgp_impl.h"

namespace nfftgp {
namespace {

template <typename T>
__global__ void __launch_bounds__(256)
k_minmax_part(const T *__restrict__ X, int64_t n, int64_t ldx, int d, int f0, int f1, int f2,
              double *__restrict__ part, int *__restrict__ nanflag)
{
    __shared__ double slo[3][256], shi[3][256];
    const int feat[3] = {f0, f1, f2};
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int q = 0; q < d; ++q) {
            double v = (double)X[i * ldx + feat[q]];
            if (!(v == v) || v == INFINITY || v == -INFINITY) bad = 1;
            lo[q] = fmin(lo[q], v);
            hi[q] = fmax(hi[q], v);
        }
    }
    if (bad) atomicOr(nanflag, 1);
    for (int q = 0; q < 3; ++q) {
        slo[q][threadIdx.x] = lo[q];
        shi[q][threadIdx.x] = hi[q];
    }
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int q = 0; q < 3; ++q) {
                slo[q][threadIdx.x] = fmin(slo[q][threadIdx.x], slo[q][threadIdx.x + off]);
                shi[q][threadIdx.x] = fmax(shi[q][threadIdx.x], shi[q][threadIdx.x + off]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) {
            part[blockIdx.x * 6 + q] = slo[q][0];
            part[blockIdx.x * 6 + 3 + q] = shi[q][0];
        }
}

__global__ void k_minmax_final(const double *__restrict__ part, int nblk, int d,
                               double *__restrict__ out)
{
    int q = threadIdx.x;
    if (q >= d) return;
    double lo = INFINITY, hi = -INFINITY;
    for (int b = 0; b < nblk; ++b) {
        lo = fmin(lo, part[b * 6 + q]);
        hi = fmax(hi, part[b * 6 + 3 + q]);
    }
    out[q] = lo;
    out[d + q] = hi;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_coords(const T *__restrict__ X, int64_t n, int64_t ldx, int d, int f0, int f1, int f2,
         double c00, double c01, double c02, double c, int N, int tb, int nb,
         T *__restrict__ t_out, int *__restrict__ keys, int *__restrict__ boxflag)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int feat[3] = {f0, f1, f2};
    const double c0[3] = {c00, c01, c02};
    const double ng = 2.0 * N;
    int key = 0, bad = 0;
    for (int q = 0; q < d; ++q) {
        double xs = c * ((double)X[i * ldx + feat[q]] - c0[q]);   // scaled into the box
        if (!(xs >= -0.25 && xs < 0.25)) bad = 1;
        T t = (T)(ng * xs + (double)N);                             // grid units in [N/2, 3N/2)
        t_out[(int64_t)q * n + i] = t;
        int a = (int)floor((double)t);
        a = a < 0 ? 0 : (a > 2 * N - 1 ? 2 * N - 1 : a);
        key = key * tb + a % tb;   // cell inside its tile (first sort pass)
    }
    keys[i] = key;
    if (bad) atomicOr(boxflag, 1);
    (void)nb;
}

// Tile ("bin") key of sorted coordinates (second sort pass).
template <typename T>
__global__ void __launch_bounds__(256)
k_bin_keys(const T *__restrict__ t, int64_t n, int d, int ng, int tb, int nb, int *__restrict__ keys)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int key = 0;
    for (int q = 0; q < d; ++q) {
        int a = (int)floor((double)t[(int64_t)q * n + i]);
        a = a < 0 ? 0 : (a > ng - 1 ? ng - 1 : a);
        key = key * nb + a / tb;
    }
    keys[i] = key;
}

// Window weights of every sorted point, evaluated in FP64 from the stored
// coordinate: record j holds psi(t_q - l) for the 2m taps l = floor(t_q)-m+1+a
// of each dimension q (a = 0..2m-1), dimension-major; for d = 3 the first
// dimension's taps are rotated: tap a sits in slot (L + a) mod 2m, L being the
// first tap's position in the padded tile, so that the taps of one position
// class modulo a divisor of 2m sit in fixed slots for every point.  anchor[j] packs the
// cell floor(t) (row-major over the (2N)^d grid); lpos[j] packs the position
// of the first tap inside the point's padded tile (edge pd = tb + 2m, origin
// one tile edge tb * bin - m): bits 0-19 the row-major offset, bits 20-26 the
// first coordinate.  Both get bit 31 when the next point has another cell, so
// that spreading can flush per run of points.
template <typename T>
__global__ void __launch_bounds__(256)
k_weights(const T *__restrict__ t, int64_t n, int d, int m, int ng, int tb, int pd, double beta,
          double knorm, T *__restrict__ rec, int *__restrict__ anchor, int *__restrict__ lpos)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int tw = 2 * m;
    int an = 0, lin = 0, l0 = 0;
    for (int q = 0; q < d; ++q) {
        double tq = (double)t[(int64_t)q * n + i];
        double fl = floor(tq);
        const int c = (int)fl;
        an = an * ng + c;
        const int L = c % tb + 1;   // first tap - padded tile origin = c - tb * bin + 1
        lin = lin * pd + L;
        if (q == 0) l0 = L;
        for (int a = 0; a < tw; ++a) {
            double u = tq - (fl - (m - 1) + a);
            double s2 = (double)m * m - u * u;
            s2 = s2 > 0.0 ? s2 : 0.0;
            double sq = sqrt(s2), z = beta * sq;
            double r = z < 1e-6 ? beta * (1.0 + z * z / 6.0) : sinh(z) / sq;
            // d = 3, first dimension: stored rotated by the first tap's tile
            // position, at (L + a) mod 2m
            const int slot = (d == 3 && q == 0) ? (L + a) % tw : a;
            rec[(i * d + q) * tw + slot] = (T)(r * knorm);
        }
    }
    anchor[i] = an;
    lpos[i] = lin | (l0 << 20);
}

// counts[tile * tb + row] = points of the tile whose first cell coordinate
// inside the tile is row (3-D).  The points are sorted by tile and, inside a
// tile, by cell with the first coordinate slowest, so each (tile, row) key is
// one contiguous range [s, e): its first point adds -s and its last e, two
// atomics per range instead of one per point.
__device__ __forceinline__ int row_key(const int *anchor, int64_t i, int ng, int tb, int nb)
{
    const int a = anchor[i] & 0x7fffffff;
    const int c2 = a % ng, c1 = (a / ng) % ng, c0 = a / (ng * ng);
    const int bin = ((c0 / tb) * nb + c1 / tb) * nb + c2 / tb;
    return bin * tb + c0 % tb;
}

__global__ void __launch_bounds__(256)
k_row_counts(const int *__restrict__ anchor, int64_t n, int ng, int tb, int nb, int *__restrict__ counts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int key = row_key(anchor, i, ng, tb, nb);
    if (i == 0 || row_key(anchor, i - 1, ng, tb, nb) != key) atomicAdd(&counts[key], -(int)i);
    if (i == n - 1 || row_key(anchor, i + 1, ng, tb, nb) != key) atomicAdd(&counts[key], (int)(i + 1));
}

__global__ void __launch_bounds__(256)
k_run_ends(int *__restrict__ anchor, int *__restrict__ lpos, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // each thread writes only its own entry; the neighbour may already carry
    // its flag, so compare the cell bits only
    const int a = anchor[i] & 0x7fffffff;
    const bool last = (i == n - 1) || ((anchor[i + 1] & 0x7fffffff) != a);
    if (last) {
        anchor[i] = a | (int)0x80000000u;
        lpos[i] = lpos[i] | (int)0x80000000u;
    }
}

// ---- stable counting sort ------------------------------------------------
// Block b owns points [b*kSortBlock, (b+1)*kSortBlock).  hist is bin-major:
// hist[bin * nblk + b], so an exclusive scan of hist gives the first sorted
// position of every (bin, block) pair, with blocks of one bin in point order.
__global__ void __launch_bounds__(256)
k_block_hist(const int *__restrict__ keys, int64_t n, int nbins, int nblk, int *__restrict__ hist)
{
    extern __shared__ int sh[];
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) sh[b] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortBlock;
    for (int k = threadIdx.x; k < kSortBlock; k += blockDim.x) {
        int64_t i = base + k;
        if (i < n) atomicAdd(&sh[keys[i]], 1);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += blockDim.x)
        hist[(int64_t)b * nblk + blockIdx.x] = sh[b];
}

// Three-phase exclusive scan of len ints (chunk of 1024 per block).
__global__ void __launch_bounds__(1024)
k_scan_chunks(const int *__restrict__ in, int64_t len, int *__restrict__ chunk_sum)
{
    __shared__ int s[1024];
    int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    s[threadIdx.x] = i < len ? in[i] : 0;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) chunk_sum[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(1024)
k_scan_sums(int *__restrict__ chunk_sum, int nchunk)
{
    // single block, sequential over groups of 1024 with a running carry
    __shared__ int s[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nchunk; base += 1024) {
        int i = base + threadIdx.x;
        int v = i < nchunk ? chunk_sum[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int t = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nchunk) chunk_sum[i] = carry + s[threadIdx.x] - v;   // exclusive
        __syncthreads();
        if (threadIdx.x == 1023) carry += s[1023];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(1024)
k_scan_apply(int *__restrict__ data, int64_t len, const int *__restrict__ chunk_off)
{
    __shared__ int s[1024];
    int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    int v = i < len ? data[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int t = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < len) data[i] = chunk_off[blockIdx.x] + s[threadIdx.x] - v;
}

// Stable scatter: within a block, points are placed in index order.  The
// rank of a point among equal keys of its 256-point round is counted by
// brute force; a per-bin LDS counter carries the rounds.
template <typename T>
__global__ void __launch_bounds__(256)
k_scatter(const int *__restrict__ keys, int64_t n, int nbins, int nblk, int d,
          const int *__restrict__ offs, const int *__restrict__ ids_in, const T *__restrict__ t_in,
          int *__restrict__ perm, T *__restrict__ t_sorted)
{
    extern __shared__ int sh[];
    int *cnt = sh;               // nbins
    int *rk = sh + nbins;        // 256 keys of the current round
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) cnt[b] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortBlock;
    for (int r0 = 0; r0 < kSortBlock; r0 += 256) {
        int64_t i = base + r0 + threadIdx.x;
        int key = i < n ? keys[i] : -1;
        rk[threadIdx.x] = key;
        __syncthreads();
        int rank = 0;
        for (int t = 0; t < (int)threadIdx.x; ++t) rank += (rk[t] == key);
        int pos = 0;
        if (key >= 0) pos = offs[(int64_t)key * nblk + blockIdx.x] + cnt[key] + rank;
        __syncthreads();
        if (key >= 0) {
            atomicAdd(&cnt[key], 1);
            perm[pos] = ids_in ? ids_in[i] : (int)i;
            for (int q = 0; q < d; ++q) t_sorted[(int64_t)q * n + pos] = t_in[(int64_t)q * n + i];
        }
        __syncthreads();
    }
}

__global__ void k_bin_start(const int *__restrict__ offs, int nbins, int nblk, int64_t n,
                            int *__restrict__ bin_start)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nbins) bin_start[b] = offs[(int64_t)b * nblk];
    if (b == nbins) bin_start[b] = (int)n;
}

}  // namespace

hipError_t launch_minmax(int prec, const void *X, int64_t n, int64_t ldx, int d, const int *feat,
                         double *part, double *out, int *nanflag, hipStream_t s)
{
    int f[3] = {feat[0], d > 1 ? feat[1] : 0, d > 2 ? feat[2] : 0};
    if (prec == NFFTGP_F32)
        k_minmax_part<float><<<kPartBlocks, 256, 0, s>>>((const float *)X, n, ldx, d, f[0], f[1], f[2],
                                                         part, nanflag);
    else
        k_minmax_part<double><<<kPartBlocks, 256, 0, s>>>((const double *)X, n, ldx, d, f[0], f[1],
                                                          f[2], part, nanflag);
    k_minmax_final<<<1, 64, 0, s>>>(part, kPartBlocks, d, out);
    return hipGetLastError();
}

hipError_t launch_coords(int prec, const void *X, int64_t n, int64_t ldx, int d, const int *feat,
                         const double *c0, double c, const WindowGeom &g, void *t_out, int *keys,
                         int *boxflag, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    int f[3] = {feat[0], d > 1 ? feat[1] : 0, d > 2 ? feat[2] : 0};
    double cc[3] = {c0[0], d > 1 ? c0[1] : 0.0, d > 2 ? c0[2] : 0.0};
    unsigned nblk = (unsigned)((n + 255) / 256);
    if (prec == NFFTGP_F32)
        k_coords<float><<<nblk, 256, 0, s>>>((const float *)X, n, ldx, d, f[0], f[1], f[2], cc[0],
                                             cc[1], cc[2], c, g.N, g.tb, g.nb, (float *)t_out, keys,
                                             boxflag);
    else
        k_coords<double><<<nblk, 256, 0, s>>>((const double *)X, n, ldx, d, f[0], f[1], f[2], cc[0],
                                              cc[1], cc[2], c, g.N, g.tb, g.nb, (double *)t_out,
                                              keys, boxflag);
    return hipGetLastError();
}

int64_t scan_scratch_ints(int64_t len) { return (len + 1023) / 1024 + 1; }

hipError_t launch_sort(int prec, int64_t n, int d, int nbins, const int *keys, const int *ids_in,
                       const void *t_in, int *hist, int *scan_tmp, int *perm, void *t_sorted,
                       int *bin_start, hipStream_t s)
{
    int nblk = (int)((n + kSortBlock - 1) / kSortBlock);
    if (nblk == 0) nblk = 1;
    int64_t len = (int64_t)nbins * nblk;
    if (n > 0)
        k_block_hist<<<nblk, 256, nbins * sizeof(int), s>>>(keys, n, nbins, nblk, hist);
    else
        hipMemsetAsync(hist, 0, len * sizeof(int), s);
    int nchunk = (int)((len + 1023) / 1024);
    k_scan_chunks<<<nchunk, 1024, 0, s>>>(hist, len, scan_tmp);
    k_scan_sums<<<1, 1024, 0, s>>>(scan_tmp, nchunk);
    k_scan_apply<<<nchunk, 1024, 0, s>>>(hist, len, scan_tmp);
    if (n > 0) {
        size_t shm = (nbins + 256) * sizeof(int);
        if (prec == NFFTGP_F32)
            k_scatter<float><<<nblk, 256, shm, s>>>(keys, n, nbins, nblk, d, hist, ids_in,
                                                    (const float *)t_in, perm, (float *)t_sorted);
        else
            k_scatter<double><<<nblk, 256, shm, s>>>(keys, n, nbins, nblk, d, hist, ids_in,
                                                     (const double *)t_in, perm,
                                                     (double *)t_sorted);
    }
    k_bin_start<<<(nbins + 1 + 255) / 256, 256, 0, s>>>(hist, nbins, nblk, n, bin_start);
    return hipGetLastError();
}

hipError_t launch_bin_keys(int prec, const void *t, int64_t n, const WindowGeom &g, int *keys,
                           hipStream_t s)
{
    if (n == 0) return hipSuccess;
    unsigned nblk = (unsigned)((n + 255) / 256);
    if (prec == NFFTGP_F32)
        k_bin_keys<float><<<nblk, 256, 0, s>>>((const float *)t, n, g.d, g.ng, g.tb, g.nb, keys);
    else
        k_bin_keys<double><<<nblk, 256, 0, s>>>((const double *)t, n, g.d, g.ng, g.tb, g.nb, keys);
    return hipGetLastError();
}

hipError_t launch_row_counts(const int *anchor, int64_t n, const WindowGeom &g, int *counts,
                             hipStream_t s)
{
    if (n == 0 || g.d != 3) return hipSuccess;
    k_row_counts<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(anchor, n, g.ng, g.tb, g.nb, counts);
    return hipGetLastError();
}

hipError_t launch_weights(int prec, const void *t, int64_t n, const WindowGeom &g, int m,
                          double knorm, void *rec, int *anchor, int *lpos, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    unsigned nblk = (unsigned)((n + 255) / 256);
    if (prec == NFFTGP_F32)
        k_weights<float><<<nblk, 256, 0, s>>>((const float *)t, n, g.d, m, g.ng, g.tb, g.pd, kb_beta(),
                                              knorm, (float *)rec, anchor, lpos);
    else
        k_weights<double><<<nblk, 256, 0, s>>>((const double *)t, n, g.d, m, g.ng, g.tb, g.pd,
                                               kb_beta(), knorm, (double *)rec, anchor, lpos);
    k_run_ends<<<nblk, 256, 0, s>>>(anchor, lpos, n);
    return hipGetLastError();
}

}  // namespace nfftgp
