// Grid kernels of the fast summation (Sec. 3.1 eq. Fourier_sum; Appendix A):
//
//   spreading      g_l = sum_j v_j psi(t_j - l)          (adjoint NFFT, gridding)
//   fold           deterministic sum of the per-tile partial grids
//   interpolation  h_i = sum_l G_l psi(t_i - l)          (NFFT, sparse window sums)
//   assembly       sigma_f^2 sum_s h^(s) + sigma_eps^2 v and derivative blocks
//
// Coordinates t are in grid units (t = 2N x~ + N, x~ in [-1/4, 1/4)), so a
// point touches the 2m cells floor(t)-m+1 .. floor(t)+m per dimension.  psi is
// the Kaiser-Bessel window of Appendix A in grid units, normalised so that its
// Fourier coefficient at frequency 0 is 1 / (2N); the plan stores psi at the
// 2m taps of every point (record `rec`, dimension-major; for d = 3 the first
// dimension's taps rotated, tap a in slot (L + a) mod 2m with L the first
// tap's position in the padded tile).
//
// All windows of one group (same dimension and bandwidth) go through each
// kernel in a single launch: work items (subproblems, tiles, grid cells) of the
// group's windows are concatenated, and a per-window descriptor gives each
// work item its window's point data.  A subproblem is a run of points of one
// tile ("bin", tb cells per dimension) in the window's sorted order.
#include "nfftgp_impl.h"
#include "nfftgp_dev.h"
#include "nfftgp_coef_sep.h"

#include <cstdint>
#include <string>
#include <cstdlib>
#include <type_traits>

namespace nfftgp {
namespace {

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

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
// One work-group of W waves per subproblem and chunk of R vectors.  Points
// arrive sorted by cell inside their tile, so consecutive points often share
// the cell floor(t) and therefore all (2m)^d target cells.  Contributions of
// such a run are accumulated in registers: for d = 3, lane (b, c) of a wave
// owns the tap column (b, c) and keeps values along the first dimension; for
// d = 2 a lane owns tap (a, b), for d = 1 tap a.  The run is added to the
// LDS tile once, after its last point.  The W waves of a group walk the same
// points and share one tile: wave w handles the first-dimension taps whose
// position in the padded tile is w modulo W, so no two waves ever touch the
// same cell.  Within a flush every lane touches a distinct cell and the
// flushes of one wave are ordered, so the tile is updated with plain loads and
// stores and the result does not depend on scheduling.
//
// The points' weights and vector values are staged in LDS in chunks of 64,
// transposed (tap-major, point-minor), so one 16-byte read gives a value for
// four consecutive points; the first-dimension weights of a 3-D point are
// stored rotated by its tile position (slot (L + a) mod 2m for tap a), so
// wave w finds its taps in the fixed slots w, w + W, ... for every point.  Points are taken four at a time whatever the run boundaries
// (one ballot over the run-end flags of the chunk gives them); the reads of
// the next four are issued before the current four are accumulated and their
// runs flushed.
template <typename T, int D, int M, int R, int W>
__global__ void __launch_bounds__(64 * W)
k_spread(const WinDesc *__restrict__ wd, const int *__restrict__ sub_win,
         const int *__restrict__ sub_start, const int *__restrict__ sub_count,
         const T *__restrict__ V, int64_t ldv, int nrhs, int pd, T *__restrict__ tilebuf)
{
    constexpr int TW = 2 * M;
    constexpr int RS = D * TW;                                  // weights per point
    constexpr int NITEM = D == 1 ? TW : TW * TW;                // lane work items
    constexpr int NG = (NITEM + 63) / 64;
    static_assert(D == 3 || W == 1, "tap splitting across waves is for d = 3");
    static_assert(TW % W == 0, "waves must divide the taps");
    constexpr int NA = D == 3 ? TW / W : 1;                     // registers per item
    constexpr int CH = 64;                                      // points staged per chunk
    constexpr int CP = CH + 4;                                  // row pitch (conflict-free 16-byte reads)
    constexpr int NQ = D == 3 ? 3 : D;                          // staged weight rows of TW
    using T4 = typename std::conditional<sizeof(T) == 4, float4, double4>::type;
    // rows: [0, TW) first-dimension taps rotated (d = 3: residue rho * NA + k),
    // then the (b) and (c) taps; vector values after them
    __shared__ __align__(16) T s_w[NQ * TW * CP];
    __shared__ __align__(16) T s_v[R * CP];
    __shared__ int s_lp[CH];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tiles = reinterpret_cast<T *>(smem_raw);
    int pc = pd;
    for (int q = 1; q < D; ++q) pc *= pd;
    const int sq = xcd_item(blockIdx.x, gridDim.x), r0 = blockIdx.y * R;
    const WinDesc &win = wd[sub_win[sq]];
    gmem<T> *rec = (gmem<T> *)win.rec;
    gmem<int> *lpos = (gmem<int> *)win.lpos;
    gmem<int> *perm = (gmem<int> *)win.perm;
    const int start = sub_start[sq], cnt = sub_count[sq];
    const int end = start + cnt;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < R * pc; i += 64 * W) tiles[i] = T(0);
    // per lane: item indices and the item's offset inside the padded tile
    int i0[NG], i1[NG], off[NG];
    bool act[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int it = lane + 64 * g;
        act[g] = it < NITEM;
        const int itc = act[g] ? it : 0;
        i0[g] = D == 1 ? itc : itc / TW;
        i1[g] = D == 1 ? 0 : itc % TW;
        off[g] = D == 3 ? i0[g] * pd + i1[g] : (D == 2 ? i0[g] * pd + i1[g] : i0[g]);
    }
    const int pd2 = D == 3 ? pd * pd : 0;
    T acc[NG][NA][R];
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int k = 0; k < NA; ++k)
#pragma unroll
            for (int r = 0; r < R; ++r) acc[g][k][r] = T(0);
    const int nr = min(R, nrhs - r0);
    // the next chunk's global data is loaded into registers while the current
    // chunk is processed
    constexpr int NT = 64 * W;
    constexpr int NREC = (CH * RS + NT - 1) / NT, NV = (CH * R + NT - 1) / NT;
    T g_rec[NREC], g_v[NV];
    int g_lp = 0;
    auto fetch = [&](int cb) {
        const int nc = min(CH, end - cb);
#pragma unroll
        for (int k = 0; k < NREC; ++k) {
            const int i = tid + k * NT;
            const bool in = i < nc * RS;
            g_rec[k] = in ? rec[(int64_t)cb * RS + i] : T(0);
        }
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int i = tid + k * NT;
            const int u = i / R, r = i % R;
            g_v[k] = (i < nc * R && r < nr) ? V[(int64_t)perm[cb + u] * ldv + r0 + r] : T(0);
        }
        g_lp = tid < nc ? lpos[cb + tid] : 0;
    };
    if (cnt > 0) fetch(start);
    for (int cb = start; cb < end; cb += CH) {
        const int nc = min(CH, end - cb);
        __syncthreads();   // tiles cleared / previous chunk consumed
#pragma unroll
        for (int k = 0; k < NREC; ++k) {
            const int i = tid + k * NT;
            if (i < CH * RS) {
                const int u = i / RS, e = i % RS;   // weight slot e of point u -> row e
                s_w[e * CP + u] = g_rec[k];
            }
        }
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int i = tid + k * NT;
            if (i < CH * R) s_v[(i % R) * CP + i / R] = g_v[k];
        }
        if (tid < CH) s_lp[tid] = g_lp;
        __syncthreads();
        if (cb + CH < end) fetch(cb + CH);
        // lane u keeps point u's tile position; run ends of the chunk (the
        // subproblem's last point ends a run)
        const int my_lp = lane < nc ? s_lp[lane] : 0;
        const bool isend = lane < nc && (my_lp < 0 || cb + lane == end - 1);
        const unsigned long long ends = __ballot(isend);
        // values of four points u .. u + 3 (16-byte reads)
        struct Grp {
            T w0[NA][4], wa[NG][4], wb[NG][4], v[R][4];
        };
        auto load = [&](Grp &G4, int u) {
#pragma unroll
            for (int k = 0; k < NA; ++k) {
                if (D == 3) {
                    const T4 x = *reinterpret_cast<const T4 *>(s_w + (wave + k * W) * CP + u);
                    G4.w0[k][0] = x.x; G4.w0[k][1] = x.y; G4.w0[k][2] = x.z; G4.w0[k][3] = x.w;
                } else {
                    G4.w0[k][0] = G4.w0[k][1] = G4.w0[k][2] = G4.w0[k][3] = T(1);
                }
            }
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                // d = 3: rows TW + b and 2 TW + c; d = 2: rows a and TW + b; d = 1: row a
                const int ra = (D == 3 ? TW : 0) + i0[g];
                const T4 x = *reinterpret_cast<const T4 *>(s_w + ra * CP + u);
                G4.wa[g][0] = x.x; G4.wa[g][1] = x.y; G4.wa[g][2] = x.z; G4.wa[g][3] = x.w;
                if (D > 1) {
                    const int rb = (D == 3 ? 2 * TW : TW) + i1[g];
                    const T4 y = *reinterpret_cast<const T4 *>(s_w + rb * CP + u);
                    G4.wb[g][0] = y.x; G4.wb[g][1] = y.y; G4.wb[g][2] = y.z; G4.wb[g][3] = y.w;
                } else {
                    G4.wb[g][0] = G4.wb[g][1] = G4.wb[g][2] = G4.wb[g][3] = T(1);
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const T4 x = *reinterpret_cast<const T4 *>(s_v + r * CP + u);
                G4.v[r][0] = x.x; G4.v[r][1] = x.y; G4.v[r][2] = x.z; G4.v[r][3] = x.w;
            }
        };
        Grp cur, nxt;
        load(cur, 0);
        for (int u = 0; u < nc; u += 4) {
            if (u + 4 < nc) load(nxt, u + 4);
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                if (u + p < nc) {
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        const T wbc = cur.wa[g][p] * cur.wb[g][p];
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            const T z = wbc * cur.v[r][p];
#pragma unroll
                            for (int k = 0; k < NA; ++k) acc[g][k][r] += cur.w0[k][p] * z;
                        }
                    }
                    if ((ends >> (u + p)) & 1ull) {
                        // flush the run: all reads first (distinct cells), then
                        // the writes
                        // register k holds slot w + kW, i.e. tap (w + kW - L) mod 2m
                        const int lp = __builtin_amdgcn_readlane(my_lp, u + p) & 0x7fffffff;
                        const int base = lp & 0xfffff, L = lp >> 20;
                        int koff[NA];
#pragma unroll
                        for (int k = 0; k < NA; ++k)
                            koff[k] = D == 3 ? (((wave + k * W - L) % TW + TW) % TW) * pd2 : 0;
                        T old[NG][NA][R];
#pragma unroll
                        for (int g = 0; g < NG; ++g)
#pragma unroll
                            for (int k = 0; k < NA; ++k)
#pragma unroll
                                for (int r = 0; r < R; ++r)
                                    old[g][k][r] = act[g] ? tiles[r * pc + base + koff[k] + off[g]] : T(0);
#pragma unroll
                        for (int g = 0; g < NG; ++g) {
                            if (act[g]) {
#pragma unroll
                                for (int k = 0; k < NA; ++k) {
                                    const int idx = base + koff[k] + off[g];
#pragma unroll
                                    for (int r = 0; r < R; ++r) tiles[r * pc + idx] = old[g][k][r] + acc[g][k][r];
                                }
                            }
                        }
#pragma unroll
                        for (int g = 0; g < NG; ++g)
#pragma unroll
                            for (int k = 0; k < NA; ++k)
#pragma unroll
                                for (int r = 0; r < R; ++r) acc[g][k][r] = T(0);
                    }
                }
            }
            cur = nxt;
        }
    }
    __syncthreads();
    for (int r = 0; r < nr; ++r) {
        T *out = tilebuf + ((int64_t)sq * nrhs + r0 + r) * pc;
        for (int i = tid; i < pc; i += 64 * W) out[i] = tiles[r * pc + i];
    }
}

// Run-ordered form of the same spreading (selectable per window group): the
// points' weights are staged point-major, and each run of equal cells is
// accumulated in groups of four points inside the run, then flushed.  It holds
// fewer registers than the four-point form above, which pays off when a
// work-group carries several vectors and runs are long.
template <typename T, int D, int M, int R, int W>
__global__ void __launch_bounds__(64 * W)
k_spread_run(const WinDesc *__restrict__ wd, const int *__restrict__ sub_win,
         const int *__restrict__ sub_start, const int *__restrict__ sub_count,
         const T *__restrict__ V, int64_t ldv, int nrhs, int pd, T *__restrict__ tilebuf)
{
    constexpr int TW = 2 * M;
    constexpr int RS = D * TW;                                  // weights per point
    constexpr int NITEM = D == 1 ? TW : TW * TW;                // lane work items
    constexpr int NG = (NITEM + 63) / 64;
    static_assert(D == 3 || W == 1, "tap splitting across waves is for d = 3");
    static_assert(TW % W == 0, "waves must divide the taps");
    constexpr int NA = D == 3 ? TW / W : 1;                     // registers per item
    constexpr int CH = 64;                                      // points staged per chunk
    __shared__ T s_rec[CH * RS];
    __shared__ T s_v[CH * R];
    __shared__ int s_lp[CH];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tiles = reinterpret_cast<T *>(smem_raw);
    int pc = pd;
    for (int q = 1; q < D; ++q) pc *= pd;
    const int sq = xcd_item(blockIdx.x, gridDim.x), r0 = blockIdx.y * R;
    const WinDesc &win = wd[sub_win[sq]];
    gmem<T> *rec = (gmem<T> *)win.rec;
    gmem<int> *lpos = (gmem<int> *)win.lpos;
    gmem<int> *perm = (gmem<int> *)win.perm;
    const int start = sub_start[sq], cnt = sub_count[sq];
    const int end = start + cnt;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < R * pc; i += 64 * W) tiles[i] = T(0);
    // per lane: item indices and the item's offset inside the padded tile
    int i0[NG], i1[NG], off[NG];
    bool act[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int it = lane + 64 * g;
        act[g] = it < NITEM;
        const int itc = act[g] ? it : 0;
        i0[g] = D == 1 ? itc : itc / TW;
        i1[g] = D == 1 ? 0 : itc % TW;
        off[g] = D == 3 ? i0[g] * pd + i1[g] : (D == 2 ? i0[g] * pd + i1[g] : i0[g]);
    }
    const int pd2 = D == 3 ? pd * pd : 0;
    T acc[NG][NA][R];
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int k = 0; k < NA; ++k)
#pragma unroll
            for (int r = 0; r < R; ++r) acc[g][k][r] = T(0);
    const int nr = min(R, nrhs - r0);
    // the next chunk's global data is loaded into registers while the current
    // chunk is processed
    constexpr int NT = 64 * W;
    constexpr int NREC = (CH * RS + NT - 1) / NT, NV = (CH * R + NT - 1) / NT;
    T g_rec[NREC], g_v[NV];
    int g_lp = 0;
    auto fetch = [&](int cb) {
        const int nc = min(CH, end - cb);
#pragma unroll
        for (int k = 0; k < NREC; ++k) {
            const int i = tid + k * NT;
            g_rec[k] = i < nc * RS ? rec[(int64_t)cb * RS + i] : T(0);
        }
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int i = tid + k * NT;
            const int u = i / R, r = i % R;
            g_v[k] = (i < nc * R && r < nr) ? V[(int64_t)perm[cb + u] * ldv + r0 + r] : T(0);
        }
        g_lp = tid < nc ? lpos[cb + tid] : 0;
    };
    if (cnt > 0) fetch(start);
    for (int cb = start; cb < end; cb += CH) {
        const int nc = min(CH, end - cb);
        __syncthreads();   // tiles cleared / previous chunk consumed
#pragma unroll
        for (int k = 0; k < NREC; ++k) {
            const int i = tid + k * NT;
            if (i < CH * RS) s_rec[i] = g_rec[k];
        }
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int i = tid + k * NT;
            if (i < CH * R) s_v[i] = g_v[k];
        }
        if (tid < CH) s_lp[tid] = g_lp;
        __syncthreads();
        if (cb + CH < end) fetch(cb + CH);
        // run ends inside this chunk (the subproblem's last point ends a run)
        // lane u keeps point u's tile position; a run reads it with readlane
        const int my_lp = lane < nc ? s_lp[lane] : 0;
        const bool isend = lane < nc && (my_lp < 0 || cb + lane == end - 1);
        const unsigned long long ends = __ballot(isend);
        int u0 = 0;
        while (u0 < nc) {
            const unsigned long long rest = ends >> u0;
            const bool flush = rest != 0ull;
            const int u1 = flush ? u0 + (int)__builtin_ctzll(rest) : nc - 1;
            const int lp = __builtin_amdgcn_readlane(my_lp, u0) & 0x7fffffff;
            // points are accumulated in groups of 4 while the run has that many
            // left, then one by one: the LDS reads of a group are issued
            // together, so one wait covers the group
            auto accumulate = [&](auto pu_tag, int u) {
                constexpr int PU = decltype(pu_tag)::value;
                T v[PU][R], w0[PU][NA], w1[PU][NG], w2[PU][NG];
#pragma unroll
                for (int p = 0; p < PU; ++p) {
                    const T *rp = s_rec + (u + p) * RS;
#pragma unroll
                    for (int r = 0; r < R; ++r) v[p][r] = s_v[(u + p) * R + r];
#pragma unroll
                    for (int k = 0; k < NA; ++k) w0[p][k] = D == 3 ? rp[wave + k * W] : T(1);
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        if (D == 3) {
                            w1[p][g] = rp[TW + i0[g]];
                            w2[p][g] = rp[2 * TW + i1[g]];
                        } else if (D == 2) {
                            w1[p][g] = rp[i0[g]];
                            w2[p][g] = rp[TW + i1[g]];
                        } else {
                            w1[p][g] = rp[i0[g]];
                            w2[p][g] = T(1);
                        }
                    }
                }
#pragma unroll
                for (int p = 0; p < PU; ++p)
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        const T wbc = w1[p][g] * w2[p][g];
                        T z[R];
#pragma unroll
                        for (int r = 0; r < R; ++r) z[r] = wbc * v[p][r];
#pragma unroll
                        for (int k = 0; k < NA; ++k)
#pragma unroll
                            for (int r = 0; r < R; ++r) acc[g][k][r] += w0[p][k] * z[r];
                    }
            };
            int u = u0;
            for (; u + 3 <= u1; u += 4) accumulate(std::integral_constant<int, 4>(), u);
            for (; u <= u1; ++u) accumulate(std::integral_constant<int, 1>(), u);
            if (flush) {
                // all reads of the flush first (distinct cells), then the
                // writes: one LDS wait per run
                // register k holds slot w + kW, i.e. tap (w + kW - L) mod 2m
                const int base = lp & 0xfffff, L = lp >> 20;
                int koff[NA];
#pragma unroll
                for (int k = 0; k < NA; ++k) koff[k] = D == 3 ? (((wave + k * W - L) % TW + TW) % TW) * pd2 : 0;
                T old[NG][NA][R];
#pragma unroll
                for (int g = 0; g < NG; ++g)
#pragma unroll
                    for (int k = 0; k < NA; ++k)
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            old[g][k][r] = act[g] ? tiles[r * pc + base + koff[k] + off[g]] : T(0);
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    if (act[g]) {
#pragma unroll
                        for (int k = 0; k < NA; ++k) {
                            const int idx = base + koff[k] + off[g];
#pragma unroll
                            for (int r = 0; r < R; ++r) tiles[r * pc + idx] = old[g][k][r] + acc[g][k][r];
                        }
                    }
                }
#pragma unroll
                for (int g = 0; g < NG; ++g)
#pragma unroll
                    for (int k = 0; k < NA; ++k)
#pragma unroll
                        for (int r = 0; r < R; ++r) acc[g][k][r] = T(0);
            }
            u0 = u1 + 1;
        }
    }
    __syncthreads();
    for (int r = 0; r < nr; ++r) {
        T *out = tilebuf + ((int64_t)sq * nrhs + r0 + r) * pc;
        for (int i = tid; i < pc; i += 64 * W) out[i] = tiles[r * pc + i];
    }
}

// Matrix-core form of 3-D FP32 spreading.  All points of a run share the
// cell floor(t), so the run's contribution to the (2m)^3 target cells of R
// vectors is one dense contraction over the run's points p:
//
//   T[(b, c), (a, r)] = sum_p  w1_p[b] w2_p[c]  *  w0_p[a] v_p[r],
//
// rows (b, c) = TW^2 tap pairs of the second and third dimension, columns
// (a, r) = first-dimension tap times vector.  It runs on
// v_mfma_f32_16x16x4_f32, four points per step (points past the run end
// enter with zero weight).  The first two dimensions are indexed by slot, the
// tap's tile position modulo TW (the weight record stores the first
// dimension that way; the second is rotated here, per run), so a tile cell's
// slot pair does not depend on the run.  Wave w keeps column block w mod NB
// (first-dimension slots 16/R (w mod NB) .. + 16/R - 1 times R vectors) and
// the 3 x 16 rows of second-dimension slots 4 (w / NB) .. + 3 times all TW
// third-dimension taps: row i = 4 q + v of its block k is second slot
// 4 (w / NB) + q and third tap 4 k + v.  Waves therefore own disjoint slot
// pairs, hence disjoint tile cells whatever the run, and each wave flushes a
// run into the LDS tile after its last point with plain loads and stores and
// no barrier (a wave's own flushes are ordered).  The LDS tile is padded (row
// stride odd, plane stride 8 and vector stride 2 modulo 32 words) so that the
// 32 lanes of a flush half-wave fall on distinct banks; it is written out
// unpadded.
template <int M, int R>
struct SpreadMfmaShape {
    static constexpr int TW = 2 * M;
    static constexpr int NB = (TW * R + 15) / 16;               // column blocks (the last may be padded)
    static constexpr int MG = TW / 4;                           // second-dimension slot groups
    static constexpr int BPW = TW / 4;                          // row blocks per wave
    static constexpr int NWAVE = NB * MG;
    static_assert(TW % 4 == 0 && 16 % R == 0, "block shape");
};

// Padded strides of the LDS tile (words): row, plane, vector.
struct SpreadMfmaPad {
    int sb, sa, sr;
};

__host__ __device__ inline SpreadMfmaPad spread_mfma_pad(int pd)
{
    SpreadMfmaPad q;
    q.sb = pd | 1;
    q.sa = pd * q.sb + ((8 - pd * q.sb) % 32 + 32) % 32;
    q.sr = pd * q.sa + ((2 - pd * q.sa) % 32 + 32) % 32;
    return q;
}

template <int M, int R>
__global__ void __launch_bounds__((64 * SpreadMfmaShape<M, R>::NWAVE))
k_spread_mfma(const WinDesc *__restrict__ wd, const int *__restrict__ sub_win,
              const int *__restrict__ sub_start, const int *__restrict__ sub_count,
              const float *__restrict__ V, int64_t ldv, int nrhs, int pd, float *__restrict__ tilebuf)
{
    using f4 = __attribute__((ext_vector_type(4))) float;
    using S = SpreadMfmaShape<M, R>;
    constexpr int TW = S::TW, NB = S::NB, BPW = S::BPW;
    constexpr int RS = 3 * TW;                                  // weights per point
    constexpr int SPB = 16 / R;                                 // first-dimension slots per column block
    constexpr int CH = 64;                                      // points staged per chunk
    constexpr int CHP = CH + 8;                                 // + zero points read past a chunk's end
    constexpr int NT = 64 * S::NWAVE;
    __shared__ float s_rec[CHP * RS];
    __shared__ float s_v[CHP * R];
    __shared__ int s_lp[CH];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float *tiles = reinterpret_cast<float *>(smem_raw);
    const SpreadMfmaPad pad = spread_mfma_pad(pd);
    const int pd2 = pd * pd, pc = pd2 * pd;
    const float inv_pd = 1.0f / (float)pd;
    const int sq = xcd_item(blockIdx.x, gridDim.x), r0 = blockIdx.y * R;
    const WinDesc &win = wd[sub_win[sq]];
    gmem<float> *rec = (gmem<float> *)win.rec;
    gmem<int> *lpos = (gmem<int> *)win.lpos;
    gmem<int> *perm = (gmem<int> *)win.perm;
    const int start = sub_start[sq], cnt = sub_count[sq];
    const int end = start + cnt;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < R * pad.sr; i += NT) tiles[i] = 0.0f;
    for (int i = tid; i < (CHP - CH) * RS; i += NT) s_rec[CH * RS + i] = 0.0f;
    for (int i = tid; i < (CHP - CH) * R; i += NT) s_v[CH * R + i] = 0.0f;
    // operand coordinates: A[i][k] and B[k][j] sit in lane i + 16 k (resp.
    // j + 16 k), the accumulator's element v in row 4 (lane / 16) + v
    const int li = lane & 15, kq = lane >> 4;
    const int nb = wave % NB, bg = wave / NB;
    const int aslot_raw = nb * SPB + li / R, br = li % R;       // B column: first slot, vector
    const bool colok = (TW * R) % 16 == 0 || aslot_raw < TW;    // columns past 2m slots pad a block
    const int aslot = colok ? aslot_raw : 0;
    const int bslot_a = 4 * bg + li / 4;                        // A row li: second slot
    const int bslot_f = 4 * bg + kq;                            // accumulator rows: second slot
    const int ac = 2 * TW + li % 4;                             // A row li, block k: third tap 4 k + li % 4
    f4 acc[BPW];
#pragma unroll
    for (int k = 0; k < BPW; ++k) acc[k] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    const int nr = min(R, nrhs - r0);
    // The global data of chunk c + 2 is loaded into registers while chunk c is
    // processed (two register sets alternate), and the sorted-order index of
    // the vector row a thread gathers for it is loaded one chunk earlier still,
    // so no load waits on another load issued in the same chunk.  Every load is
    // issued on every path, at an index clamped into the subproblem (values
    // past its end are masked when staged): the number of loads in flight is
    // then the same on all paths and each wait covers only the loads it needs.
    constexpr int NREC = (CH * RS + NT - 1) / NT, NV = (CH * R + NT - 1) / NT;
    struct Stage {
        float rec[NREC], v[NV];
        int lp;
    };
    // (chunk bases at or past the end read the subproblem's last point)
    const int rc = min(tid % R, nr - 1) + r0;                   // vector column this thread gathers
    auto prefetch_rows = [&](int (&pi)[NV], int cb) {
        const int cx = min(cb, end - 1), last = end - 1 - cx;
        gmem<int> *pb = perm + cx;
#pragma unroll
        for (int k = 0; k < NV; ++k) pi[k] = pb[min(min((tid + k * NT) / R, CH - 1), last)];
    };
    auto fetch = [&](Stage &g, int cb, const int (&pi)[NV]) {
        const int cx = min(cb, end - 1), last = end - 1 - cx;
        gmem<float> *rb = rec + (int64_t)cx * RS;
        const int rlast = (last + 1) * RS - 1;
#pragma unroll
        for (int k = 0; k < NREC; ++k) g.rec[k] = rb[min(tid + k * NT, rlast)];
#pragma unroll
        for (int k = 0; k < NV; ++k) g.v[k] = V[(int64_t)pi[k] * ldv + rc];
        g.lp = lpos[cx + min(tid, last)];
    };
    Stage ga, gb;
    int pq[NV], pn[NV];
    if (cnt > 0) {
        // (issued in the loop's order: the index for chunk 2 before the
        // fetch of chunk 1, so the wait counts at the loop header agree)
        prefetch_rows(pn, start);
        fetch(ga, start, pn);
        prefetch_rows(pn, start + CH);
        prefetch_rows(pq, start + 2 * CH);
        fetch(gb, start + CH, pn);
    }
    auto chunk = [&](int cb, Stage &g) {
        const int nc = min(CH, end - cb);                      // <= 0 for the empty last chunk of an odd count
        __syncthreads();   // tiles cleared / previous chunk consumed
#pragma unroll
        for (int k = 0; k < NREC; ++k) {
            const int i = tid + k * NT;
            if (i < CH * RS) s_rec[i] = i < nc * RS ? g.rec[k] : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const int i = tid + k * NT;
            if (i < CH * R) s_v[i] = (i < nc * R && i % R < nr) ? g.v[k] : 0.0f;
        }
        if (tid < CH) s_lp[tid] = tid < nc ? g.lp : 0;
        __syncthreads();
        prefetch_rows(pn, cb + 3 * CH);
        fetch(g, cb + 2 * CH, pq);
#pragma unroll
        for (int k = 0; k < NV; ++k) pq[k] = pn[k];
        const int my_lp = lane < nc ? s_lp[lane] : 0;
        const bool isend = lane < nc && (my_lp < 0 || cb + lane == end - 1);
        const unsigned long long ends = __ballot(isend);
        int u0 = 0;
        while (u0 < nc) {
            const unsigned long long rest = ends >> u0;
            const bool flush = rest != 0ull;
            const int u1 = flush ? u0 + (int)__builtin_ctzll(rest) : nc - 1;
            // the run's first tap is cell (a0, b0, c0) of the padded tile
            const int lp = __builtin_amdgcn_readlane(my_lp, u0) & 0x7fffffff;
            const int base = lp & 0xfffff, a0 = lp >> 20;
            const int rem = base - a0 * pd2;
            const int b0 = fdiv_small(rem, pd, inv_pd), c0 = rem - b0 * pd;
            // second-dimension tap of the lane's A row (slot bslot_a)
            const int a0m = a0 % TW, b0m = b0 % TW;
            const int abt = bslot_a - b0m;
            const int ab = TW + (abt < 0 ? abt + TW : abt);
            // operands of step u: B = w0[slot] v[r], A = w1[b] w2[c] of the
            // lane's point u + kq, weight 0 past the run end (the reads there
            // hit later points of the chunk or the zero padding).  Two operand
            // sets alternate, so the reads of step u + 4 are in flight while
            // step u's products run.
            struct Ops {
                float w0, v, wb, wc[BPW];
            };
            const float *pr = s_rec + (u0 + kq) * RS;
            const float *pv = s_v + (u0 + kq) * R + br;
            auto load = [&](Ops &o) {
                o.w0 = pr[aslot];
                o.v = *pv;
                o.wb = pr[ab];
#pragma unroll
                for (int k = 0; k < BPW; ++k) o.wc[k] = pr[ac + 4 * k];
                pr += 4 * RS;
                pv += 4 * R;
            };
            // lim = points of the step that belong to the run (4 but for a
            // run's last step)
            // (a step's operand products are formed before its matrix
            // products issue, so no product waits on the vector unit; the
            // products issue at raised wave priority)
            auto step = [&](const Ops &o, int lim) {
                const float bv = colok && kq < lim ? o.w0 * o.v : 0.0f;
                float av[BPW];
#pragma unroll
                for (int k = 0; k < BPW; ++k) av[k] = o.wb * o.wc[k];
                __builtin_amdgcn_sched_barrier(0);
                __builtin_amdgcn_s_setprio(1);
#pragma unroll
                for (int k = 0; k < BPW; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[k], bv, acc[k], 0, 0, 0);
                __builtin_amdgcn_s_setprio(0);
            };
            auto step_full = [&](const Ops &o) {
                const float bv = colok ? o.w0 * o.v : 0.0f;
                float av[BPW];
#pragma unroll
                for (int k = 0; k < BPW; ++k) av[k] = o.wb * o.wc[k];
                __builtin_amdgcn_sched_barrier(0);
                __builtin_amdgcn_s_setprio(1);
#pragma unroll
                for (int k = 0; k < BPW; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[k], bv, acc[k], 0, 0, 0);
                __builtin_amdgcn_s_setprio(0);
            };
            // (scheduling barriers keep each set's reads ahead of the other
            // set's products).  Whole groups of four full steps run in a loop
            // with one exit and no masking; the last 0-3 full steps and the
            // run's partial step follow it.
            const int np = u1 - u0 + 1, nfull = np >> 2, tail = np & 3;
            Ops opa, opb;
            load(opa);
            int st = 0;
            for (; st + 4 <= nfull; st += 4) {
                load(opb);
                __builtin_amdgcn_sched_barrier(0);
                step_full(opa);
                __builtin_amdgcn_sched_barrier(0);
                load(opa);
                __builtin_amdgcn_sched_barrier(0);
                step_full(opb);
                __builtin_amdgcn_sched_barrier(0);
                load(opb);
                __builtin_amdgcn_sched_barrier(0);
                step_full(opa);
                __builtin_amdgcn_sched_barrier(0);
                load(opa);
                __builtin_amdgcn_sched_barrier(0);
                step_full(opb);
                __builtin_amdgcn_sched_barrier(0);
            }
            const int nrest = nfull - st + (tail > 0);         // 0..4 steps left
            const int llim = tail > 0 ? tail : 4;
            if (nrest > 0) {
                if (nrest > 1) load(opb);
                __builtin_amdgcn_sched_barrier(0);
                step(opa, nrest == 1 ? llim : 4);
                __builtin_amdgcn_sched_barrier(0);
                if (nrest > 1) {
                    if (nrest > 2) load(opa);
                    __builtin_amdgcn_sched_barrier(0);
                    step(opb, nrest == 2 ? llim : 4);
                    __builtin_amdgcn_sched_barrier(0);
                    if (nrest > 2) {
                        if (nrest > 3) load(opb);
                        __builtin_amdgcn_sched_barrier(0);
                        step(opa, nrest == 3 ? llim : 4);
                        __builtin_amdgcn_sched_barrier(0);
                        if (nrest > 3) step(opb, llim);
                    }
                }
            }
            if (flush && colok) {
                // lane's cells: first tap (aslot - a0) mod TW, second tap
                // (bslot_f - b0) mod TW, third taps 4 k + v; all reads first,
                // then the writes
                const int at0 = aslot - a0m, bt0 = bslot_f - b0m;
                const int at = at0 < 0 ? at0 + TW : at0;
                const int bt = bt0 < 0 ? bt0 + TW : bt0;
                float *tp = tiles + br * pad.sr + (a0 + at) * pad.sa + (b0 + bt) * pad.sb + c0;
                float old[BPW][4];
#pragma unroll
                for (int k = 0; k < BPW; ++k)
#pragma unroll
                    for (int v = 0; v < 4; ++v) old[k][v] = tp[4 * k + v];
#pragma unroll
                for (int k = 0; k < BPW; ++k) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) tp[4 * k + v] = old[k][v] + acc[k][v];
                    acc[k] = f4{0.0f, 0.0f, 0.0f, 0.0f};
                }
            }
            u0 = u1 + 1;
        }
    };
    for (int cb = start; cb < end; cb += 2 * CH) {
        chunk(cb, ga);
        chunk(cb + CH, gb);
    }
    __syncthreads();
    // cell i = (a, b, c) advances by NT per iteration: (a, b, c) and the padded
    // offset are stepped with carries instead of divided out per cell
    {
        float *out = tilebuf + ((int64_t)sq * nrhs + r0) * pc;
        const int da = NT / pd2, db = (NT - da * pd2) / pd, dc = NT - da * pd2 - db * pd;
        const int a = fdiv_small(tid, pd2, 1.0f / (float)pd2), rm = tid - a * pd2;
        int b = fdiv_small(rm, pd, inv_pd), c = rm - b * pd;
        int off = a * pad.sa + b * pad.sb + c;
        const int doff = da * pad.sa + db * pad.sb + dc;
        for (int i = tid; i < pc; i += NT) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (r < nr) out[(int64_t)r * pc + i] = tiles[r * pad.sr + off];
            off += doff;
            c += dc;
            b += db;
            if (c >= pd) {
                c -= pd;
                ++b;
                off += pad.sb - pd;
            }
            if (b >= pd) {
                b -= pd;
                off += pad.sa - pd * pad.sb;
            }
        }
    }
}

// ---------------------------------------------------------------- fold
// Phase 1: the subproblems of one tile are summed into the first one's slot
// (in place, fixed order: 4 slices per cell combined through LDS).
// Only tiles with two or more subproblems are listed (fb: window * nbins + tile).
template <typename T>
__global__ void __launch_bounds__(256)
k_fold_bins(const WinDesc *__restrict__ wd, const int *__restrict__ fb, T *__restrict__ tilebuf,
            int nbins, int nrhs, int pc)
{
    __shared__ T part[4][64];
    const int wb = fb[blockIdx.y], r = blockIdx.z;
    gmem<int> *bsp = (gmem<int> *)wd[wb / nbins].bin_sub_ptr;
    const int bin = wb % nbins;
    const int s0 = bsp[bin], s1 = bsp[bin + 1];
    if (s1 - s0 < 2) return;
    const int ci = threadIdx.x & 63, slice = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + ci;
    // four independent partial sums per thread: four loads in flight
    T sum = T(0);
    if (i < pc) {
        const T *src = tilebuf + (int64_t)r * pc + i;
        const int64_t step = (int64_t)nrhs * pc;
        T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
        int s = s0 + 1 + slice;
        for (; s + 12 < s1; s += 16) {
            a0 += src[(int64_t)s * step];
            a1 += src[(int64_t)(s + 4) * step];
            a2 += src[(int64_t)(s + 8) * step];
            a3 += src[(int64_t)(s + 12) * step];
        }
        for (; s < s1; s += 4) a0 += src[(int64_t)s * step];
        sum = (a0 + a1) + (a2 + a3);
    }
    part[slice][ci] = sum;
    __syncthreads();
    if (slice == 0 && i < pc) {
        T *dst = tilebuf + ((int64_t)s0 * nrhs + r) * pc;
        dst[i] = dst[i] + ((part[0][ci] + part[1][ci]) + (part[2][ci] + part[3][ci]));
    }
}

// Phase 2: every grid cell of the occupied range (cells olo .. olo + on - 1 of
// each axis; the FFT reads no other cell) sums the (at most 3^d) tiles whose
// padded region covers it.  Output layout [window][vector][cell].
template <typename T, int D>
__global__ void __launch_bounds__(256)
k_fold(const WinDesc *__restrict__ wd, const T *__restrict__ tilebuf, int nrhs, int tb, int nb,
       int ng, int m, int pd, int pc, int64_t cells, int olo, int on, int ocells,
       typename Cplx<T>::type *__restrict__ grid, int nwr, int coef_blocks, int coef_nper, int cd, int cN,
       CoefParams prm, const double *__restrict__ cinv2, const double *__restrict__ cw,
       double *__restrict__ cpart)
{
    // rows blockIdx.y >= nwr: the group's separable coefficients (coef_sep_block),
    // block (blk, arr, w) numbered row-major after the fold rows
    if ((int)blockIdx.y >= nwr) {
        __shared__ double lds[4 * kCoefMaxH + 256];
        const int cb = ((int)blockIdx.y - nwr) * (int)gridDim.x + (int)blockIdx.x;
        if (cb >= coef_blocks) return;
        const int blk = cb % coef_nper, aw = cb / coef_nper;
        coef_sep_block<T>(cd, cN, prm, cinv2, cw, wd, cpart, blk, coef_nper, aw % 2, aw / 2, lds);
        return;
    }
    // one thread per occupied cell; blockIdx.y = window * nrhs + vector
    const int ci = xcd_item(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (ci >= ocells) return;
    const int wr = blockIdx.y;
    const int w = wr / nrhs, r = wr % nrhs;
    int rem = ci;
    const float inv_on = 1.0f / (float)on;
    gmem<int> *bsp = (gmem<int> *)wd[w].bin_sub_ptr;
    int l[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    int64_t cell = 0, cstride = 1;
    for (int q = D - 1; q >= 0; --q) {
        const int qt = fdiv_small(rem, on, inv_on);
        l[q] = olo + (rem - qt * on);
        rem = qt;
        cell += (int64_t)l[q] * cstride;
        cstride *= ng;
        // bins b with b*tb - m <= l <= b*tb - m + pd - 1
        int num = l[q] + m - pd + 1;
        // tb is a power of two: floor / ceil division by shifts
        const int sh = __ffs(tb) - 1;
        int blo = -((-num) >> sh);   // ceil(num / tb)
        int bhi = (l[q] + m) >> sh;
        lo[q] = blo < 0 ? 0 : blo;
        hi[q] = bhi > nb - 1 ? nb - 1 : bhi;
    }
    // at most 3 covering tiles per axis (pd <= 3 tb): the loops are unrolled
    // over 3 with predicates, so all CSR and tile loads are issued together
    constexpr int K1 = D > 1 ? 3 : 1, K2 = D > 2 ? 3 : 1;
    int sidx[3 * K1 * K2], lidx[3 * K1 * K2];
#pragma unroll
    for (int u0 = 0; u0 < 3; ++u0)
#pragma unroll
        for (int u1 = 0; u1 < K1; ++u1)
#pragma unroll
            for (int u2 = 0; u2 < K2; ++u2) {
                const int t = (u0 * K1 + u1) * K2 + u2;
                const int b0 = lo[0] + u0, b1 = lo[1] + u1, b2 = lo[2] + u2;
                const bool ok = b0 <= hi[0] && (D < 2 || b1 <= hi[1]) && (D < 3 || b2 <= hi[2]);
                int bin = b0, li = l[0] - b0 * tb + m;
                if (D > 1) {
                    bin = bin * nb + b1;
                    li = li * pd + (l[1] - b1 * tb + m);
                }
                if (D > 2) {
                    bin = bin * nb + b2;
                    li = li * pd + (l[2] - b2 * tb + m);
                }
                int s0 = -1;
                if (ok && bsp[bin + 1] > bsp[bin]) s0 = bsp[bin];
                sidx[t] = s0;
                lidx[t] = li;
            }
    T sum = T(0);
#pragma unroll
    for (int t = 0; t < 3 * K1 * K2; ++t)
        if (sidx[t] >= 0) sum += tilebuf[((int64_t)sidx[t] * nrhs + r) * pc + lidx[t]];
    typename Cplx<T>::type o;
    o.x = sum;
    o.y = T(0);
    grid[(int64_t)wr * cells + cell] = o;
}

// ---------------------------------------------------------------- interpolation
// One thread per PT points (subproblems of at most 256 PT points of one
// tile): points t, t + 256, ..., or with ADJ (d = 3, PT = 2) the adjacent
// sorted points 2t and 2t + 1.  The padded tile of the grid (and of the
// derivative grid) is staged in LDS for one vector at a time; the point's
// window weights are loaded once and reused for every vector.  Each window
// writes its own block of the per-window output buffer (one owner thread per
// entry).
template <typename T, int D, int M, bool DER, int PT, bool ADJ = false, bool SLOT = false>
__global__ void __launch_bounds__(256)
k_interp(const WinDesc *__restrict__ wd, const int *__restrict__ sub_win,
         const int *__restrict__ sub_bin, const int *__restrict__ sub_start,
         const int *__restrict__ sub_count, int tb, int nb, int ng, int nwin, int rows,
         const typename Cplx<T>::type *__restrict__ grid, int64_t cells, int nrhs, int64_t n,
         T *__restrict__ hbuf, T *__restrict__ dout, T dscale)
{
    using C = typename Cplx<T>::type;
    constexpr int TW = 2 * M;
    constexpr int RS = D * TW;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // the tile of the grid, interleaved with the derivative grid's tile when
    // DER (one LDS read gives both values of a tap)
    T *tK = reinterpret_cast<T *>(smem_raw);
    C *tKD = reinterpret_cast<C *>(smem_raw);
    const int pd = tb + 2 * M;
    int pc = pd;
    for (int q = 1; q < D; ++q) pc *= pd;
    const float inv_pd = 1.0f / (float)pd;
    const int sq = xcd_item(blockIdx.x, gridDim.x);
    const int wi = sub_win[sq];
    const WinDesc &win = wd[wi];
    gmem<T> *rec = (gmem<T> *)win.rec;
    const int start = sub_start[sq], cnt = sub_count[sq];
    // 3-D: only first-axis rows a0 .. a0 + rows - 1 of the padded tile are
    // staged (a0 in bits 24-31 of the tile index)
    int org[3] = {0, 0, 0};
    const int bw = sub_bin[sq];
    const int a0 = D == 3 ? (bw >> 24) : 0;
    bin_origin<D>(bw & 0xffffff, nb, tb, org);
    // PT points per thread (thread t takes points t, t + 256, ...): weights
    // and first-tap positions in registers for all vectors; for d = 3 the
    // first dimension's weights are re-read inside its (rolled) loop so that
    // no register array is indexed by a loop variable
    bool mine[PT];
    gmem<T> *rp[PT];
    T w[PT][D][TW];
    int lin[PT], f0[PT];
    int64_t orow[PT];
    // SLOT (d = 3, two points per thread): thread t takes slot start + t, one
    // point or two consecutive points of one cell (then every tap read below
    // serves both); an unpaired slot repeats its point without an output
    int slot0 = 0;
    if constexpr (SLOT) {
        slot0 = (int)threadIdx.x < cnt ? ((gmem<int> *)win.slots)[start + (int)threadIdx.x] : 0;
    }
#pragma unroll
    for (int p = 0; p < PT; ++p) {
        const int k = ADJ ? 2 * (int)threadIdx.x + p : (int)threadIdx.x + 256 * p;
        int64_t j;
        if constexpr (SLOT) {
            mine[p] = (int)threadIdx.x < cnt && (p == 0 || slot0 < 0);
            j = (int64_t)(slot0 & 0x7fffffff) + (mine[p] ? p : 0);
        } else {
            mine[p] = k < cnt;
            j = start + (mine[p] ? k : 0);
        }
        rp[p] = rec + j * RS;
#pragma unroll
        for (int q = (D == 3 ? 1 : 0); q < D; ++q)
#pragma unroll
            for (int a = 0; a < TW; ++a) w[p][q][a] = rp[p][q * TW + a];
        const int lpj = ((gmem<int> *)win.lpos)[j];
        lin[p] = (lpj & 0xfffff) - a0 * pd * pd * (D == 3);   // first tap inside the staged rows
        f0[p] = (lpj >> 20) & 0x7f;                         // first-dimension weights sit rotated by it
        orow[p] = (int64_t)((gmem<int> *)win.perm)[j] * nrhs;
    }
    T *hout = hbuf + (int64_t)win.s_global * n * nrhs;
    T *dblk = DER ? dout + (int64_t)win.s_global * n * nrhs : nullptr;
    // one tap: value times weight into the K (and derivative) sums
    auto tap = [&](int idx, T wt, T &sK, T &sD) {
        if constexpr (DER) {
            const C v = tKD[idx];
            sK += v.x * wt;
            sD += v.y * wt;
        } else {
            sK += tK[idx] * wt;
        }
    };
    // d = 3 staging: thread t takes cells t, t + 256, ... of the tile's
    // (second, third) plane -- their grid offsets inside a plane are fixed --
    // and walks the first dimension, so a cell costs one add and no division
    constexpr int PDM = 8 + 2 * M;                        // largest padded width (tb <= 8)
    constexpr int NS = D == 3 ? (PDM * PDM + 255) / 256 : 1;
    int prel[NS];
    bool pin[NS];
    if constexpr (D == 3) {
        const int pd2 = pd * pd;
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int q = (int)threadIdx.x + 256 * j;
            const int b = fdiv_small(q, pd, inv_pd), c = q - b * pd;
            const int l1 = org[1] - M + b, l2 = org[2] - M + c;
            pin[j] = q < pd2 && l1 >= 0 && l1 < ng && l2 >= 0 && l2 < ng;
            prel[j] = pin[j] ? l1 * ng + l2 : 0;
        }
    }
    for (int r = 0; r < nrhs; ++r) {
        const C *gK = grid + ((int64_t)wi * nrhs + r) * cells;
        // the derivative grid is the imaginary part of the same grid
        const C *gD = gK;
        if (r > 0) __syncthreads();
        if constexpr (D == 3) {
            const int pd2 = pd * pd;
            // SA planes per batch: all loads of a batch in flight before the
            // first LDS store
            constexpr int SA = NS == 1 ? 8 : (NS == 2 ? 4 : 2);
            for (int ab = 0; ab < rows; ab += SA) {
                T vK[SA][NS], vD[SA][NS];
#pragma unroll
                for (int aa = 0; aa < SA; ++aa) {
                    const int la = org[0] - M + a0 + ab + aa;
                    const bool ina = ab + aa < rows && la >= 0 && la < ng;
                    const int64_t pl = (int64_t)(ina ? la : 0) * ng * ng;
#pragma unroll
                    for (int j = 0; j < NS; ++j) {
                        const bool in = ina && pin[j];
                        vK[aa][j] = in ? gK[pl + prel[j]].x : T(0);
                        vD[aa][j] = (DER && in) ? gD[pl + prel[j]].y : T(0);
                    }
                }
#pragma unroll
                for (int aa = 0; aa < SA; ++aa) {
#pragma unroll
                    for (int j = 0; j < NS; ++j) {
                        const int q = (int)threadIdx.x + 256 * j;
                        if (ab + aa < rows && q < pd2) {
                            const int i = (ab + aa) * pd2 + q;
                            if constexpr (DER) {
                                C v;
                                v.x = vK[aa][j];
                                v.y = vD[aa][j];
                                tKD[i] = v;
                            } else {
                                tK[i] = vK[aa][j];
                            }
                        }
                    }
                }
            }
        } else {
        // staged in batches of SB cells per thread: the loads of a batch are
        // all in flight before the first LDS store
        constexpr int SB = 8;
        for (int i0 = 0; i0 < pc; i0 += SB * 256) {
            T vK[SB], vD[SB];
#pragma unroll
            for (int b = 0; b < SB; ++b) {
                const int i = i0 + b * 256 + (int)threadIdx.x;
                int rem = i, loc[3] = {0, 0, 0};
                for (int q = D - 1; q >= 0; --q) {
                    const int qt = fdiv_small(rem, pd, inv_pd);
                    loc[q] = rem - qt * pd;
                    rem = qt;
                }
                bool in = i < pc;
                int64_t g = 0;
                for (int q = 0; q < D; ++q) {
                    int l = org[q] - M + loc[q];
                    in = in && (l >= 0) && (l < ng);
                    g = g * ng + l;
                }
                vK[b] = in ? gK[g].x : T(0);
                vD[b] = (DER && in) ? gD[g].y : T(0);
            }
#pragma unroll
            for (int b = 0; b < SB; ++b) {
                const int i = i0 + b * 256 + (int)threadIdx.x;
                if (i < pc) {
                    if constexpr (DER) {
                        C v;
                        v.x = vK[b];
                        v.y = vD[b];
                        tKD[i] = v;
                    } else {
                        tK[i] = vK[b];
                    }
                }
            }
        }
        }
        __syncthreads();
        if constexpr (ADJ && D == 3 && PT == 2) {
            // two adjacent sorted points per thread: where they share a cell
            // (same first tap) each tap value read serves both; the second
            // point's rows are read again only in lanes whose cells differ
            if (mine[0]) {
                const bool same = SLOT || lin[0] == lin[1];
                T hK[2] = {T(0), T(0)}, hD[2] = {T(0), T(0)};
#pragma unroll 1
                for (int aa = 0; aa < TW; ++aa) {
                    const T wa[2] = {rp[0][(f0[0] + aa) % TW], rp[1][(f0[1] + aa) % TW]};
                    T sK[2] = {T(0), T(0)}, sD[2] = {T(0), T(0)};
#pragma unroll
                    for (int bb = 0; bb < TW; ++bb) {
                        const int off = (aa * pd + bb) * pd;
                        T aK[TW], aD[TW];
#pragma unroll
                        for (int cc = 0; cc < TW; ++cc) {
                            if constexpr (DER) {
                                const C v = tKD[lin[0] + off + cc];
                                aK[cc] = v.x;
                                aD[cc] = v.y;
                            } else {
                                aK[cc] = tK[lin[0] + off + cc];
                                aD[cc] = T(0);
                            }
                        }
                        T bK[TW], bD[TW];
#pragma unroll
                        for (int cc = 0; cc < TW; ++cc) {
                            bK[cc] = aK[cc];
                            bD[cc] = aD[cc];
                        }
                        if (!SLOT && !same) {
#pragma unroll
                            for (int cc = 0; cc < TW; ++cc) {
                                if constexpr (DER) {
                                    const C v = tKD[lin[1] + off + cc];
                                    bK[cc] = v.x;
                                    bD[cc] = v.y;
                                } else {
                                    bK[cc] = tK[lin[1] + off + cc];
                                }
                            }
                        }
                        T cK0 = T(0), cD0 = T(0), cK1 = T(0), cD1 = T(0);
#pragma unroll
                        for (int cc = 0; cc < TW; ++cc) {
                            cK0 += aK[cc] * w[0][2][cc];
                            cK1 += bK[cc] * w[1][2][cc];
                            if (DER) {
                                cD0 += aD[cc] * w[0][2][cc];
                                cD1 += bD[cc] * w[1][2][cc];
                            }
                        }
                        sK[0] += cK0 * w[0][1][bb];
                        sK[1] += cK1 * w[1][1][bb];
                        if (DER) {
                            sD[0] += cD0 * w[0][1][bb];
                            sD[1] += cD1 * w[1][1][bb];
                        }
                        // the row's sums are complete here, before the next
                        // row's reads (else the compiler defers every row's
                        // FMAs until all rows are loaded)
                        asm volatile("" : "+v"(sK[0]), "+v"(sK[1]), "+v"(sD[0]), "+v"(sD[1]));
                    }
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        hK[q] += sK[q] * wa[q];
                        if (DER) hD[q] += sD[q] * wa[q];
                    }
                }
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    if (!mine[q]) continue;
                    hout[orow[q] + r] = hK[q];
                    if (DER) dblk[orow[q] + r] = dscale * hD[q];
                }
            }
            continue;
        }
#pragma unroll
        for (int p = 0; p < PT; ++p) {
            if (!mine[p]) continue;
            T hK = T(0), hD = T(0);
            if (D == 1) {
#pragma unroll
                for (int aa = 0; aa < TW; ++aa) tap(lin[p] + aa, w[p][0][aa], hK, hD);
            } else if (D == 2) {
#pragma unroll
                for (int aa = 0; aa < TW; ++aa) {
                    T sK = T(0), sD = T(0);
                    const int row = lin[p] + aa * pd;
#pragma unroll
                    for (int bb = 0; bb < TW; ++bb) tap(row + bb, w[p][D > 1 ? 1 : 0][bb], sK, sD);
                    hK += sK * w[p][0][aa];
                    if (DER) hD += sD * w[p][0][aa];
                }
            } else {
#pragma unroll 1
                for (int aa = 0; aa < TW; ++aa) {
                    const T w0 = rp[p][(f0[p] + aa) % TW];
                    T sK = T(0), sD = T(0);
#pragma unroll
                    for (int bb = 0; bb < TW; ++bb) {
                        const int row = lin[p] + (aa * pd + bb) * pd;
                        T cK = T(0), cD = T(0);
#pragma unroll
                        for (int cc = 0; cc < TW; ++cc) tap(row + cc, w[p][D > 2 ? 2 : 0][cc], cK, cD);
                        sK += cK * w[p][D > 1 ? 1 : 0][bb];
                        if (DER) sD += cD * w[p][D > 1 ? 1 : 0][bb];
                    }
                    hK += sK * w0;
                    if (DER) hD += sD * w0;
                }
            }
            hout[orow[p] + r] = hK;
            if (DER) dblk[orow[p] + r] = dscale * hD;
        }
    }
}

// Matrix-core form of 3-D FP32 interpolation.  A block is at most 16 points
// of one cell, so its points read the same (2m)^3 taps of the tile and
//
//   X[p, (a, e)] = sum_(b, c)  w1_p[b] w2_p[c]  *  G_e[a0 + a, b0 + b, c0 + c]
//
// is one dense product: rows p (the block's points, missing rows with zero
// weight), reduction over the TW^2 tap pairs (b, c), four at a time on
// v_mfma_f32_16x16x4_f32, columns (a, e) = four first-dimension taps times
// four staged values e per cell (K and dK of two vectors with derivative
// outputs, else K of four vectors); TW / 4 column blocks cover the TW first-
// dimension taps.  Then h_p[e] = sum_a w0_p[a] X[p, (a, e)]: each lane
// weights its accumulators and four lanes are summed.  A work-group of 8
// waves takes a subproblem of at most 16 blocks of one tile; the blocks'
// weights, output rows and first taps sit in LDS for the whole subproblem,
// and the staged rows of the padded tile (plane stride 8 modulo 32 words:
// the 32 lanes of a half-wave read distinct banks) hold four values per cell.
template <int M, bool DER, int NWV, bool WLDS>
__global__ void __launch_bounds__((64 * NWV))
k_interp_mfma(const WinDesc *__restrict__ wd, const int *__restrict__ sub_win,
              const int *__restrict__ sub_bin, const int *__restrict__ sub_start,
              const int *__restrict__ sub_count, int tb, int nb, int ng, int rows,
              const float2 *__restrict__ grid, int64_t cells, int nrhs, int64_t n,
              float *__restrict__ hbuf, float *__restrict__ dout, float dscale)
{
    using f4 = __attribute__((ext_vector_type(4))) float;
    constexpr int TW = 2 * M, RS = 3 * TW;
    constexpr int NBK = TW / 4;                 // column blocks (four first-dimension taps each)
    constexpr int KS = TW * TW / 4;             // reduction steps over (b, c)
    constexpr int VPS = DER ? 2 : 4;            // vectors per staging
    constexpr int NT = 64 * NWV;
    constexpr int MB = WLDS ? kInterpSubBlocksLds : kInterpSubBlocks;   // blocks per subproblem, at most
    constexpr int MAXP = 16 * MB;
    // the points' weights: copied to LDS once per subproblem (WLDS), or read
    // from the weight record (L2) per block and pass, which leaves the LDS to
    // two work-groups per CU
    __shared__ float s_w[WLDS ? MAXP * RS : 1];
    __shared__ int s_row[MAXP];
    __shared__ int s_blk[MB + 1];
    __shared__ int s_lp[MB];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float *tile = reinterpret_cast<float *>(smem_raw);
    const int pd = tb + 2 * M, pd2 = pd * pd;
    const int ps = 4 * pd2 + ((8 - 4 * pd2) % 32 + 32) % 32;   // plane stride (words)
    const int sq = xcd_item(blockIdx.x, gridDim.x);
    const int wi = sub_win[sq];
    const WinDesc &win = wd[wi];
    gmem<float> *rec = (gmem<float> *)win.rec;
    gmem<int> *blocks = (gmem<int> *)win.blocks;
    gmem<int> *lposg = (gmem<int> *)win.lpos;
    gmem<int> *permg = (gmem<int> *)win.perm;
    const int start = sub_start[sq], cnt = sub_count[sq];
    int org[3] = {0, 0, 0};
    const int bw = sub_bin[sq];
    const int a0s = bw >> 24;                   // first staged row of the padded tile
    bin_origin<3>(bw & 0xffffff, nb, tb, org);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // the subproblem's points [P0, P1): weights, output rows, block starts
    const int P0 = blocks[start], P1 = blocks[start + cnt];
    if (WLDS)
        for (int i = tid; i < (P1 - P0) * RS; i += NT) s_w[i] = rec[(int64_t)P0 * RS + i];
    // weight idx of the subproblem's points (local point index x RS + slot)
    auto wread = [&](int idx) -> float {
        if constexpr (WLDS)
            return s_w[idx];
        else
            return rec[(int64_t)P0 * RS + idx];
    };
    for (int i = tid; i < P1 - P0; i += NT) s_row[i] = permg[P0 + i];
    if (tid <= cnt) s_blk[tid] = blocks[start + tid] - P0;
    if (tid < cnt) s_lp[tid] = lposg[blocks[start + tid]];
    // staging: thread t takes cell t of the tile's (second, third) plane
    const bool qin = tid < pd2;
    int prel = 0;
    bool pin = false;
    {
        const int b = tid / pd, c = tid - (tid / pd) * pd;
        const int l1 = org[1] - M + b, l2 = org[2] - M + c;
        pin = qin && l1 >= 0 && l1 < ng && l2 >= 0 && l2 < ng;
        prel = pin ? l1 * ng + l2 : 0;
    }
    const int li = lane & 15, kq = lane >> 4;
    const int al = li >> 2, e = li & 3;         // B / accumulator column: first-dimension tap, value
    for (int r0 = 0; r0 < nrhs; r0 += VPS) {
        __syncthreads();   // weights staged / previous pass consumed
        constexpr int SA = 12;
        for (int ab = 0; ab < rows; ab += SA) {
            f4 v4[SA];
#pragma unroll
            for (int aa = 0; aa < SA; ++aa) {
                const int la = org[0] - M + a0s + ab + aa;
                const bool in = ab + aa < rows && pin && la >= 0 && la < ng;
                const int64_t g = (int64_t)(in ? la : 0) * ng * ng + prel;
                f4 v = f4{0.0f, 0.0f, 0.0f, 0.0f};
                if (DER) {
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        if (in && r0 + q < nrhs) {
                            const float2 c = grid[((int64_t)wi * nrhs + r0 + q) * cells + g];
                            v[2 * q] = c.x;
                            v[2 * q + 1] = c.y;
                        }
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (in && r0 + q < nrhs) v[q] = grid[((int64_t)wi * nrhs + r0 + q) * cells + g].x;
                }
                v4[aa] = v;
            }
#pragma unroll
            for (int aa = 0; aa < SA; ++aa)
                if (ab + aa < rows && qin) *reinterpret_cast<f4 *>(tile + (ab + aa) * ps + 4 * tid) = v4[aa];
        }
        __syncthreads();
        for (int k = wave; k < cnt; k += NWV) {
            const int j0 = s_blk[k], np = s_blk[k + 1] - j0;
            const int lp = s_lp[k];
            const int lin = (lp & 0xfffff) - a0s * pd2;   // first tap inside the staged rows
            const int frow = fdiv_small(lin, pd2, 1.0f / (float)pd2), rem = lin - frow * pd2;
            // A row li: point j0 + li (rows past the block: weight 0)
            const int rb = (j0 + min(li, np - 1)) * RS;
            float w1[TW], w2k[TW / 4];
#pragma unroll
            for (int t = 0; t < TW; ++t) w1[t] = wread(rb + TW + t);
#pragma unroll
            for (int t = 0; t < TW / 4; ++t) w2k[t] = li < np ? wread(rb + 2 * TW + 4 * t + kq) : 0.0f;
            // first-dimension weights of the epilogue, loaded now so that their
            // latency overlaps the products: lane (al, e, kq) weights its
            // accumulator element v of block c with w0 of point 4 kq + v at
            // tap 4 c + al (slot (L + 4 c + al) mod TW of the rotated record)
            const int L = (lp >> 20) & 0x7f;
            float w0e[4][NBK];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int wb = (j0 + min(4 * kq + v, np - 1)) * RS;
#pragma unroll
                for (int c = 0; c < NBK; ++c) w0e[v][c] = wread(wb + (L + 4 * c + al) % TW);
            }
            const float *tb0 = tile + (frow + al) * ps + (rem + kq) * 4 + e;
            f4 acc[NBK];
#pragma unroll
            for (int c = 0; c < NBK; ++c) acc[c] = f4{0.0f, 0.0f, 0.0f, 0.0f};
            // one second-dimension tap b per round: its TW / 4 steps times NBK
            // column blocks; the next round's B values are read while this
            // round's products run
            constexpr int SPR = TW / 4;
            float bv[2][SPR][NBK];
            auto load_row = [&](float (&dst)[SPR][NBK], int b) {
#pragma unroll
                for (int t = 0; t < SPR; ++t)
#pragma unroll
                    for (int c = 0; c < NBK; ++c) dst[t][c] = tb0[(b * pd + 4 * t) * 4 + c * 4 * ps];
            };
            load_row(bv[0], 0);
#pragma unroll
            for (int b = 0; b < TW; ++b) {
                if (b + 1 < TW) load_row(bv[(b + 1) & 1], b + 1);
                __builtin_amdgcn_sched_barrier(0);
                // (waves issuing matrix products run at raised priority, so
                // they are picked before waves that are staging)
                __builtin_amdgcn_s_setprio(1);
#pragma unroll
                for (int t = 0; t < SPR; ++t) {
                    const float av = w1[b] * w2k[t];
#pragma unroll
                    for (int c = 0; c < NBK; ++c)
                        acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[b & 1][t][c], acc[c], 0, 0, 0);
                }
                __builtin_amdgcn_s_setprio(0);
                __builtin_amdgcn_sched_barrier(0);
            }
            // first dimension: lane (al, e, kq) holds X[4 kq + v][(4 c + al, e)]
            float h[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float sum = 0.0f;
#pragma unroll
                for (int c = 0; c < NBK; ++c) sum += w0e[v][c] * acc[c][v];
                sum += __shfl_xor(sum, 4);
                sum += __shfl_xor(sum, 8);
                h[v] = sum;
            }
            if (al == 0) {
                const int vec = r0 + (DER ? e / 2 : e);
                const bool isd = DER && (e & 1);
                if (vec < nrhs) {
                    float *out = (isd ? dout : hbuf) + (int64_t)win.s_global * n * nrhs;
                    const float sc = isd ? dscale : 1.0f;
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (4 * kq + v < np) out[(int64_t)s_row[j0 + 4 * kq + v] * nrhs + vec] = sc * h[v];
                }
            }
        }
    }
}

// 2-D FP32 interpolation on matrix cores: the 3-D kernel's block contraction
// with one reduction dimension.  A block of at most 16 points of one cell
// reads the same taps, so X[p, (a, e)] = sum_b w1_p[b] G_e[a0 + a, b0 + b] is
// a product of the points' second-dimension weights (rows = points, the
// reduction over b four taps per v_mfma_f32_16x16x4_f32 step) and the staged
// tile (columns = four first-dimension taps times the four values e staged
// per cell: K and dK of two vectors, or K of four); the epilogue weights the
// columns with w0_p[a] and sums four lanes, as in 3-D.  A work-group of four
// waves takes a subproblem of blocks of one tile and stages the whole padded
// tile per pass (row stride = 8 modulo 32 words: the lanes of a half-wave
// read distinct banks).  The 2-D weight record is not rotated.
template <int M, bool DER>
__global__ void __launch_bounds__(256)
k_interp_mfma2(const WinDesc *__restrict__ wd, const int *__restrict__ sub_win,
               const int *__restrict__ sub_bin, const int *__restrict__ sub_start,
               const int *__restrict__ sub_count, int tb, int nb, int ng,
               const float2 *__restrict__ grid, int64_t cells, int nrhs, int64_t n,
               float *__restrict__ hbuf, float *__restrict__ dout, float dscale)
{
    using f4 = __attribute__((ext_vector_type(4))) float;
    constexpr int TW = 2 * M, RS = 2 * TW;
    constexpr int NBK = TW / 4;                 // column blocks (four first-dimension taps each)
    constexpr int KS = TW / 4;                  // reduction steps over b
    constexpr int NV = kInterp2Values;          // values staged per cell and pass
    constexpr int NG = NV / 4;                  // value groups of four (one MFMA column set each)
    constexpr int VPS = DER ? NV / 2 : NV;      // vectors per pass
    constexpr int CS = NV + 4;                  // cell stride (words): adjacent cells on other banks
    constexpr int NWV = 4, NT = 64 * NWV;
    constexpr int MB = kInterpSubBlocks, MAXP = 16 * MB;
    __shared__ int s_row[MAXP];
    __shared__ int s_blk[MB + 1];
    __shared__ int s_lp[MB];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float *tile = reinterpret_cast<float *>(smem_raw);
    const int pd = tb + 2 * M;
    const int rstr = pd * CS + ((8 - pd * CS) % 32 + 32) % 32;   // row stride (words)
    const int sq = xcd_item(blockIdx.x, gridDim.x);
    const int wi = sub_win[sq];
    const WinDesc &win = wd[wi];
    gmem<float> *rec = (gmem<float> *)win.rec;
    gmem<int> *blocks = (gmem<int> *)win.blocks;
    gmem<int> *lposg = (gmem<int> *)win.lpos;
    gmem<int> *permg = (gmem<int> *)win.perm;
    const int start = sub_start[sq], cnt = sub_count[sq];
    int org[3] = {0, 0, 0};
    bin_origin<2>(sub_bin[sq] & 0xffffff, nb, tb, org);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int P0 = blocks[start], P1 = blocks[start + cnt];
    for (int i = tid; i < P1 - P0; i += NT) s_row[i] = permg[P0 + i];
    if (tid <= cnt) s_blk[tid] = blocks[start + tid] - P0;
    if (tid < cnt) s_lp[tid] = lposg[blocks[start + tid]];
    const int li = lane & 15, kq = lane >> 4;
    const int al = li >> 2, e = li & 3;         // B / accumulator column: first-dimension tap, value
    const int pc = pd * pd;
    const float inv_ng = 1.0f / (float)NG, inv_pd = 1.0f / (float)pd;
    for (int r0 = 0; r0 < nrhs; r0 += VPS) {
        __syncthreads();   // block lists staged / previous pass consumed
        // unit u = (cell, value group); a value group holds K and dK of two
        // vectors (DER) or K of four
        for (int u = tid; u < pc * NG; u += NT) {
            const int c = fdiv_small(u, NG, inv_ng), gq = u - c * NG;
            const int a = fdiv_small(c, pd, inv_pd), b = c - a * pd;
            const int l0 = org[0] - M + a, l1 = org[1] - M + b;
            const bool in = l0 >= 0 && l0 < ng && l1 >= 0 && l1 < ng;
            const int64_t g = in ? (int64_t)l0 * ng + l1 : 0;
            f4 v = f4{0.0f, 0.0f, 0.0f, 0.0f};
            if (DER) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int vec = r0 + 2 * gq + q;
                    if (in && vec < nrhs) {
                        const float2 z = grid[((int64_t)wi * nrhs + vec) * cells + g];
                        v[2 * q] = z.x;
                        v[2 * q + 1] = z.y;
                    }
                }
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int vec = r0 + 4 * gq + q;
                    if (in && vec < nrhs) v[q] = grid[((int64_t)wi * nrhs + vec) * cells + g].x;
                }
            }
            *reinterpret_cast<f4 *>(tile + a * rstr + b * CS + 4 * gq) = v;
        }
        __syncthreads();
        for (int k = wave; k < cnt; k += NWV) {
            const int j0 = s_blk[k], np = s_blk[k + 1] - j0;
            const int lp = s_lp[k];
            const int L0 = (lp >> 20) & 0x7f, L1 = (lp & 0xfffff) - L0 * pd;   // first tap in the tile
            // A row li: point j0 + li (rows past the block: weight 0), taps 4 t + kq
            const int64_t rb = (int64_t)(P0 + j0 + min(li, np - 1)) * RS;
            float w1k[KS];
#pragma unroll
            for (int t = 0; t < KS; ++t) w1k[t] = li < np ? rec[rb + TW + 4 * t + kq] : 0.0f;
            // epilogue weights: w0 of point 4 kq + v at tap 4 c + al
            float w0e[4][NBK];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t wb = (int64_t)(P0 + j0 + min(4 * kq + v, np - 1)) * RS;
#pragma unroll
                for (int c = 0; c < NBK; ++c) w0e[v][c] = rec[wb + 4 * c + al];
            }
            int orow[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) orow[v] = 4 * kq + v < np ? s_row[j0 + 4 * kq + v] : -1;
            const float *tb0 = tile + (L0 + al) * rstr + (L1 + kq) * CS + e;
            for (int gq = 0; gq < NG; ++gq) {
                f4 acc[NBK];
#pragma unroll
                for (int c = 0; c < NBK; ++c) acc[c] = f4{0.0f, 0.0f, 0.0f, 0.0f};
                float bv[KS][NBK];
#pragma unroll
                for (int t = 0; t < KS; ++t)
#pragma unroll
                    for (int c = 0; c < NBK; ++c) bv[t][c] = tb0[4 * c * rstr + 4 * t * CS + 4 * gq];
                __builtin_amdgcn_s_setprio(1);
#pragma unroll
                for (int t = 0; t < KS; ++t)
#pragma unroll
                    for (int c = 0; c < NBK; ++c)
                        acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(w1k[t], bv[t][c], acc[c], 0, 0, 0);
                __builtin_amdgcn_s_setprio(0);
                // first dimension: lane (al, e, kq) holds X[4 kq + v][(4 c + al, e)]
                float h[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float sum = 0.0f;
#pragma unroll
                    for (int c = 0; c < NBK; ++c) sum += w0e[v][c] * acc[c][v];
                    sum += __shfl_xor(sum, 4);
                    sum += __shfl_xor(sum, 8);
                    h[v] = sum;
                }
                if (al == 0) {
                    const int vec = r0 + (DER ? 2 * gq + e / 2 : 4 * gq + e);
                    const bool isd = DER && (e & 1);
                    if (vec < nrhs) {
                        float *out = (isd ? dout : hbuf) + (int64_t)win.s_global * n * nrhs;
                        const float sc = isd ? dscale : 1.0f;
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            if (orow[v] >= 0) out[(int64_t)orow[v] * nrhs + vec] = sc * h[v];
                    }
                }
            }
        }
    }
}

// d <= 2 with at least 16 / sizeof(T) vectors: the tiles of up to vb vectors
// are staged at once, cell-major (a cell's vb values, for DER then its vb
// derivative values, then 16 bytes of padding that put neighbouring cells on
// different LDS banks; vectors past nrhs in the last chunk are staged as
// zeros).  One barrier serves vb vectors, one 16-byte LDS read gives a tap for
// 16 / sizeof(T) vectors, and a point's outputs fill its output row in order,
// in 16-byte stores when vst (rows 16-byte aligned), else element by element.
// Taps are summed in the order of k_interp.
template <typename T, int D, int M, bool DER, int PT>
__global__ void __launch_bounds__(256)
k_interp_vb(const WinDesc *__restrict__ wd, const int *__restrict__ sub_win,
            const int *__restrict__ sub_bin, const int *__restrict__ sub_start,
            const int *__restrict__ sub_count, int tb, int nb, int ng, int nwin,
            const typename Cplx<T>::type *__restrict__ grid, int64_t cells, int nrhs, int vb,
            int vst, int64_t n, T *__restrict__ hbuf, T *__restrict__ dout, T dscale)
{
    static_assert(D <= 2, "d <= 2 only");
    using C = typename Cplx<T>::type;
    constexpr int CH = 16 / (int)sizeof(T);
    struct alignas(16) V { T x[CH]; };
    constexpr int TW = 2 * M;
    constexpr int RS = D * TW;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *tile = reinterpret_cast<T *>(smem_raw);
    const int pd = tb + 2 * M;
    const int pc = D == 1 ? pd : pd * pd;
    const int S = vb * (DER ? 2 : 1) + CH;   // values per staged cell
    const float inv_pd = 1.0f / (float)pd, inv_pc = 1.0f / (float)pc;
    const int sq = xcd_item(blockIdx.x, gridDim.x);
    const int wi = sub_win[sq];
    const WinDesc &win = wd[wi];
    gmem<T> *rec = (gmem<T> *)win.rec;
    const int start = sub_start[sq], cnt = sub_count[sq];
    int org[3] = {0, 0, 0};
    bin_origin<D>(sub_bin[sq] & 0xffffff, nb, tb, org);
    // the subproblem's points are taken 256 PT at a time (point k of a chunk
    // by thread k mod 256): a single chunk keeps its weights in registers for
    // every vector batch, longer subproblems reload them per batch and chunk
    bool mine[PT];
    T w[PT][D][TW];
    int lin[PT];
    int64_t orow[PT];
    auto load_pts = [&](int pc0) {
#pragma unroll
        for (int p = 0; p < PT; ++p) {
            const int k = pc0 + (int)threadIdx.x + 256 * p;
            mine[p] = k < cnt;
            const int64_t j = start + (mine[p] ? k : 0);
            gmem<T> *rp = rec + j * RS;
#pragma unroll
            for (int q = 0; q < D; ++q)
#pragma unroll
                for (int a = 0; a < TW; ++a) w[p][q][a] = rp[q * TW + a];
            lin[p] = ((gmem<int> *)win.lpos)[j] & 0xfffff;
            orow[p] = (int64_t)((gmem<int> *)win.perm)[j] * nrhs;
        }
    };
    const bool one_chunk = cnt <= 256 * PT;
    if (one_chunk) load_pts(0);
    T *hout = hbuf + (int64_t)win.s_global * n * nrhs;
    T *dblk = DER ? dout + (int64_t)win.s_global * n * nrhs : nullptr;
    for (int r0 = 0; r0 < nrhs; r0 += vb) {
        const int nv = min(vb, nrhs - r0);
        const int nch = (nv + CH - 1) / CH;   // 16-byte chunks of vectors in this batch
        if (r0 > 0) __syncthreads();
        // staging: unit u = (chunk, cell), cells fastest so that a wave's
        // grid reads run along grid rows; UB units per thread in flight
        constexpr int UB = 4;
        const int nu = nch * pc;
        for (int u0 = 0; u0 < nu; u0 += UB * 256) {
            V vK[UB], vD[UB];
            int dst[UB];
#pragma unroll
            for (int b = 0; b < UB; ++b) {
                const int u = u0 + b * 256 + (int)threadIdx.x;
                const bool ok = u < nu;
                const int ch = fdiv_small(ok ? u : 0, pc, inv_pc);
                const int cell = (ok ? u : 0) - ch * pc;
                bool in = ok;
                int64_t g;
                if constexpr (D == 1) {
                    const int l = org[0] - M + cell;
                    in = in && l >= 0 && l < ng;
                    g = l;
                } else {
                    const int a = fdiv_small(cell, pd, inv_pd);
                    const int l0 = org[0] - M + a, l1 = org[1] - M + (cell - a * pd);
                    in = in && l0 >= 0 && l0 < ng && l1 >= 0 && l1 < ng;
                    g = (int64_t)l0 * ng + l1;
                }
                dst[b] = ok ? cell * S + ch * CH : -1;
                const int vrow = r0 + ch * CH;
                const C *gK = grid + ((int64_t)wi * nrhs + vrow) * cells + (in ? g : 0);
                const C *gD = gK;   // derivative grid: imaginary parts
#pragma unroll
                for (int e = 0; e < CH; ++e) {
                    const bool ine = in && vrow + e < nrhs;
                    vK[b].x[e] = ine ? gK[(int64_t)e * cells].x : T(0);
                    vD[b].x[e] = (DER && ine) ? gD[(int64_t)e * cells].y : T(0);
                }
            }
#pragma unroll
            for (int b = 0; b < UB; ++b) {
                if (dst[b] < 0) continue;
                *reinterpret_cast<V *>(tile + dst[b]) = vK[b];
                if (DER) *reinterpret_cast<V *>(tile + dst[b] + vb) = vD[b];
            }
        }
        __syncthreads();
        for (int pc0 = 0; pc0 < cnt; pc0 += 256 * PT) {
        if (!one_chunk) load_pts(pc0);
#pragma unroll
        for (int p = 0; p < PT; ++p) {
            if (!mine[p]) continue;
#pragma unroll 1
            for (int c = 0; c < nch; ++c) {
                const T *tc = tile + c * CH;
                V hK, hD;
#pragma unroll
                for (int e = 0; e < CH; ++e) hK.x[e] = hD.x[e] = T(0);
                if constexpr (D == 1) {
#pragma unroll
                    for (int aa = 0; aa < TW; ++aa) {
                        const T *cp = tc + (lin[p] + aa) * S;
                        const V xK = *reinterpret_cast<const V *>(cp);
#pragma unroll
                        for (int e = 0; e < CH; ++e) hK.x[e] += xK.x[e] * w[p][0][aa];
                        if constexpr (DER) {
                            const V xD = *reinterpret_cast<const V *>(cp + vb);
#pragma unroll
                            for (int e = 0; e < CH; ++e) hD.x[e] += xD.x[e] * w[p][0][aa];
                        }
                    }
                } else {
#pragma unroll
                    for (int aa = 0; aa < TW; ++aa) {
                        V sK, sD;
#pragma unroll
                        for (int e = 0; e < CH; ++e) sK.x[e] = sD.x[e] = T(0);
                        const int row = lin[p] + aa * pd;
#pragma unroll
                        for (int bb = 0; bb < TW; ++bb) {
                            const T *cp = tc + (row + bb) * S;
                            const V xK = *reinterpret_cast<const V *>(cp);
#pragma unroll
                            for (int e = 0; e < CH; ++e) sK.x[e] += xK.x[e] * w[p][D - 1][bb];
                            if constexpr (DER) {
                                const V xD = *reinterpret_cast<const V *>(cp + vb);
#pragma unroll
                                for (int e = 0; e < CH; ++e) sD.x[e] += xD.x[e] * w[p][D - 1][bb];
                            }
                        }
#pragma unroll
                        for (int e = 0; e < CH; ++e) {
                            hK.x[e] += sK.x[e] * w[p][0][aa];
                            if (DER) hD.x[e] += sD.x[e] * w[p][0][aa];
                        }
                    }
                }
#pragma unroll
                for (int e = 0; e < CH; ++e) hD.x[e] *= dscale;
                const int64_t o = orow[p] + r0 + c * CH;
                if (vst) {
                    *reinterpret_cast<V *>(hout + o) = hK;
                    if (DER) *reinterpret_cast<V *>(dblk + o) = hD;
                } else {
                    const int ne = min(CH, nv - c * CH);
                    for (int e = 0; e < ne; ++e) {
                        hout[o + e] = hK.x[e];
                        if (DER) dblk[o + e] = hD.x[e];
                    }
                }
            }
        }
        }
    }
}

// Sum over the 64 lanes of a wave, returned in every lane.  FP32: DPP moves
// inside rows of 16 lanes (swap neighbours, swap pairs, rotate by 4 and by 8),
// then the four row sums are read with readlane; FP64 uses shuffles.
__device__ __forceinline__ float dpp_f(float v, int ctrl_sel)
{
    int x = __float_as_int(v), r;
    switch (ctrl_sel) {
    case 0: r = __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false); break;    // quad_perm [1,0,3,2]
    case 1: r = __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false); break;    // quad_perm [2,3,0,1]
    case 2: r = __builtin_amdgcn_update_dpp(0, x, 0x124, 0xF, 0xF, false); break;   // row_ror:4
    default: r = __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false); break;  // row_ror:8
    }
    return __int_as_float(r);
}

__device__ __forceinline__ float wave_sum(float v)
{
    v += dpp_f(v, 0);
    v += dpp_f(v, 1);
    v += dpp_f(v, 2);
    v += dpp_f(v, 3);
    const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (a + b) + (c + d);
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over each row of 16 lanes, returned in every lane of the row.
__device__ __forceinline__ float row_sum(float v)
{
    v += dpp_f(v, 0);
    v += dpp_f(v, 1);
    v += dpp_f(v, 2);
    v += dpp_f(v, 3);
    return v;
}

__device__ __forceinline__ double row_sum(double v)
{
    for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Interpolation for windows whose points come in long runs of equal cells.
// One wave per subproblem; lane (b, c) holds the (b, c) tap column of the
// run's grid footprint in registers (loaded once per run and vector), so each
// point costs 2m FMAs per column plus one cross-lane sum, instead of (2m)^d
// LDS reads per thread.  Point data are staged in LDS in chunks of 64.
template <typename T, int D, int M, bool DER>
__global__ void __launch_bounds__(64)
k_interp_run(const WinDesc *__restrict__ wd, const int *__restrict__ sub_win,
             const int *__restrict__ sub_start, const int *__restrict__ sub_count, int ng, int tb, int nwin,
             const typename Cplx<T>::type *__restrict__ grid, int64_t cells, int nrhs, int64_t n,
             T *__restrict__ hbuf, T *__restrict__ dout, T dscale)
{
    constexpr int TW = 2 * M;
    constexpr int RS = D * TW;
    constexpr int NITEM = D == 1 ? TW : TW * TW;
    constexpr int NG = (NITEM + 63) / 64;
    constexpr int NA = D == 3 ? TW : 1;
    constexpr int CH = 64;
    __shared__ T s_rec[CH * RS];
    __shared__ int s_an[CH];
    __shared__ int s_perm[CH];
    __shared__ T s_part[CH][4], s_partD[CH][4];
    const int lane = threadIdx.x;
    const int sblk = xcd_item(blockIdx.x, gridDim.x);
    const int wi = sub_win[sblk];
    const WinDesc &win = wd[wi];
    gmem<T> *rec = (gmem<T> *)win.rec;
    const int start = sub_start[sblk], cnt = sub_count[sblk];
    const int end = start + cnt;
    // 3-D windows with 16 items past the last full group of 64 (m = 2, 6):
    // that group is spread over the wave as (item, quarter of the first
    // dimension's taps) instead of leaving 48 lanes idle
    constexpr bool SPLIT = D == 3 && (NITEM % 64) == 16;
    constexpr int NGF = SPLIT ? NG - 1 : NG;   // groups handled item-per-lane
    constexpr int QA = TW / 4;
    const int itL = 64 * NGF + (lane & 15), qL = lane >> 4;
    const int i0L = itL / TW, i1L = itL % TW;
    int i0[NG], i1[NG];
    T actv[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int it = lane + 64 * g;
        const bool a = it < NITEM;
        actv[g] = a ? T(1) : T(0);
        const int itc = a ? it : 0;
        i0[g] = D == 1 ? itc : itc / TW;
        i1[g] = D == 1 ? 0 : itc % TW;
    }
    T *hout = hbuf + (int64_t)win.s_global * n * nrhs;
    T *dblk = DER ? dout + (int64_t)win.s_global * n * nrhs : nullptr;
    for (int cb = start; cb < end; cb += CH) {
        const int nc = min(CH, end - cb);
        __syncthreads();
        {
            // all loads of the chunk in flight before the LDS stores
            T v[RS];
#pragma unroll
            for (int k = 0; k < RS; ++k) {
                const int i = lane + 64 * k;
                v[k] = i < nc * RS ? rec[(int64_t)cb * RS + i] : T(0);
            }
            const int an = lane < nc ? ((gmem<int> *)win.anchor)[cb + lane] & 0x7fffffff : 0;
            const int pm = lane < nc ? ((gmem<int> *)win.perm)[cb + lane] : 0;
#pragma unroll
            for (int k = 0; k < RS; ++k) s_rec[lane + 64 * k] = v[k];
            s_an[lane] = an;
            s_perm[lane] = pm;
        }
        __syncthreads();
        for (int r = 0; r < nrhs; ++r) {
            const typename Cplx<T>::type *gK = grid + ((int64_t)wi * nrhs + r) * cells;
            const typename Cplx<T>::type *gD = gK;   // derivative grid: imaginary parts
            T G[NG][NA], GD[NG][NA], GL[QA], GDL[QA];
            int cur = -1, fr = 0;   // fr: first tap's tile position (first-dimension weights sit rotated by it)
            for (int u = 0; u < nc; ++u) {
                const int an = s_an[u];
                if (an != cur) {
                    cur = an;
                    int c[3] = {0, 0, 0}, cell = an;
                    for (int q = D - 1; q >= 0; --q) {
                        c[q] = cell % ng - M + 1;
                        cell /= ng;
                    }
                    fr = (c[0] + M - 1) % tb + 1;
                    if (SPLIT) {
#pragma unroll
                        for (int k = 0; k < QA; ++k) {
                            const int64_t gi = ((int64_t)(c[0] + qL * QA + k) * ng + c[1] + i0L) * ng + c[2] + i1L;
                            GL[k] = gK[gi].x;
                            if (DER) GDL[k] = gD[gi].y;
                        }
                    }
#pragma unroll
                    for (int g = 0; g < NGF; ++g)
#pragma unroll
                        for (int a = 0; a < NA; ++a) {
                            int64_t gi;
                            if (D == 3) gi = ((int64_t)(c[0] + a) * ng + c[1] + i0[g]) * ng + c[2] + i1[g];
                            else if (D == 2) gi = (int64_t)(c[0] + i0[g]) * ng + c[1] + i1[g];
                            else gi = c[0] + i0[g];
                            G[g][a] = gK[gi].x;
                            if (DER) GD[g][a] = gD[gi].y;
                        }
                }
                const T *rp = s_rec + u * RS;
                T t = T(0), td = T(0);
                if (SPLIT) {
                    T sk = T(0), sd = T(0);
#pragma unroll
                    for (int k = 0; k < QA; ++k) {
                        const T w0 = rp[(fr + qL * QA + k) % TW];
                        sk += w0 * GL[k];
                        if (DER) sd += w0 * GDL[k];
                    }
                    const T wbc = rp[TW + i0L] * rp[2 * TW + i1L];
                    t += sk * wbc;
                    if (DER) td += sd * wbc;
                }
#pragma unroll
                for (int g = 0; g < NGF; ++g) {
                    if (D == 3) {
                        T sk = T(0), sd = T(0);
#pragma unroll
                        for (int a = 0; a < NA; ++a) {
                            const T w0 = rp[(fr + a) % TW];
                            sk += w0 * G[g][a];
                            if (DER) sd += w0 * GD[g][a];
                        }
                        const T wbc = actv[g] * rp[TW + i0[g]] * rp[2 * TW + i1[g]];
                        t += sk * wbc;
                        if (DER) td += sd * wbc;
                    } else if (D == 2) {
                        const T wab = actv[g] * rp[i0[g]] * rp[TW + i1[g]];
                        t += G[g][0] * wab;
                        if (DER) td += GD[g][0] * wab;
                    } else {
                        const T wa = actv[g] * rp[i0[g]];
                        t += G[g][0] * wa;
                        if (DER) td += GD[g][0] * wa;
                    }
                }
                // sums over the rows of 16 lanes now; the four row sums of
                // every point are added once the chunk is done
                const T h = row_sum(t);
                if ((lane & 15) == 0) s_part[u][lane >> 4] = h;
                if (DER) {
                    const T hd = row_sum(td);
                    if ((lane & 15) == 0) s_partD[u][lane >> 4] = hd;
                }
            }
            __builtin_amdgcn_wave_barrier();
            if (lane < nc) {
                const int64_t o = (int64_t)s_perm[lane] * nrhs + r;
                hout[o] = (s_part[lane][0] + s_part[lane][1]) + (s_part[lane][2] + s_part[lane][3]);
                if (DER)
                    dblk[o] = dscale * ((s_partD[lane][0] + s_partD[lane][1]) +
                                        (s_partD[lane][2] + s_partD[lane][3]));
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
}

// sigma_f^2 sum_s h^(s) + sigma_eps^2 v, summed over windows in order with
// Kahan compensation; derivative blocks for sigma_f and sigma_eps.
template <typename T>
__global__ void k_assemble(int64_t n, int nrhs, int P, const T *__restrict__ V, int64_t ldv,
                           const T *__restrict__ hbuf, T sf2, T se2, T two_sf, T two_se,
                           T *__restrict__ KV, T *__restrict__ dsf, T *__restrict__ dse)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = n * nrhs;
    if (idx >= tot) return;
    int64_t i;
    int r;
    if (tot < (int64_t(1) << 31)) {   // 32-bit division suffices
        const unsigned q = (unsigned)idx / (unsigned)nrhs;
        i = q;
        r = (int)((unsigned)idx - q * (unsigned)nrhs);
    } else {
        i = idx / nrhs;
        r = (int)(idx % nrhs);
    }
    const T v = V[i * ldv + r];
    // windows in order (compensated sum); the loads of eight windows are
    // issued together
    T s = T(0), c = T(0);
    for (int w0 = 0; w0 < P; w0 += 8) {
        T h[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) h[j] = w0 + j < P ? hbuf[(int64_t)(w0 + j) * tot + idx] : T(0);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (w0 + j < P) {
                const T y = h[j] - c;
                const T t = s + y;
                c = (t - s) - y;
                s = t;
            }
        }
    }
    KV[idx] = sf2 * s + se2 * v;
    if (dsf) dsf[idx] = two_sf * s;
    if (dse) dse[idx] = two_se * v;
}

// Kernels that need more than 64 KiB of dynamic LDS must say so before launch.
// Vectors per staging of k_interp_vb: the batch count is the smallest whose
// tiles (pc cells of vb values, twice that with derivatives, plus 16 bytes of
// padding per cell) fit lds bytes, and the vectors are then dealt evenly in
// 16-byte chunks.  0 (one vector per staging) when nrhs is below a chunk or
// one chunk does not fit.
int interp_vectors_per_batch(int pc, int nrhs, bool der, int tsize, size_t lds)
{
    const int ch = 16 / tsize;
    if (nrhs < ch || pc <= 0) return 0;
    const long per_cell = (long)(lds / (size_t)pc) - 16;
    int vmax = (int)(per_cell / ((der ? 2 : 1) * tsize));
    vmax -= vmax % ch;
    if (vmax < ch) return 0;
    const int nbatch = (nrhs + vmax - 1) / vmax;
    int vb = (nrhs + nbatch - 1) / nbatch;
    vb += (ch - vb % ch) % ch;
    return vb;
}

template <typename K>
hipError_t allow_lds(K kernel, size_t bytes)
{
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename T, int D, int M, int R, int W>
hipError_t spread_launch(const Group &G, const void *V, int64_t ldv, int nrhs, void *tilebuf,
                         hipStream_t s)
{
    const WindowGeom &g = G.g;
    const size_t shm = (size_t)g.pc * sizeof(T) * R;
    dim3 grid((unsigned)G.nsub, (unsigned)((nrhs + R - 1) / R));
    // four-point form for one vector per work-group unless the group asks
    // for the run-ordered form (spread_form: 0 rule, 1 four-point, 2 runs)
    const bool quad = G.spread_form == 1 || (G.spread_form == 0 && R == 1);
    hipError_t e;
    if (quad) {
        e = allow_lds(k_spread<T, D, M, R, W>, shm);
        if (e != hipSuccess) return e;
        k_spread<T, D, M, R, W><<<grid, 64 * W, shm, s>>>(G.desc, G.sub_win, G.sub_start, G.sub_count,
                                                            (const T *)V, ldv, nrhs, g.pd, (T *)tilebuf);
    } else {
        e = allow_lds(k_spread_run<T, D, M, R, W>, shm);
        if (e != hipSuccess) return e;
        k_spread_run<T, D, M, R, W><<<grid, 64 * W, shm, s>>>(G.desc, G.sub_win, G.sub_start, G.sub_count,
                                                                (const T *)V, ldv, nrhs, g.pd, (T *)tilebuf);
    }
    return hipGetLastError();
}

constexpr bool kSpreadMfmaRule = true;

// Vectors per work-group of the VALU spreading forms.  d = 3: four waves
// share a tile (2m taps split four ways).  R vectors per work-group share the
// points' weights; R tiles must fit in 64 KiB, and R = 4 is taken only when
// it leaves no partial group of vectors (measured: 32 vectors 4 > 2 > 1,
// 17 vectors 2 > 1 > 4, 16 vectors of m = 6: 2 > 1)
int spread_vectors_per_group(const Group &G, int nrhs, size_t tsize)
{
    const size_t tile = (size_t)G.g.pc * tsize;
    int R = 1;
    if (G.spread_R > 0) {
        R = G.spread_R;
        if (R * tile > 64 * 1024 || R > nrhs) R = (2 * tile <= 64 * 1024 && nrhs >= 2) ? 2 : 1;
    } else if (nrhs % 4 == 0 && 4 * tile <= 64 * 1024) {
        R = 4;
    } else if (nrhs >= 2 && 2 * tile <= 64 * 1024) {
        R = 2;
    }
    return R;
}

// Matrix-core spreading applies to FP32, d = 3, 2m = 8 or 12 and tiles whose
// four vectors fit the LDS next to the staged points.
constexpr size_t kSpreadMfmaLds = 148 * 1024;

template <typename T, int D, int M>
bool spread_mfma_ok(const Group &G)
{
    return std::is_same<T, float>::value && D == 3 && (M == 4 || M == 6) &&
           (size_t)spread_mfma_pad(G.g.pd).sr * sizeof(float) * 4 <= kSpreadMfmaLds;
}

template <int M, int R>
hipError_t spread_mfma_launch(const Group &G, const void *V, int64_t ldv, int nrhs, void *tilebuf,
                              hipStream_t s)
{
    constexpr int NW = SpreadMfmaShape<M, R>::NWAVE;
    const size_t shm = (size_t)spread_mfma_pad(G.g.pd).sr * sizeof(float) * R;
    hipError_t e = allow_lds(k_spread_mfma<M, R>, shm);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)G.nsub, (unsigned)((nrhs + R - 1) / R));
    k_spread_mfma<M, R><<<grid, 64 * NW, shm, s>>>(G.desc, G.sub_win, G.sub_start, G.sub_count,
                                                   (const float *)V, ldv, nrhs, G.g.pd, (float *)tilebuf);
    return hipGetLastError();
}

template <typename T, int D, int M>
hipError_t spread_dm(const Group &G, const void *V, int64_t ldv, int nrhs, void *tilebuf,
                     hipStream_t s)
{
    // matrix-core form: by request (spread_form 3), or by rule for four or
    // more vectors at 2m = 12 (at 2m = 8 the VALU run form was measured
    // faster: C3 3-D group 1.3 vs 1.56 ms; the tuner tries both)
    if constexpr (std::is_same<T, float>::value && D == 3 && (M == 4 || M == 6)) {
        if (spread_mfma_ok<T, D, M>(G) &&
            (G.spread_form == 3 || (G.spread_form == 0 && nrhs >= 4 && M == 6 && kSpreadMfmaRule)))
            return G.spread_mfma_R == 2 ? spread_mfma_launch<M, 2>(G, V, ldv, nrhs, tilebuf, s)
                                        : spread_mfma_launch<M, 4>(G, V, ldv, nrhs, tilebuf, s);
    }
    const int R = spread_vectors_per_group(G, nrhs, sizeof(T));
    // waves sharing a tile: 4 for d = 3 unless the group asks for 2
    auto go = [&](auto w_tag) -> hipError_t {
        constexpr int W = decltype(w_tag)::value;
        if (R == 4) return spread_launch<T, D, M, 4, W>(G, V, ldv, nrhs, tilebuf, s);
        if (R == 2) return spread_launch<T, D, M, 2, W>(G, V, ldv, nrhs, tilebuf, s);
        return spread_launch<T, D, M, 1, W>(G, V, ldv, nrhs, tilebuf, s);
    };
    if constexpr (D == 3) {
        if (G.spread_W == 2) return go(std::integral_constant<int, 2>());
        return go(std::integral_constant<int, 4>());
    } else {
        return go(std::integral_constant<int, 1>());
    }
}

template <typename T, int D, int M>
hipError_t interp_dm(const Group &G, int64_t n, int nrhs, const void *grid, bool with_der,
                     void *hbuf, void *dout, double dscale, hipStream_t s)
{
    const WindowGeom &g = G.g;
    using C = typename Cplx<T>::type;
    if (G.use_run_interp) {
        if (with_der)
            k_interp_run<T, D, M, true><<<(unsigned)G.nrsub, 64, 0, s>>>(
                G.desc, G.rsub_win, G.rsub_start, G.rsub_count, g.ng, g.tb, G.nwin, (const C *)grid, g.cells,
                nrhs, n, (T *)hbuf, (T *)dout, (T)dscale);
        else
            k_interp_run<T, D, M, false><<<(unsigned)G.nrsub, 64, 0, s>>>(
                G.desc, G.rsub_win, G.rsub_start, G.rsub_count, g.ng, g.tb, G.nwin, (const C *)grid, g.cells,
                nrhs, n, (T *)hbuf, nullptr, (T)dscale);
        return hipGetLastError();
    }
    if constexpr (std::is_same<T, float>::value && D == 2 && (M == 4 || M == 6)) {
        if (G.interp_mfma) {
            constexpr int CS = kInterp2Values + 4;
            const int rstr = g.pd * CS + ((8 - g.pd * CS) % 32 + 32) % 32;
            const size_t shm = (size_t)g.pd * rstr * sizeof(float);
            auto go = [&](auto der_tag) -> hipError_t {
                constexpr bool DR = decltype(der_tag)::value;
                hipError_t e = allow_lds(k_interp_mfma2<M, DR>, shm);
                if (e != hipSuccess) return e;
                k_interp_mfma2<M, DR><<<(unsigned)G.nisub, 256, shm, s>>>(
                    G.desc, G.isub_win, G.isub_bin, G.isub_start, G.isub_count, g.tb, g.nb, g.ng,
                    (const float2 *)grid, g.cells, nrhs, n, (float *)hbuf, DR ? (float *)dout : nullptr,
                    (float)dscale);
                return hipGetLastError();
            };
            return with_der ? go(std::true_type()) : go(std::false_type());
        }
    }
    if constexpr (D <= 2) {
        // several vectors per staging from 16 bytes of vectors on; 16-byte
        // output stores when the output rows are 16-byte aligned
        const int vb = G.interp_vb_lds > 0
                           ? interp_vectors_per_batch(g.pc, nrhs, with_der, (int)sizeof(T), G.interp_vb_lds)
                           : 0;
        const int vst = nrhs % (16 / (int)sizeof(T)) == 0 && reinterpret_cast<uintptr_t>(hbuf) % 16 == 0 &&
                        (!with_der || reinterpret_cast<uintptr_t>(dout) % 16 == 0);
        if (vb > 0) {
            const size_t shm = (size_t)g.pc * (vb * (with_der ? 2 : 1) + 16 / sizeof(T)) * sizeof(T);
            auto go = [&](auto der_tag, auto pt_tag) -> hipError_t {
                constexpr bool DR = decltype(der_tag)::value;
                constexpr int PT = decltype(pt_tag)::value;
                hipError_t e = allow_lds(k_interp_vb<T, D, M, DR, PT>, shm);
                if (e != hipSuccess) return e;
                k_interp_vb<T, D, M, DR, PT><<<(unsigned)G.nvsub, 256, shm, s>>>(
                    G.desc, G.vsub_win, G.vsub_bin, G.vsub_start, G.vsub_count, g.tb, g.nb, g.ng, G.nwin,
                    (const C *)grid, g.cells, nrhs, vb, vst, n, (T *)hbuf, DR ? (T *)dout : nullptr,
                    (T)dscale);
                return hipGetLastError();
            };
            using t1 = std::integral_constant<int, 1>;
            using t2 = std::integral_constant<int, 2>;
            if (with_der)
                return G.interp_pt == 2 ? go(std::true_type(), t2()) : go(std::true_type(), t1());
            return G.interp_pt == 2 ? go(std::false_type(), t2()) : go(std::false_type(), t1());
        }
    }
    // the 3-D staging covers a padded plane of at most (8 + 2m)^2 cells and
    // rows <= pd first-axis rows of it
    const int rows = D == 3 ? G.interp_rows : g.pd;
    if (D == 3 && (g.pd > 8 + 2 * M || rows < 2 * M || rows > g.pd)) return hipErrorInvalidValue;
    if constexpr (std::is_same<T, float>::value && D == 3 && (M == 4 || M == 6)) {
        if (G.interp_mfma) {
            const int pd2 = g.pd * g.pd;
            const int ps = 4 * pd2 + ((8 - 4 * pd2) % 32 + 32) % 32;
            const size_t shm = (size_t)rows * ps * sizeof(float);
            auto go = [&](auto der_tag, auto nw_tag) -> hipError_t {
                constexpr bool DR = decltype(der_tag)::value;
                constexpr int NW = decltype(nw_tag)::value;
                // 16 waves keep the weights in LDS; 8 waves read them from L2
                // so that two work-groups share a CU
                constexpr bool WL = NW == 16;
                hipError_t e = allow_lds(k_interp_mfma<M, DR, NW, WL>, shm);
                if (e != hipSuccess) return e;
                k_interp_mfma<M, DR, NW, WL><<<(unsigned)G.nisub, 64 * NW, shm, s>>>(
                    G.desc, G.isub_win, G.isub_bin, G.isub_start, G.isub_count, g.tb, g.nb, g.ng, rows,
                    (const float2 *)grid, g.cells, nrhs, n, (float *)hbuf, DR ? (float *)dout : nullptr,
                    (float)dscale);
                return hipGetLastError();
            };
            using w8 = std::integral_constant<int, 8>;
            using w16 = std::integral_constant<int, 16>;
            if (G.interp_mfma_waves == 8) return with_der ? go(std::true_type(), w8()) : go(std::false_type(), w8());
            return with_der ? go(std::true_type(), w16()) : go(std::false_type(), w16());
        }
    }
    const size_t cells_staged = D == 3 ? (size_t)rows * g.pd * g.pd : (size_t)g.pc;
    size_t shm = cells_staged * sizeof(T) * (with_der ? 2 : 1);
    auto go = [&](auto der_tag, auto pt_tag) -> hipError_t {
        constexpr bool DR = decltype(der_tag)::value;
        constexpr int PT = decltype(pt_tag)::value;
        if constexpr (D == 3 && PT == 2) {
            if (G.interp_slot) {
                hipError_t e = allow_lds(k_interp<T, D, M, DR, 2, true, true>, shm);
                if (e != hipSuccess) return e;
                k_interp<T, D, M, DR, 2, true, true><<<(unsigned)G.nisub, 256, shm, s>>>(
                    G.desc, G.isub_win, G.isub_bin, G.isub_start, G.isub_count, g.tb, g.nb, g.ng, G.nwin, rows,
                    (const C *)grid, g.cells, nrhs, n, (T *)hbuf, DR ? (T *)dout : nullptr, (T)dscale);
                return hipGetLastError();
            }
            if (G.interp_adj) {
                hipError_t e = allow_lds(k_interp<T, D, M, DR, 2, true>, shm);
                if (e != hipSuccess) return e;
                k_interp<T, D, M, DR, 2, true><<<(unsigned)G.nisub, 256, shm, s>>>(
                    G.desc, G.isub_win, G.isub_bin, G.isub_start, G.isub_count, g.tb, g.nb, g.ng, G.nwin, rows,
                    (const C *)grid, g.cells, nrhs, n, (T *)hbuf, DR ? (T *)dout : nullptr, (T)dscale);
                return hipGetLastError();
            }
        }
        hipError_t e = allow_lds(k_interp<T, D, M, DR, PT>, shm);
        if (e != hipSuccess) return e;
        k_interp<T, D, M, DR, PT><<<(unsigned)G.nisub, 256, shm, s>>>(
            G.desc, G.isub_win, G.isub_bin, G.isub_start, G.isub_count, g.tb, g.nb, g.ng, G.nwin, rows,
            (const C *)grid, g.cells, nrhs, n, (T *)hbuf, DR ? (T *)dout : nullptr, (T)dscale);
        return hipGetLastError();
    };
    using t1 = std::integral_constant<int, 1>;
    using t2 = std::integral_constant<int, 2>;
    if (with_der)
        return G.interp_pt == 2 ? go(std::true_type(), t2()) : go(std::true_type(), t1());
    return G.interp_pt == 2 ? go(std::false_type(), t2()) : go(std::false_type(), t1());
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
hipError_t spread_t(const Group &G, int m, const void *V, int64_t ldv, int nrhs, void *tilebuf,
                    hipStream_t s)
{
    switch (G.g.d) {
    case 1: NFFTGP_DISPATCH_DM(spread_dm, T, 1, m, G, V, ldv, nrhs, tilebuf, s)
    case 2: NFFTGP_DISPATCH_DM(spread_dm, T, 2, m, G, V, ldv, nrhs, tilebuf, s)
    case 3: NFFTGP_DISPATCH_DM(spread_dm, T, 3, m, G, V, ldv, nrhs, tilebuf, s)
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t interp_t(const Group &G, int m, int64_t n, int nrhs, const void *grid, bool with_der,
                    void *hbuf, void *dout, double dscale, hipStream_t s)
{
    switch (G.g.d) {
    case 1: NFFTGP_DISPATCH_DM(interp_dm, T, 1, m, G, n, nrhs, grid, with_der, hbuf, dout, dscale, s)
    case 2: NFFTGP_DISPATCH_DM(interp_dm, T, 2, m, G, n, nrhs, grid, with_der, hbuf, dout, dscale, s)
    case 3: NFFTGP_DISPATCH_DM(interp_dm, T, 3, m, G, n, nrhs, grid, with_der, hbuf, dout, dscale, s)
    default: return hipErrorInvalidValue;
    }
}

// 3-D fold by tiles: work-group (tile of the occupied box, window and
// vector) reads the first subproblem of the 27 tiles around its tile once,
// then each cell of the tile sums the covering tiles' values (a cell of tile
// b is covered by tiles b - 1, b, b + 1 per axis at most, since m <= tb), in
// increasing tile order as k_fold does, so the sums agree bit for bit.
// Cells outside the occupied box are not written, as in k_fold.  Rows
// blockIdx.y >= nwr: the group's separable coefficients, as in k_fold.
template <typename T>
__global__ void __launch_bounds__(256)
k_fold_tiles(const WinDesc *__restrict__ wd, const T *__restrict__ tilebuf, int nrhs, int tb, int nb,
             int ng, int m, int pd, int pc, int64_t cells, int olo, int on, int t0, int nt,
             typename Cplx<T>::type *__restrict__ grid, int nwr, int coef_blocks, int coef_nper, int cd,
             int cN, CoefParams prm, const double *__restrict__ cinv2, const double *__restrict__ cw,
             double *__restrict__ cpart)
{
    if ((int)blockIdx.y >= nwr) {
        __shared__ double lds[4 * kCoefMaxH + 256];
        const int cb = ((int)blockIdx.y - nwr) * (int)gridDim.x + (int)blockIdx.x;
        if (cb >= coef_blocks) return;
        const int blk = cb % coef_nper, aw = cb / coef_nper;
        coef_sep_block<T>(cd, cN, prm, cinv2, cw, wd, cpart, blk, coef_nper, aw % 2, aw / 2, lds);
        return;
    }
    __shared__ int s_first[27];
    const int wr = blockIdx.y;
    const int w = wr / nrhs, r = wr % nrhs;
    const int ti = xcd_item(blockIdx.x, gridDim.x);
    const int b0 = t0 + ti / (nt * nt), b1 = t0 + (ti / nt) % nt, b2 = t0 + ti % nt;
    if (threadIdx.x < 27) {
        const int c0 = b0 + (int)threadIdx.x / 9 - 1, c1 = b1 + ((int)threadIdx.x / 3) % 3 - 1,
                  c2 = b2 + (int)threadIdx.x % 3 - 1;
        int s0 = -1;
        if (c0 >= 0 && c0 < nb && c1 >= 0 && c1 < nb && c2 >= 0 && c2 < nb) {
            gmem<int> *bsp = (gmem<int> *)wd[w].bin_sub_ptr;
            const int bin = (c0 * nb + c1) * nb + c2;
            if (bsp[bin + 1] > bsp[bin]) s0 = bsp[bin];
        }
        s_first[threadIdx.x] = s0;
    }
    __syncthreads();
    const int sh = __ffs(tb) - 1;   // tb is a power of two
    const T *tr = tilebuf + (int64_t)r * pc;
    for (int q = threadIdx.x; q < tb * tb * tb; q += 256) {
        const int x = q >> (2 * sh), y = (q >> sh) & (tb - 1), z = q & (tb - 1);
        const int l0 = b0 * tb + x, l1 = b1 * tb + y, l2 = b2 * tb + z;
        if (l0 < olo || l0 >= olo + on || l1 < olo || l1 >= olo + on || l2 < olo || l2 >= olo + on) continue;
        T sum = T(0);
#pragma unroll
        for (int u0 = 0; u0 < 3; ++u0) {
            const int i0 = x - (u0 - 1) * tb + m;
            if (i0 < 0 || i0 >= pd) continue;
#pragma unroll
            for (int u1 = 0; u1 < 3; ++u1) {
                const int i1 = y - (u1 - 1) * tb + m;
                if (i1 < 0 || i1 >= pd) continue;
#pragma unroll
                for (int u2 = 0; u2 < 3; ++u2) {
                    const int i2 = z - (u2 - 1) * tb + m;
                    const int s0 = s_first[(u0 * 3 + u1) * 3 + u2];
                    if (i2 < 0 || i2 >= pd || s0 < 0) continue;
                    sum += tr[(int64_t)s0 * nrhs * pc + (i0 * pd + i1) * pd + i2];
                }
            }
        }
        typename Cplx<T>::type o;
        o.x = sum;
        o.y = T(0);
        grid[(int64_t)wr * cells + ((int64_t)l0 * ng + l1) * ng + l2] = o;
    }
}

// 3-D fold by tiles of the occupied box (k_fold_tiles) when cells have up to
// 27 covering tiles (m > tb / 2) and there are many window-vector rows; per
// cell (k_fold) otherwise: at m = 4 every cell has 8 covering tiles and the
// per-cell form's longer contiguous runs win.  Fold per launch, tiles vs
// cells: n = 2e6, m = 6, 6 windows x 16 vectors 0.73 vs 0.89 ms; n = 5e5,
// m = 4, 32 vectors 68 vs 57 us; n = 1e5, m = 4, 3 windows x 1 vector 21 vs
// 17 us.  G.fold_form 1 / 2 forces cells / tiles.
bool fold_by_tiles(const Group &G, int m, int nrhs)
{
    if (G.g.d != 3) return false;
    if (G.fold_form != 0) return G.fold_form == 2;
    return 2 * m > G.g.tb && G.nwin * nrhs >= 32;
}

template <typename T>
hipError_t fold_t(const Group &G, int m, int nrhs, void *tilebuf, void *grid, bool with_coef, hipStream_t s)
{
    const WindowGeom &g = G.g;
    using C = typename Cplx<T>::type;
    // k_fold visits at most 3 covering tiles per axis
    if (g.pd > 3 * g.tb) return hipErrorInvalidValue;
    if (G.nfb > 0)
        k_fold_bins<T><<<dim3((unsigned)((g.pc + 63) / 64), (unsigned)G.nfb, (unsigned)nrhs), 256, 0, s>>>(
            G.desc, G.fb, (T *)tilebuf, g.nbins, nrhs, g.pc);
    // occupied cells per axis: N/2 - m + 1 .. 3N/2 + m (every t lies in [N/2, 3N/2])
    const int olo = g.N / 2 - m + 1, on = g.N + 2 * m;
    int64_t ocells = 1;
    for (int q = 0; q < g.d; ++q) ocells *= on;
    const int gx = (int)((ocells + 255) / 256), nwr = G.nwin * nrhs;
    // coefficient blocks: (N+1)^d / 256 per window and array, in extra rows
    int64_t KD = 1;
    for (int q = 0; q < g.d; ++q) KD *= g.N + 1;
    const int nper = (int)((KD + 255) / 256);
    const int coef_blocks = with_coef ? nper * 2 * G.nwin : 0;
    const int crows = (coef_blocks + gx - 1) / gx;
    const dim3 fgrid((unsigned)gx, (unsigned)(nwr + crows));
#define NFFTGP_FOLD(DD)                                                                              \
    k_fold<T, DD><<<fgrid, 256, 0, s>>>(G.desc, (const T *)tilebuf, nrhs, g.tb, g.nb, g.ng, m, g.pd, \
                                        g.pc, g.cells, olo, on, (int)ocells, (C *)grid, nwr,      \
                                        coef_blocks, nper, g.d, g.N, G.prm, G.cinv2, G.cw, G.coef_part);
    switch (fold_by_tiles(G, m, nrhs) ? 4 : g.d) {
    case 1: NFFTGP_FOLD(1) break;
    case 2: NFFTGP_FOLD(2) break;
    case 3: NFFTGP_FOLD(3) break;
    case 4: {
        const int t0 = olo / g.tb, nt = (olo + on - 1) / g.tb - t0 + 1;
        const int tx = nt * nt * nt;
        const dim3 tgrid((unsigned)tx, (unsigned)(nwr + (coef_blocks + tx - 1) / tx));
        k_fold_tiles<T><<<tgrid, 256, 0, s>>>(G.desc, (const T *)tilebuf, nrhs, g.tb, g.nb, g.ng, m, g.pd, g.pc,
                                              g.cells, olo, on, t0, nt, (C *)grid, nwr, coef_blocks, nper, g.d,
                                              g.N, G.prm, G.cinv2, G.cw, G.coef_part);
        break;
    }
    default: return hipErrorInvalidValue;
    }
#undef NFFTGP_FOLD
    return hipGetLastError();
}

}  // namespace

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

hipError_t launch_spread(int prec, const Group &G, int m, const void *V, int64_t ldv, int nrhs,
                         void *tilebuf, hipStream_t s)
{
    if (G.nsub == 0) return hipSuccess;
    return prec == NFFTGP_F32 ? spread_t<float>(G, m, V, ldv, nrhs, tilebuf, s)
                              : spread_t<double>(G, m, V, ldv, nrhs, tilebuf, s);
}

hipError_t launch_fold(int prec, const Group &G, int m, int nrhs, void *tilebuf, void *grid,
                       bool with_coef, hipStream_t s)
{
    return prec == NFFTGP_F32 ? fold_t<float>(G, m, nrhs, tilebuf, grid, with_coef, s)
                              : fold_t<double>(G, m, nrhs, tilebuf, grid, with_coef, s);
}

hipError_t launch_interp(int prec, const Group &G, int m, int64_t n, int nrhs, const void *grid,
                         bool with_der, void *hbuf, void *dout, double dscale, hipStream_t s)
{
    if (G.nisub == 0 && G.nrsub == 0) return hipSuccess;
    return prec == NFFTGP_F32
               ? interp_t<float>(G, m, n, nrhs, grid, with_der, hbuf, dout, dscale, s)
               : interp_t<double>(G, m, n, nrhs, grid, with_der, hbuf, dout, dscale, s);
}

std::string describe_group(int prec, const Group &G, int m, int nrhs)
{
    std::string sp;
    const bool mfma_ok = prec == NFFTGP_F32 && G.g.d == 3 && (m == 4 || m == 6) &&
                         (size_t)spread_mfma_pad(G.g.pd).sr * sizeof(float) * 4 <= kSpreadMfmaLds;
    if (mfma_ok && (G.spread_form == 3 || (G.spread_form == 0 && nrhs >= 4 && m == 6 && kSpreadMfmaRule))) {
        sp = "mfma (4 vectors per work-group)";
    } else {
        const int R = spread_vectors_per_group(G, nrhs, prec == NFFTGP_F32 ? 4 : 8);
        const bool quad = G.spread_form == 1 || (G.spread_form == 0 && R == 1);
        sp = std::string(quad ? "four-point" : "run") + " (" + std::to_string(R) + " vectors per work-group" +
             (G.g.d == 3 ? (G.spread_W == 2 ? ", 2 waves per tile)" : ", 4 waves per tile)") : ")");
    }
    std::string ip;
    if (G.use_run_interp)
        ip = "run";
    else if (G.interp_mfma)
        ip = "mfma (" + std::to_string(G.g.d == 2 ? 4 : G.interp_mfma_waves) + " waves per work-group)";
    else if (G.interp_slot)
        ip = "tileslot";
    else if (G.interp_adj)
        ip = "tilepair";
    else
        ip = G.interp_pt == 2 ? "tile2" : "tile";
    if (!G.use_run_interp && G.g.d == 3)
        ip += ", " + std::to_string(G.interp_rows) + " of " + std::to_string(G.g.pd) + " rows staged";
    return "group d=" + std::to_string(G.g.d) + " N=" + std::to_string(G.g.N) + " windows=" +
           std::to_string(G.nwin) + ": spread=" + sp + "; subproblem " + std::to_string(G.sub_sp) +
           " points; interp=" + ip + "; fold=" + (fold_by_tiles(G, m, nrhs) ? "tiles" : "cells") + "\n";
}

hipError_t launch_assemble(int prec, int64_t n, int nrhs, int P, const void *V, int64_t ldv,
                           const void *hbuf, double sf, double se, void *KV, void *dsf, void *dse,
                           hipStream_t s)
{
    int64_t tot = n * nrhs;
    if (tot == 0) return hipSuccess;
    unsigned nblk = (unsigned)((tot + 255) / 256);
    if (prec == NFFTGP_F32)
        k_assemble<float><<<nblk, 256, 0, s>>>(n, nrhs, P, (const float *)V, ldv, (const float *)hbuf,
                                               (float)(sf * sf), (float)(se * se), (float)(2 * sf),
                                               (float)(2 * se), (float *)KV, (float *)dsf,
                                               (float *)dse);
    else
        k_assemble<double><<<nblk, 256, 0, s>>>(n, nrhs, P, (const double *)V, ldv,
                                                (const double *)hbuf, sf * sf, se * se, 2 * sf,
                                                2 * se, (double *)KV, (double *)dsf, (double *)dse);
    return hipGetLastError();
}

}  // namespace nfftgp
