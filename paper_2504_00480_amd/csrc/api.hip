// C ABI of libnfftgp: plan creation (window scaling and sorting), per-theta
// coefficients, the additive apply, CG, dot products and the Lanczos
// quadrature.  See include/nfftgp.h for the contract of every entry point.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "nfftgp_impl.h"

namespace nfftgp {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

}  // namespace nfftgp

using namespace nfftgp;

namespace {

nfftgp_status fail(nfftgp_status st, const std::string &m)
{
    set_error(m);
    return st;
}

size_t prec_bytes(int prec) { return prec == NFFTGP_F32 ? sizeof(float) : sizeof(double); }

nfftgp_status dalloc(nfftgp_plan p, void **ptr, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        return fail(NFFTGP_E_NOMEM, "hipMalloc(" + std::to_string(bytes) + " bytes) failed: " +
                                        hipGetErrorString(e));
    }
    p->allocs.push_back(*ptr);
    p->bytes += bytes;
    return NFFTGP_OK;
}

void free_plan(nfftgp_plan p)
{
    if (!p) return;
    (void)hipStreamSynchronize(p->stream);
    for (void *a : p->allocs) (void)hipFree(a);
    for (void *a : p->host_allocs) (void)hipHostFree(a);
    for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
    if (p->minb_host) (void)hipHostFree(p->minb_host);
    if (p->cg_exec) (void)hipGraphExecDestroy(p->cg_exec);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    delete p;
}

// Event pair around one launch when its category is being timed.
int prof_begin(nfftgp_plan p, int cat)
{
    if (!((p->prof >> cat) & 1u)) return -1;
    while (p->ev_used + 2 > p->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        p->ev_pool.push_back(e);
    }
    int i = (int)p->ev_used;
    p->ev_used += 2;
    (void)hipEventRecord(p->ev_pool[i], p->stream);
    return i;
}

void prof_end(nfftgp_plan p, int cat, int i)
{
    if (i < 0) return;
    (void)hipEventRecord(p->ev_pool[i + 1], p->stream);
    p->prof_cat.push_back(cat);
    p->prof_ev.push_back(i);
}

#define PROF_LAUNCH(plan_, cat_, expr_)                   \
    do {                                                   \
        int pi_ = prof_begin(plan_, cat_);                 \
        NFFTGP_HIP_TRY(expr_);                             \
        prof_end(plan_, cat_, pi_);                        \
    } while (0)

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

WindowGeom make_geom(int d, int N, int m)
{
    WindowGeom g;
    g.d = d;
    g.N = N;
    g.ng = 2 * N;
    int tb = d == 3 ? 8 : (d == 2 ? 16 : 64);
    g.tb = std::min(tb, g.ng);
    g.nb = g.ng / g.tb;
    g.nbins = 1;
    g.pd = g.tb + 2 * m;
    g.pc = 1;
    g.cells = 1;
    g.dcells = 1;
    for (int q = 0; q < d; ++q) {
        g.nbins *= g.nb;
        g.pc *= g.pd;
        g.cells *= g.ng;
        g.dcells *= (N + 1);
    }
    return g;
}

// Temporary device buffers of plan creation, freed on every exit path.
struct Scratch {
    std::vector<void *> p;
    ~Scratch()
    {
        for (void *x : p) (void)hipFree(x);
    }
    hipError_t get(void **ptr, size_t bytes)
    {
        if (bytes == 0) bytes = 256;
        hipError_t e = hipMalloc(ptr, bytes);
        if (e == hipSuccess) p.push_back(*ptr);
        return e;
    }
};

#define TRYS(expr)                                                 \
    do {                                                           \
        nfftgp_status st_ = (expr);                                \
        if (st_ != NFFTGP_OK) {                                    \
            free_plan(plan);                                       \
            return st_;                                            \
        }                                                          \
    } while (0)

#define TRYH(expr)                                                                  \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess) {                                                     \
            set_error(std::string(#expr) + ": " + hipGetErrorString(e_));           \
            free_plan(plan);                                                        \
            return NFFTGP_E_HIP;                                                    \
        }                                                                           \
    } while (0)

}  // namespace

namespace nfftgp {

// Coefficients recorded by set_hyper but not yet computed (they are computed
// by the next apply's fold launch) are computed now by their own launch.
hipError_t resolve_coef(nfftgp_plan p)
{
    for (Group &G : p->groups) {
        if (!G.coef_pending) continue;
        const int pi_ = prof_begin(p, NFFTGP_PROF_COEF);
        const hipError_t e = launch_coefficients(p->prec, G, G.prm, G.cinv2, p->coef, p->stream);
        if (e != hipSuccess) return e;
        prof_end(p, NFFTGP_PROF_COEF, pi_);
        G.coef_pending = false;
    }
    return hipSuccess;
}

// Enqueue one additive apply; no validation, no allocation, no host sync.
nfftgp_status apply_impl(nfftgp_plan p, const void *V, int64_t ldv, int nrhs, void *KV,
                         void *dell, void *dsf, void *dse)
{
    const hipStream_t s = p->stream;
    const bool with_der = dell != nullptr;
    if (p->n == 0) return NFFTGP_OK;
    for (Group &G : p->groups) {
        PROF_LAUNCH(p, NFFTGP_PROF_SPREAD, launch_spread(p->prec, G, p->m, V, ldv, nrhs, p->tilebuf, s));
        // the fold launch also computes coefficients recorded by set_hyper
        PROF_LAUNCH(p, NFFTGP_PROF_FOLD,
                    launch_fold(p->prec, G, p->m, nrhs, p->tilebuf, p->grid, G.coef_pending, s));
        G.coef_pending = false;
        if (G.g.d > 1)
            PROF_LAUNCH(p, NFFTGP_PROF_FFT_FWD, launch_fft_fwd(p->prec, G, p->m, p->grid, nrhs, s));
        PROF_LAUNCH(p, NFFTGP_PROF_DIAG, launch_fft_diag(p->prec, G, p->m, p->grid, nrhs, with_der, s));
        if (G.g.d > 1)
            PROF_LAUNCH(p, NFFTGP_PROF_FFT_INV, launch_fft_inv(p->prec, G, p->m, p->grid, nrhs, with_der, s));
        PROF_LAUNCH(p, NFFTGP_PROF_INTERP,
                    launch_interp(p->prec, G, p->m, p->n, nrhs, p->grid, with_der, p->hbuf, dell,
                                  p->sigma_f * p->sigma_f, s));
    }
    PROF_LAUNCH(p, NFFTGP_PROF_ASSEMBLE,
                launch_assemble(p->prec, p->n, nrhs, p->P, V, ldv, p->hbuf, p->sigma_f, p->sigma_eps,
                                KV, dsf, dse, s));
    return NFFTGP_OK;
}

int prof_begin_cat(nfftgp_plan p, int cat) { return prof_begin(p, cat); }
void prof_end_cat(nfftgp_plan p, int cat, int i) { prof_end(p, cat, i); }

}  // namespace nfftgp

namespace {

// Smallest spreading subproblem the tuner tries; list arrays are sized for it.
constexpr int kMinSubSp = 64;

// (Re)build a group's spreading work list for subproblems of sub_sp points:
// the list arrays, the per-window tile -> subproblem CSR and the list of
// split tiles; the tile workspace is grown when the new list needs more.
nfftgp_status build_spread_lists(nfftgp_plan plan, Group &G, int sub_sp)
{
    std::vector<int> sw, sb, ss, sc, fbl;
    for (int wl = 0; wl < G.nwin; ++wl) {
        Window &w = plan->win[G.wins[wl]];
        const std::vector<int> &bs = w.h_bin_start;
        std::vector<int> bsp(w.g.nbins + 1, 0);
        bsp[0] = (int)sb.size();
        for (int b = 0; b < w.g.nbins; ++b) {
            const int cnt = bs[b + 1] - bs[b];
            for (int off = 0; off < cnt; off += sub_sp) {
                sw.push_back(wl);
                sb.push_back(b);
                ss.push_back(bs[b] + off);
                sc.push_back(std::min(sub_sp, cnt - off));
            }
            bsp[b + 1] = (int)sb.size();
            if (bsp[b + 1] - bsp[b] >= 2) fbl.push_back(wl * w.g.nbins + b);
        }
        NFFTGP_HIP_TRY(hipMemcpy(w.bin_sub_ptr, bsp.data(), (w.g.nbins + 1) * sizeof(int), hipMemcpyHostToDevice));
    }
    if ((int)sb.size() > G.sub_cap) return fail(NFFTGP_E_ARG, "spreading list exceeds its capacity");
    int32_t *dst[5] = {G.sub_win, G.sub_bin, G.sub_start, G.sub_count, G.fb};
    std::vector<int> *srcv[5] = {&sw, &sb, &ss, &sc, &fbl};
    for (int k = 0; k < 5; ++k)
        if (!srcv[k]->empty())
            NFFTGP_HIP_TRY(hipMemcpy(dst[k], srcv[k]->data(), srcv[k]->size() * sizeof(int), hipMemcpyHostToDevice));
    G.nsub = (int)sb.size();
    G.nfb = (int)fbl.size();
    G.sub_sp = sub_sp;
    const size_t need = std::max<size_t>(1, (size_t)G.nsub * G.g.pc);
    if (need > plan->tile_cap) {
        const size_t eb = plan->prec == NFFTGP_F32 ? 4 : 8;
        if (plan->tilebuf) {
            NFFTGP_HIP_TRY(hipStreamSynchronize(plan->stream));
            NFFTGP_HIP_TRY(hipFree(plan->tilebuf));
            for (void *&a : plan->allocs)
                if (a == plan->tilebuf) a = nullptr;
            plan->tilebuf = nullptr;
            plan->bytes -= plan->tile_cap * plan->max_nrhs * eb;
        }
        nfftgp_status e = dalloc(plan, &plan->tilebuf, need * plan->max_nrhs * eb);
        if (e != NFFTGP_OK) return e;
        plan->tile_cap = need;
    }
    return NFFTGP_OK;
}

// (Re)build a group's tile-interpolation work list: subproblems of up to
// 256 * pt points of one tile (pt points per thread).
nfftgp_status build_interp_lists(nfftgp_plan plan, Group &G, int pt, int rows, bool slot = false,
                                 bool blk = false)
{
    // 3-D: a subproblem stages only `rows` first-axis rows of the padded tile
    // (points of first-tap rows f0..f1 read rows f0 .. f1 + 2m - 1, since the
    // points of a tile are sorted by cell, first axis slowest), so it is cut
    // where its rows would no longer fit; its first staged row a0 is packed
    // into bits 24-31 of the tile index
    const int isp = kInterpSubPoints * pt;
    const WindowGeom &g = G.g;
    const int m = plan->m;
    const bool cut = g.d == 3 && rows < g.pd;
    if (g.d != 3) rows = g.pd;
    // 3-D slots: the lists count slots (one or two points of one cell), one per thread;
    // 3-D and 2-D FP32 matrix-core blocks: the lists count blocks
    blk = blk && (g.d == 3 || g.d == 2) && plan->n > 0 && plan->prec == NFFTGP_F32 && (m == 4 || m == 6);
    slot = slot && !blk && g.d == 3 && plan->n > 0;
    const int isp_s = blk ? G.interp_sub_blocks : (slot ? kInterpSubPoints : isp);
    if (rows < 2 * m || rows > g.pd) return fail(NFFTGP_E_ARG, "bad interpolation row count");
    std::vector<int> iw, ib, is, ic;
    auto push = [&](int wl, int b, int start, int cnt, int f0) {
        const int a0 = cut ? std::min(f0, g.pd - rows) : 0;
        iw.push_back(wl);
        ib.push_back(b | (a0 << 24));
        is.push_back(start);
        ic.push_back(cnt);
    };
    for (int wl = 0; wl < G.nwin; ++wl) {
        const Window &w = plan->win[G.wins[wl]];
        const std::vector<int> &bs = blk ? w.h_block_start : (slot ? w.h_slot_start : w.h_bin_start);
        const std::vector<int> &rc = blk ? w.h_row_blocks : (slot ? w.h_row_slots : w.h_row_cnt);
        for (int b = 0; b < g.nbins; ++b) {
            const int cnt = bs[b + 1] - bs[b];
            if (cnt == 0) continue;
            if (!cut) {
                for (int off = 0; off < cnt; off += isp_s) push(wl, b, bs[b] + off, std::min(isp_s, cnt - off), 0);
                continue;
            }
            int start = bs[b], k = 0, f0 = 0;   // open subproblem: k points (slots) from row f0
            for (int r = 0; r < g.tb; ++r) {
                int left = rc[(size_t)b * g.tb + r];
                const int f = r + 1;             // first-tap row of the points of cell row r
                while (left > 0) {
                    if (k > 0 && (k == isp_s || f - f0 + 2 * m > rows)) {
                        push(wl, b, start, k, f0);
                        start += k;
                        k = 0;
                    }
                    if (k == 0) f0 = f;
                    const int take = std::min(left, isp_s - k);
                    k += take;
                    left -= take;
                }
            }
            if (k > 0) push(wl, b, start, k, f0);
            if (start + k != bs[b + 1]) return fail(NFFTGP_E_ARG, "row counts do not match the tile");
        }
    }
    if ((int)iw.size() > G.isub_cap) return fail(NFFTGP_E_ARG, "interpolation list exceeds its capacity");
    int32_t *dst[4] = {G.isub_win, G.isub_bin, G.isub_start, G.isub_count};
    std::vector<int> *srcv[4] = {&iw, &ib, &is, &ic};
    for (int k = 0; k < 4; ++k)
        if (!srcv[k]->empty())
            NFFTGP_HIP_TRY(hipMemcpy(dst[k], srcv[k]->data(), srcv[k]->size() * sizeof(int), hipMemcpyHostToDevice));
    G.nisub = (int)iw.size();
    G.interp_pt = slot ? 2 : pt;
    G.interp_rows = rows;
    G.interp_slot = slot;
    G.interp_mfma = blk;
    if (slot || blk) G.interp_adj = false;
    return NFFTGP_OK;
}

// Staged rows of the 3-D tile interpolation by rule: a window of half a tile
// of first-tap rows plus the taps (tb/2 + 2m - 1; 11 of 16 rows at m = 4),
// which lets more work-groups share a CU's LDS.
int interp_rows_rule(const WindowGeom &g, int m)
{
    if (g.d != 3) return g.pd;
    return std::min(g.pd, g.tb / 2 + 2 * m - 1);
}

// Staged rows of the 3-D matrix-core interpolation by rule: one first-axis cell
// row per subproblem (2m rows), so that the staged tile (77 KB at m = 6) lets
// two work-groups of eight waves share a CU (measured at C5: 10.4 ms per launch
// against 11.4 with sixteen waves and 15 rows, one work-group per CU).
int interp_mfma_rows_rule(const WindowGeom &g, int m)
{
    return std::min(g.pd, 2 * m);
}

// Plan creation; given_c0 / given_c (both host, or both NULL) carry a scaling
// chosen by the caller (nfftgp_plan_create_scaled), otherwise scale_mode rules.
nfftgp_status plan_create_impl(nfftgp_plan *out, const void *X_dev, int64_t n, int32_t p,
                               int64_t ldx, int32_t P, const int32_t *win_ptr,
                               const int32_t *win_idx, const int32_t *kernel, const int32_t *N,
                               int32_t m, int32_t prec, int32_t scale_mode,
                               const double *given_c0, const double *given_c,
                               int32_t max_nrhs, void *stream)
{
    if (!out) return fail(NFFTGP_E_ARG, "out is NULL");
    *out = nullptr;
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(NFFTGP_E_ARG, "n out of range");
    if (n > 0 && !X_dev) return fail(NFFTGP_E_ARG, "X_dev is NULL");
    if (p < 1 || ldx < p) return fail(NFFTGP_E_ARG, "need p >= 1 and ldx >= p");
    if (P < 1 || P > NFFTGP_MAX_WINDOWS) return fail(NFFTGP_E_ARG, "P out of range");
    if (!win_ptr || !win_idx || !kernel || !N) return fail(NFFTGP_E_ARG, "window arrays are NULL");
    if (prec != NFFTGP_F32 && prec != NFFTGP_F64) return fail(NFFTGP_E_ARG, "bad precision");
    if (scale_mode != NFFTGP_SCALE_AUTO && scale_mode != NFFTGP_SCALE_NONE)
        return fail(NFFTGP_E_ARG, "bad scale_mode");
    if (max_nrhs < 1 || max_nrhs > 64) return fail(NFFTGP_E_ARG, "max_nrhs must be in 1..64");
    if (!(m == 2 || m == 4 || m == 6 || m == 8))
        return fail(NFFTGP_E_DIM, "cutoff m must be 2, 4, 6 or 8");
    if (win_ptr[0] != 0) return fail(NFFTGP_E_ARG, "win_ptr[0] must be 0");
    std::vector<char> seen(p, 0);
    for (int s = 0; s < P; ++s) {
        int d = win_ptr[s + 1] - win_ptr[s];
        if (d < 1 || d > 3) return fail(NFFTGP_E_DIM, "window dimension must be 1..3");
        for (int q = win_ptr[s]; q < win_ptr[s + 1]; ++q) {
            int f = win_idx[q];
            if (f < 0 || f >= p) return fail(NFFTGP_E_ARG, "feature index out of range");
            if (seen[f]) return fail(NFFTGP_E_ARG, "windows overlap");
            seen[f] = 1;
        }
        if (kernel[s] < NFFTGP_GAUSS || kernel[s] > NFFTGP_SINC)
            return fail(NFFTGP_E_ARG, "unknown kernel type");
        int Nmax = d == 3 ? 64 : 128;
        if (!is_pow2(N[s]) || N[s] < 8 || N[s] > Nmax)
            return fail(NFFTGP_E_DIM, "bandwidth must be a power of two in 8..64 (d=3) or 8..128");
        if (2 * m >= N[s]) return fail(NFFTGP_E_DIM, "cutoff must satisfy m < N/2");
        if (given_c && !(given_c[s] > 0.0 && std::isfinite(given_c[s])))
            return fail(NFFTGP_E_ARG, "scale factors must be finite and > 0");
    }
    if (given_c) {
        for (int q = 0; q < win_ptr[P]; ++q)
            if (!std::isfinite(given_c0[q])) return fail(NFFTGP_E_ARG, "scale centres must be finite");
    }

    nfftgp_plan plan = new nfftgp_plan_s();
    plan->n = n;
    plan->p = p;
    plan->P = P;
    plan->m = m;
    plan->prec = prec;
    plan->max_nrhs = max_nrhs;
    plan->scale_mode = scale_mode;
    plan->stream = (hipStream_t)stream;
    TRYH(hipGetDevice(&plan->device));
    const hipStream_t st = plan->stream;
    const size_t eb = prec_bytes(prec);
    int max_lds = 0;
    TRYH(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, plan->device));
    for (int s = 0; s < P; ++s) {
        WindowGeom g = make_geom(win_ptr[s + 1] - win_ptr[s], N[s], m);
        if ((size_t)2 * g.pc * eb > (size_t)max_lds) {
            free_plan(plan);
            return fail(NFFTGP_E_DIM, "window tile needs " + std::to_string(2 * g.pc * eb) +
                                          " bytes of LDS, device allows " + std::to_string(max_lds));
        }
    }

    Scratch tmp;
    double *part = nullptr, *mm = nullptr;
    int *flags = nullptr, *keys = nullptr, *hist = nullptr, *scan_tmp = nullptr, *bin_start = nullptr;
    int *ids1 = nullptr;
    void *t_uns = nullptr, *t1 = nullptr, *t2 = nullptr;
    int nblk = (int)std::max<int64_t>(1, (n + kSortBlock - 1) / kSortBlock);
    int max_keys = 1;
    for (int s = 0; s < P; ++s) {
        WindowGeom g = make_geom(win_ptr[s + 1] - win_ptr[s], N[s], m);
        int local = 1;
        for (int q = 0; q < g.d; ++q) local *= g.tb;
        max_keys = std::max(max_keys, std::max(g.nbins, local));
    }
    int64_t hist_len = (int64_t)max_keys * nblk;
    int64_t rowc_len = 1;   // 3-D windows: points per (tile, first-axis row)
    for (int s = 0; s < P; ++s) {
        WindowGeom g = make_geom(win_ptr[s + 1] - win_ptr[s], N[s], m);
        if (g.d == 3) rowc_len = std::max<int64_t>(rowc_len, (int64_t)g.nbins * g.tb);
    }
    int *rowc = nullptr;
    const int64_t n1 = std::max<int64_t>(n, 1);
    TRYH(tmp.get((void **)&part, kPartBlocks * 6 * sizeof(double)));
    TRYH(tmp.get((void **)&mm, 8 * sizeof(double)));
    TRYH(tmp.get((void **)&flags, 4 * sizeof(int)));
    TRYH(tmp.get((void **)&keys, n1 * sizeof(int)));
    TRYH(tmp.get((void **)&ids1, n1 * sizeof(int)));
    TRYH(tmp.get((void **)&hist, (hist_len + 1) * sizeof(int)));
    TRYH(tmp.get((void **)&scan_tmp, scan_scratch_ints(hist_len) * sizeof(int)));
    TRYH(tmp.get((void **)&bin_start, (max_keys + 1) * sizeof(int)));
    TRYH(tmp.get((void **)&rowc, rowc_len * sizeof(int)));
    TRYH(tmp.get(&t_uns, n1 * 3 * eb));
    TRYH(tmp.get(&t1, n1 * 3 * eb));
    TRYH(tmp.get(&t2, n1 * 3 * eb));
    // points per spreading work-group: short runs for small n (enough groups to
    // fill the device), longer runs for large n (fewer partial tiles to fold);
    // measured on 1e5..2e6 points: 256 at 1e5 (four-point form), 1024 at 2e5,
    // 2048 at 5e5, 4096 at 2e6
    int sub_sp = n <= 65536 ? 128 : 256;
    if (n > 131072) {
        sub_sp = 256;
        while (sub_sp < 4096 && (int64_t)sub_sp * 256 < n) sub_sp *= 2;
    }

    int64_t max_cells = 1, maxK = 1;
    plan->win.resize(P);
    for (int s = 0; s < P; ++s) {
        Window &w = plan->win[s];
        const int d = win_ptr[s + 1] - win_ptr[s];
        w.g = make_geom(d, N[s], m);
        w.kernel = kernel[s];
        for (int q = 0; q < d; ++q) w.feat[q] = win_idx[win_ptr[s] + q];
        // --- scaling into [-1/4, 1/4)^d
        double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        int hflags[3] = {0, 0, 0};
        TRYH(hipMemsetAsync(flags, 0, 4 * sizeof(int), st));
        if (n > 0) {
            TRYH(launch_minmax(prec, X_dev, n, ldx, d, w.feat, part, mm, flags, st));
            double hm[6];
            TRYH(hipMemcpyAsync(hm, mm, 2 * d * sizeof(double), hipMemcpyDeviceToHost, st));
            TRYH(hipMemcpyAsync(hflags, flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
            TRYH(hipStreamSynchronize(st));
            if (hflags[0]) {
                free_plan(plan);
                return fail(NFFTGP_E_ARG, "X holds NaN or Inf in window " + std::to_string(s));
            }
            for (int q = 0; q < d; ++q) {
                lo[q] = hm[q];
                hi[q] = hm[d + q];
            }
        }
        w.c = 1.0;
        if (given_c) {
            w.c = given_c[s];
            for (int q = 0; q < d; ++q) w.c0[q] = given_c0[win_ptr[s] + q];
        } else if (scale_mode == NFFTGP_SCALE_AUTO && n > 0) {
            bool inside = true;
            for (int q = 0; q < d; ++q) inside = inside && lo[q] >= -0.25 && hi[q] < 0.25;
            if (!inside) {
                double h = 0.0;
                for (int q = 0; q < d; ++q) {
                    w.c0[q] = (lo[q] + hi[q]) * 0.5;
                    h = std::max(h, std::max(hi[q] - w.c0[q], w.c0[q] - lo[q]));
                }
                if (h > 0.0) w.c = 0.25 * (1.0 - std::ldexp(1.0, -20)) / h;
            }
        }
        // --- grid coordinates; two stable counting-sort passes (cell inside the
        // tile, then tile) leave the points grouped by tile and, inside a tile,
        // by cell
        int local = 1;
        for (int q = 0; q < d; ++q) local *= w.g.tb;
        TRYS(dalloc(plan, (void **)&w.perm, n1 * sizeof(int)));
        TRYS(dalloc(plan, &w.rec, n1 * d * 2 * m * eb));
        TRYS(dalloc(plan, (void **)&w.anchor, n1 * sizeof(int)));
        TRYS(dalloc(plan, (void **)&w.lpos, n1 * sizeof(int)));
        TRYH(launch_coords(prec, X_dev, n, ldx, d, w.feat, w.c0, w.c, w.g, t_uns, keys, flags + 1, st));
        TRYH(launch_sort(prec, n, d, local, keys, nullptr, t_uns, hist, scan_tmp, ids1, t1, bin_start, st));
        TRYH(launch_bin_keys(prec, t1, n, w.g, keys, st));
        TRYH(launch_sort(prec, n, d, w.g.nbins, keys, ids1, t1, hist, scan_tmp, w.perm, t2,
                         bin_start, st));
        TRYH(launch_weights(prec, t2, n, w.g, m, kb_knorm(m), w.rec, w.anchor, w.lpos, st));
        std::vector<int> bs(w.g.nbins + 1);
        TRYH(hipMemcpyAsync(bs.data(), bin_start, (w.g.nbins + 1) * sizeof(int), hipMemcpyDeviceToHost, st));
        if (d == 3 && n > 0) {
            w.h_row_cnt.assign((size_t)w.g.nbins * w.g.tb, 0);
            TRYH(hipMemsetAsync(rowc, 0, w.h_row_cnt.size() * sizeof(int), st));
            TRYH(launch_row_counts(w.anchor, n, w.g, rowc, st));
            TRYH(hipMemcpyAsync(w.h_row_cnt.data(), rowc, w.h_row_cnt.size() * sizeof(int),
                                hipMemcpyDeviceToHost, st));
        }
        std::vector<int> hanchor;
        if ((d == 3 || d == 2) && n > 0) {
            hanchor.resize(n);
            TRYH(hipMemcpyAsync(hanchor.data(), w.anchor, n * sizeof(int), hipMemcpyDeviceToHost, st));
        }
        TRYH(hipMemcpyAsync(hflags, flags, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
        TRYH(hipStreamSynchronize(st));
        if (hflags[1]) {
            free_plan(plan);
            return fail(NFFTGP_E_BOX, "window " + std::to_string(s) +
                                          ": a scaled point lies outside [-1/4, 1/4)^d");
        }
        w.h_bin_start = bs;
        if ((d == 3 || d == 2) && n > 0) {
            const int ng = w.g.ng, tb = w.g.tb;
            if (d == 3) {
            // interpolation slots: consecutive points of a run of equal cells
            // are paired (a run never crosses a tile); slots per tile and per
            // (tile, first-axis cell row) for the work lists
            std::vector<int> sl;
            sl.reserve(n);
            w.h_slot_start.assign(w.g.nbins + 1, 0);
            w.h_row_slots.assign((size_t)w.g.nbins * w.g.tb, 0);
            for (int b = 0; b < w.g.nbins; ++b) {
                w.h_slot_start[b] = (int)sl.size();
                for (int j = bs[b]; j < bs[b + 1];) {
                    const bool last = hanchor[j] < 0;
                    const bool pair = !last && j + 1 < bs[b + 1];
                    sl.push_back(pair ? (int)((unsigned)j | 0x80000000u) : j);
                    const int a = hanchor[j] & 0x7fffffff;
                    w.h_row_slots[(size_t)b * tb + (a / (ng * ng)) % tb] += 1;
                    j += pair ? 2 : 1;
                }
            }
            w.h_slot_start[w.g.nbins] = (int)sl.size();
            TRYS(dalloc(plan, (void **)&w.slots, sl.size() * sizeof(int)));
            TRYH(hipMemcpy(w.slots, sl.data(), sl.size() * sizeof(int), hipMemcpyHostToDevice));
            }
            // matrix-core interpolation blocks (3-D and 2-D windows): each run
            // of equal cells cut into pieces of at most 16 points; block
            // starts, then n (the per-row counts serve the 3-D lists)
            std::vector<int> bl;
            bl.reserve(n / 8 + 1);
            w.h_block_start.assign(w.g.nbins + 1, 0);
            w.h_row_blocks.assign((size_t)w.g.nbins * w.g.tb, 0);
            for (int b = 0; b < w.g.nbins; ++b) {
                w.h_block_start[b] = (int)bl.size();
                for (int j = bs[b]; j < bs[b + 1];) {
                    int e = j;
                    while (e < bs[b + 1] - 1 && hanchor[e] >= 0) ++e;   // e: last point of the run
                    const int a = hanchor[j] & 0x7fffffff;
                    for (int k = j; k <= e; k += 16) {
                        bl.push_back(k);
                        if (d == 3) w.h_row_blocks[(size_t)b * tb + (a / (ng * ng)) % tb] += 1;
                    }
                    j = e + 1;
                }
            }
            w.h_block_start[w.g.nbins] = (int)bl.size();
            bl.push_back((int)n);
            TRYS(dalloc(plan, (void **)&w.blocks, bl.size() * sizeof(int)));
            TRYH(hipMemcpy(w.blocks, bl.data(), bl.size() * sizeof(int), hipMemcpyHostToDevice));
        }
        TRYS(dalloc(plan, &w.Dk, w.g.dcells * eb));
        TRYS(dalloc(plan, &w.Dder, w.g.dcells * eb));
        int64_t K = 1;
        for (int q = 0; q < d; ++q) K *= N[s];
        maxK = std::max(maxK, K);
    }
    // --- window groups (equal dimension and bandwidth) and their work lists:
    // spreading subproblems are runs of at most sub_sp points of one tile,
    // interpolation subproblems runs of at most kInterpSubPoints
    for (int s = 0; s < P; ++s) {
        int gi = -1;
        for (int k = 0; k < (int)plan->groups.size(); ++k)
            if (plan->groups[k].g.d == plan->win[s].g.d && plan->groups[k].g.N == plan->win[s].g.N) gi = k;
        if (gi < 0) {
            plan->groups.emplace_back();
            gi = (int)plan->groups.size() - 1;
            plan->groups[gi].g = plan->win[s].g;
        }
        plan->groups[gi].wins.push_back(s);
    }
    size_t grid_need = 1, coef_need = 8;
    for (Group &G : plan->groups) {
        G.nwin = (int)G.wins.size();
        G.sep = true;
        for (int s : G.wins) G.sep = G.sep && plan->win[s].kernel == NFFTGP_GAUSS;
        std::vector<WinDesc> hd(G.nwin);
        int64_t cap = 0, icap = 0;
        const bool d3 = G.g.d == 3;
        for (int wl = 0; wl < G.nwin; ++wl) {
            Window &w = plan->win[G.wins[wl]];
            const std::vector<int> &bs = w.h_bin_start;
            for (int b = 0; b < w.g.nbins; ++b) {
                const int cnt = bs[b + 1] - bs[b];
                G.nbins_used += cnt > 0;
                cap += (cnt + kMinSubSp - 1) / kMinSubSp;
                icap += (cnt + kInterpSubPoints - 1) / kInterpSubPoints + (d3 && cnt > 0 ? G.g.tb : 0);
                if (!w.h_block_start.empty()) {
                    // the block lists (at most kInterpSubBlocks blocks per subproblem) may be longer
                    const int nbl = w.h_block_start[b + 1] - w.h_block_start[b];
                    icap += (nbl + kInterpSubBlocksLds - 1) / kInterpSubBlocksLds;
                }
            }
            TRYS(dalloc(plan, (void **)&w.bin_sub_ptr, (w.g.nbins + 1) * sizeof(int)));
            hd[wl] = WinDesc{w.rec,  w.anchor, w.lpos,   w.perm,        w.bin_sub_ptr, w.Dk,
                             w.Dder, w.slots,  w.blocks, G.wins[wl], 0};
        }
        G.sub_cap = (int)std::max<int64_t>(cap, 1);
        {
            int32_t **sd[4] = {&G.sub_win, &G.sub_bin, &G.sub_start, &G.sub_count};
            for (int k = 0; k < 4; ++k) TRYS(dalloc(plan, (void **)sd[k], (size_t)G.sub_cap * sizeof(int)));
            TRYS(dalloc(plan, (void **)&G.fb, std::max<size_t>(1, (size_t)G.nwin * G.g.nbins) * sizeof(int)));
        }
        TRYS(build_spread_lists(plan, G, sub_sp));
        G.isub_cap = (int)std::max<int64_t>(icap, 1);
        {
            int32_t **id[4] = {&G.isub_win, &G.isub_bin, &G.isub_start, &G.isub_count};
            for (int k = 0; k < 4; ++k) TRYS(dalloc(plan, (void **)id[k], (size_t)G.isub_cap * sizeof(int)));
        }
        if (!d3) {
            // several-vector interpolation list (d <= 2): subproblems of up to
            // vsub_sp points (rule: from 512 doubled up to kInterpVbSubPoints
            // while the group keeps at least 256 of them; NFFTGP_INTERP_VB_SUB=
            // <points> overrides, a multiple of 512)
            const char *vsv = std::getenv("NFFTGP_INTERP_VB_SUB");
            int vsp = 512;
            if (vsv) {
                vsp = std::atoi(vsv);
            } else {
                const int64_t pts = (int64_t)G.nwin * n;
                while (vsp < kInterpVbSubPoints && pts / (2 * vsp) >= 256) vsp *= 2;
            }
            vsp = std::max(512, std::min(1 << 16, vsp - vsp % 512));
            G.vsub_sp = vsp;
            int64_t vcap = 0;
            for (int wl = 0; wl < G.nwin; ++wl) {
                const std::vector<int> &bs = plan->win[G.wins[wl]].h_bin_start;
                for (int b = 0; b < G.g.nbins; ++b) vcap += (bs[b + 1] - bs[b] + vsp - 1) / vsp;
            }
            G.vsub_cap = (int)std::max<int64_t>(vcap, 1);
            int32_t **vd[4] = {&G.vsub_win, &G.vsub_bin, &G.vsub_start, &G.vsub_count};
            for (int k = 0; k < 4; ++k) TRYS(dalloc(plan, (void **)vd[k], (size_t)G.vsub_cap * sizeof(int)));
            std::vector<int> vw, vbn, vs, vc;
            for (int wl = 0; wl < G.nwin; ++wl) {
                const std::vector<int> &bs = plan->win[G.wins[wl]].h_bin_start;
                for (int b = 0; b < G.g.nbins; ++b)
                    for (int off = 0; off < bs[b + 1] - bs[b]; off += vsp) {
                        vw.push_back(wl);
                        vbn.push_back(b);
                        vs.push_back(bs[b] + off);
                        vc.push_back(std::min(vsp, bs[b + 1] - bs[b] - off));
                    }
            }
            std::vector<int> *vsrc[4] = {&vw, &vbn, &vs, &vc};
            for (int k = 0; k < 4; ++k)
                if (!vsrc[k]->empty())
                    TRYH(hipMemcpy(*vd[k], vsrc[k]->data(), vsrc[k]->size() * sizeof(int), hipMemcpyHostToDevice));
            G.nvsub = (int)vw.size();
        }
        // interpolation variant: the per-point tile variant by default (the
        // faster one on every measured workload once its tile staging was
        // batched); nfftgp_autotune may switch, NFFTGP_INTERP=run|tile|tile2|tilepair|tilefull|tileslot|mfma
        // forces (tile2: two points per thread; tilepair: two adjacent sorted points
        // per thread sharing tap reads, 3-D; tilefull: whole padded tiles staged)
        const char *swv = std::getenv("NFFTGP_SPREAD_W");   // "2": two waves per 3-D tile
        G.spread_W = swv && std::strcmp(swv, "2") == 0 ? 2 : 0;
        const char *srv = std::getenv("NFFTGP_SPREAD_R");   // vectors per work-group: 1, 2, 4
        if (srv) {
            const int rv = std::atoi(srv);
            G.spread_R = (rv == 1 || rv == 2 || rv == 4) ? rv : 0;
        }
        const char *sfv = std::getenv("NFFTGP_SPREAD_FORM");   // "quad" | "run" | "mfma"
        G.spread_form = !sfv ? 0
                             : (std::strcmp(sfv, "quad") == 0 ? 1
                                                               : (std::strcmp(sfv, "run") == 0 ? 2
                                                                                                : (std::strcmp(sfv, "mfma") == 0 ? 3 : 0)));
        const char *iov = std::getenv("NFFTGP_INTERP");
        // d <= 2: LDS bytes of the several-vector staging, NFFTGP_INTERP_VB=<bytes>
        // overrides ("0": one vector per staging)
        const char *ivb = std::getenv("NFFTGP_INTERP_VB");
        G.interp_vb_lds = ivb ? std::max(0, std::atoi(ivb)) : (80 << 10);
        G.use_run_interp = iov && std::strcmp(iov, "run") == 0 && n > 0;
        const bool full = iov && std::strcmp(iov, "tilefull") == 0;
        const bool pair = iov && std::strcmp(iov, "tilepair") == 0;
        const bool slot = iov && std::strcmp(iov, "tileslot") == 0;
        // 3-D and 2-D FP32 with m = 4 or 6 and several vectors: matrix-core
        // blocks unless another variant is forced (2-D: measured C3 4.28 ->
        // 4.21 ms, C4 1.45 -> 1.43 ms, C5 36.13 -> 36.05 ms per step; the tuner
        // also times the tile forms)
        const bool blk = iov ? std::strcmp(iov, "mfma") == 0
                             : ((G.g.d == 3 || G.g.d == 2) && prec == NFFTGP_F32 && (m == 4 || m == 6) &&
                                max_nrhs >= 2);
        const char *smr = std::getenv("NFFTGP_SPREAD_MFMA_R");   // "2" | "4"
        G.spread_mfma_R = smr && std::strcmp(smr, "2") == 0 ? 2 : 4;
        const char *ffm = std::getenv("NFFTGP_FOLD");   // "cells" | "tiles"
        G.fold_form = ffm ? (std::strcmp(ffm, "tiles") == 0 ? 2 : (std::strcmp(ffm, "cells") == 0 ? 1 : 0)) : 0;
        const char *imw = std::getenv("NFFTGP_INTERP_MFMA_WAVES");   // "8" | "16"
        G.interp_mfma_waves = imw && std::strcmp(imw, "16") == 0 ? 16 : 8;
        // blocks per subproblem (NFFTGP_INTERP_SUB_BLOCKS, default the
        // kernel form's maximum): more blocks share one staging of the tile
        // rows per vector pass; measured at C5 (n = 2e6, m = 6, 16 vectors),
        // 3-D interpolation per launch: 16 blocks 10.20 ms, 32 blocks 9.71 ms
        {
            const char *isb = std::getenv("NFFTGP_INTERP_SUB_BLOCKS");
            const int cap = G.interp_mfma_waves == 16 ? kInterpSubBlocksLds : kInterpSubBlocks;
            G.interp_sub_blocks = isb ? std::max(1, std::min(cap, std::atoi(isb))) : cap;
        }
        G.interp_adj = pair && G.g.d == 3;
        // matrix-core blocks stage NFFTGP_INTERP_MFMA_ROWS first-axis rows
        // (default: the rule's window)
        const char *imr = std::getenv("NFFTGP_INTERP_MFMA_ROWS");
        const int mrows = imr ? std::max(2 * m, std::min(G.g.pd, std::atoi(imr))) : interp_mfma_rows_rule(G.g, m);
        TRYS(build_interp_lists(plan, G, iov && (pair || std::strcmp(iov, "tile2") == 0) ? 2 : 1,
                                full ? G.g.pd : (blk ? mrows : interp_rows_rule(G.g, m)), slot, blk));
        {
            // run-interpolation list (built for every group, so that the
            // variant can be switched): points per wave up to kRunSubPoints,
            // fewer while that leaves under 8192 waves for the group
            int rsp = kRunSubPoints;
            while (rsp > 64 && (int64_t)G.nwin * n < (int64_t)rsp * 8192) rsp /= 2;
            std::vector<int> rw, rs, rc;
            for (int wl = 0; wl < G.nwin; ++wl)
                for (int64_t off = 0; off < n; off += rsp) {
                    rw.push_back(wl);
                    rs.push_back((int)off);
                    rc.push_back((int)std::min<int64_t>(rsp, n - off));
                }
            G.nrsub = (int)rw.size();
            int32_t **rdst[3] = {&G.rsub_win, &G.rsub_start, &G.rsub_count};
            std::vector<int> *rsrc[3] = {&rw, &rs, &rc};
            for (int k = 0; k < 3; ++k) {
                TRYS(dalloc(plan, (void **)rdst[k], std::max<size_t>(1, rsrc[k]->size()) * sizeof(int)));
                if (!rsrc[k]->empty())
                    TRYH(hipMemcpy(*rdst[k], rsrc[k]->data(), rsrc[k]->size() * sizeof(int), hipMemcpyHostToDevice));
            }
        }
        TRYS(dalloc(plan, (void **)&G.cinv2, (G.g.N + 1) * sizeof(double)));
        TRYS(dalloc(plan, (void **)&G.cw, (size_t)(G.g.N / 2 + 1) * (G.g.N / 2 + 1) * sizeof(double)));
        TRYH(launch_window_coef(G.g.N, m, G.cinv2, G.cw, st));
        coef_need = std::max(coef_need, (size_t)coef_scratch_doubles(G.g, G.nwin));
        TRYS(dalloc(plan, (void **)&G.coef_part, (size_t)coef_part_doubles(G.g, G.nwin) * sizeof(double)));
        TRYS(dalloc(plan, (void **)&G.desc, G.nwin * sizeof(WinDesc)));
        TRYH(hipMemcpy(G.desc, hd.data(), G.nwin * sizeof(WinDesc), hipMemcpyHostToDevice));
        grid_need = std::max(grid_need, (size_t)G.nwin * G.g.cells);
    }
    TRYS(dalloc(plan, &plan->grid, grid_need * max_nrhs * 2 * eb));
    const size_t vec_bytes = std::max<int64_t>(n, 1) * max_nrhs * eb;
    TRYS(dalloc(plan, &plan->hbuf, vec_bytes * P));
    TRYS(dalloc(plan, (void **)&plan->coef, coef_need * sizeof(double)));
    {
        void *h = nullptr;
        TRYH(hipHostMalloc(&h, 2 * P * sizeof(double), hipHostMallocDefault));
        plan->minb_host = (double *)h;
    }
    TRYS(dalloc(plan, (void **)&plan->dot_part, (size_t)2 * kDotBlocks * 64 * sizeof(double) + 64 * sizeof(double)));
    TRYS(dalloc(plan, (void **)&plan->cg_scal, (size_t)kCgSlots * 64 * sizeof(double)));
    TRYS(dalloc(plan, (void **)&plan->cg_hist, (size_t)NFFTGP_MAX_CG_HISTORY * max_nrhs * 2 * sizeof(double)));
    TRYS(dalloc(plan, &plan->cg_r, vec_bytes));
    TRYS(dalloc(plan, &plan->cg_p, vec_bytes));
    TRYS(dalloc(plan, &plan->cg_ap, vec_bytes));
    TRYH(hipStreamSynchronize(st));
    *out = plan;
    return NFFTGP_OK;
}

}  // namespace

extern "C" {

const char *nfftgp_last_error(void) { return g_err.c_str(); }

nfftgp_status nfftgp_plan_create(nfftgp_plan *out, const void *X_dev, int64_t n, int32_t p,
                                 int64_t ldx, int32_t P, const int32_t *win_ptr,
                                 const int32_t *win_idx, const int32_t *kernel, const int32_t *N,
                                 int32_t m, int32_t prec, int32_t scale_mode,
                                 int32_t max_nrhs, void *stream)
{
    set_error("");
    if (scale_mode != NFFTGP_SCALE_AUTO && scale_mode != NFFTGP_SCALE_NONE)
        return fail(NFFTGP_E_ARG, "bad scale_mode");
    return plan_create_impl(out, X_dev, n, p, ldx, P, win_ptr, win_idx, kernel, N, m, prec, scale_mode,
                            nullptr, nullptr, max_nrhs, stream);
}

nfftgp_status nfftgp_plan_create_scaled(nfftgp_plan *out, const void *X_dev, int64_t n, int32_t p,
                                        int64_t ldx, int32_t P, const int32_t *win_ptr,
                                        const int32_t *win_idx, const int32_t *kernel,
                                        const int32_t *N, int32_t m, int32_t prec,
                                        const double *c0, const double *c, int32_t max_nrhs,
                                        void *stream)
{
    set_error("");
    if (!c0 || !c) return fail(NFFTGP_E_ARG, "c0 or c is NULL");
    return plan_create_impl(out, X_dev, n, p, ldx, P, win_ptr, win_idx, kernel, N, m, prec,
                            NFFTGP_SCALE_NONE, c0, c, max_nrhs, stream);
}

nfftgp_status nfftgp_set_hyper(nfftgp_plan plan, double sigma_f, const double *ell,
                               double sigma_eps)
{
    set_error("");
    if (!plan) return fail(NFFTGP_E_ARG, "plan is NULL");
    if (!ell) return fail(NFFTGP_E_ARG, "ell is NULL");
    if (!(sigma_f >= 0.0) || !std::isfinite(sigma_f) || !(sigma_eps >= 0.0) || !std::isfinite(sigma_eps))
        return fail(NFFTGP_E_ARG, "sigma_f and sigma_eps must be finite and >= 0");
    for (int s = 0; s < plan->P; ++s)
        if (!(ell[s] > 0.0) || !std::isfinite(ell[s])) return fail(NFFTGP_E_ARG, "ell must be finite and > 0");
    const hipStream_t st = plan->stream;
    for (Group &G : plan->groups) {
        CoefParams prm;
        std::memset(&prm, 0, sizeof(prm));
        prm.nwin = G.nwin;
        for (int wl = 0; wl < G.nwin; ++wl) {
            const int s = G.wins[wl];
            prm.ell[wl] = ell[s];
            prm.c[wl] = plan->win[s].c;
            prm.kernel[wl] = plan->win[s].kernel;
        }
        G.prm = prm;
        if (G.sep) {
            G.coef_pending = true;   // computed by the next apply's fold launch
        } else {
            G.coef_pending = false;
            PROF_LAUNCH(plan, NFFTGP_PROF_COEF,
                        launch_coefficients(plan->prec, G, prm, G.cinv2, plan->coef, st));
        }
    }
    // min_k b_k is reduced from the block minima only when asked for
    // (nfftgp_get_window_info), so set_hyper neither waits nor launches it
    plan->minb_pending = true;
    for (int s = 0; s < plan->P; ++s) plan->win[s].ell = ell[s];
    plan->sigma_f = sigma_f;
    plan->sigma_eps = sigma_eps;
    plan->have_hyper = true;
    // the preconditioner's factors follow theta
    if (plan->pc.on) return precond_refresh(plan);
    return NFFTGP_OK;
}

nfftgp_status nfftgp_apply(nfftgp_plan plan, const void *V_dev, int64_t ldv, int32_t nrhs,
                           void *KV_dev, void *dKV_dell_dev, void *dKV_dsf_dev, void *dKV_dse_dev)
{
    set_error("");
    if (!plan) return fail(NFFTGP_E_ARG, "plan is NULL");
    if (!plan->have_hyper) return fail(NFFTGP_E_STATE, "nfftgp_set_hyper has not been called");
    if (nrhs < 1 || nrhs > plan->max_nrhs) return fail(NFFTGP_E_ARG, "nrhs out of range 1..max_nrhs");
    if (ldv < nrhs) return fail(NFFTGP_E_ARG, "ldv < nrhs");
    if (plan->n > 0 && (!V_dev || !KV_dev)) return fail(NFFTGP_E_ARG, "V or KV is NULL");
    return apply_impl(plan, V_dev, ldv, nrhs, KV_dev, dKV_dell_dev, dKV_dsf_dev, dKV_dse_dev);
}

nfftgp_status nfftgp_autotune(nfftgp_plan plan, int32_t nrhs, int32_t with_derivs, int32_t reps,
                              char *report, int64_t report_len)
{
    set_error("");
    if (!plan) return fail(NFFTGP_E_ARG, "plan is NULL");
    if (!plan->have_hyper) return fail(NFFTGP_E_STATE, "nfftgp_set_hyper has not been called");
    if (nrhs < 1 || nrhs > plan->max_nrhs) return fail(NFFTGP_E_ARG, "nrhs out of range 1..max_nrhs");
    if (reps < 1) return fail(NFFTGP_E_ARG, "reps must be >= 1");
    if (report && report_len > 0) report[0] = '\0';
    const int64_t n = plan->n;
    if (n == 0) return NFFTGP_OK;
    const hipStream_t st = plan->stream;
    const size_t eb = plan->prec == NFFTGP_F32 ? 4 : 8;
    const size_t vb = (size_t)n * nrhs * eb;
    // inputs and outputs of the timed applies (tuning-time allocations)
    void *V = nullptr, *KV = nullptr, *dl = nullptr, *dsf = nullptr, *dse = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto release = [&]() {
        (void)hipStreamSynchronize(st);
        for (void *q : {V, KV, dl, dsf, dse})
            if (q) (void)hipFree(q);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    hipError_t he = hipMalloc(&V, vb);
    if (he == hipSuccess) he = hipMalloc(&KV, vb);
    if (he == hipSuccess && with_derivs) he = hipMalloc(&dl, vb * plan->P);
    if (he == hipSuccess && with_derivs) he = hipMalloc(&dsf, vb);
    if (he == hipSuccess && with_derivs) he = hipMalloc(&dse, vb);
    if (he == hipSuccess) he = hipMemsetAsync(V, 0, vb, st);
    if (he == hipSuccess) he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        release();
        return fail(NFFTGP_E_HIP, std::string("autotune buffers: ") + hipGetErrorString(he));
    }
    if (plan->cg_exec) {   // the captured CG iteration holds the old work lists
        (void)hipGraphExecDestroy(plan->cg_exec);
        plan->cg_exec = nullptr;
    }
    const uint32_t prof = plan->prof;
    plan->prof = 0;
    // best of two trials of `reps` applies, in milliseconds
    auto timed = [&](double &ms) -> nfftgp_status {
        ms = 1e300;
        for (int trial = 0; trial < 2; ++trial) {
            NFFTGP_HIP_TRY(hipEventRecord(e0, st));
            for (int k = 0; k < reps; ++k) {
                nfftgp_status e = apply_impl(plan, V, nrhs, nrhs, KV, dl, dsf, dse);
                if (e != NFFTGP_OK) return e;
            }
            NFFTGP_HIP_TRY(hipEventRecord(e1, st));
            NFFTGP_HIP_TRY(hipEventSynchronize(e1));
            float t = 0.f;
            NFFTGP_HIP_TRY(hipEventElapsedTime(&t, e0, e1));
            ms = std::min(ms, (double)t / reps);
        }
        return NFFTGP_OK;
    };
    std::string rep;
    nfftgp_status stt = NFFTGP_OK;
    double ms = 0.0;
    stt = timed(ms);   // warm-up and reference
    // short applies: enough repetitions for about 5 ms per trial, so that
    // launch jitter does not decide between candidates
    if (stt == NFFTGP_OK && ms > 0.0) reps = std::max(reps, std::min(200, (int)std::ceil(5.0 / ms)));
    for (size_t gi = 0; gi < plan->groups.size() && stt == NFFTGP_OK; ++gi) {
        Group &G = plan->groups[gi];
        // 1) spreading subproblem size (skipping sizes whose tiles would exceed 8 GiB)
        double best = 0.0;
        if ((stt = timed(best)) != NFFTGP_OK) break;
        int best_sp = G.sub_sp;
        for (int sp = kMinSubSp; sp <= 4096 && stt == NFFTGP_OK; sp *= 2) {
            if (sp == best_sp) continue;
            int64_t nsub = 0;
            for (int wl = 0; wl < G.nwin; ++wl) {
                const std::vector<int> &bs = plan->win[G.wins[wl]].h_bin_start;
                for (int b = 0; b < G.g.nbins; ++b) nsub += (bs[b + 1] - bs[b] + sp - 1) / sp;
            }
            if ((double)nsub * G.g.pc * plan->max_nrhs * eb > 8.0 * (1 << 30)) continue;
            if ((stt = build_spread_lists(plan, G, sp)) != NFFTGP_OK) break;
            double t = 0.0;
            if ((stt = timed(t)) != NFFTGP_OK) break;
            if (t < best) {
                best = t;
                best_sp = sp;
            }
        }
        if (stt != NFFTGP_OK) break;
        if ((stt = build_spread_lists(plan, G, best_sp)) != NFFTGP_OK) break;
        // 2) vectors per spreading work-group (0 = rule)
        int best_R = G.spread_R;
        for (int R : {1, 2, 4}) {
            if (R > nrhs || R == best_R) continue;
            G.spread_R = R;
            double t = 0.0;
            if ((stt = timed(t)) != NFFTGP_OK) break;
            if (t < best) {
                best = t;
                best_R = R;
            }
        }
        G.spread_R = best_R;
        if (stt != NFFTGP_OK) break;
        // 2a) spreading form: four-point and run-ordered, and matrix cores
        //     (FP32, d = 3, m = 4 or 6, four or more vectors)
        {
            const int cur_F = G.spread_form;
            std::vector<int> forms = {1, 2};
            if (plan->prec == NFFTGP_F32 && G.g.d == 3 && (plan->m == 4 || plan->m == 6) && nrhs >= 4)
                forms.push_back(3);
            int best_F = cur_F;
            for (int f : forms) {
                G.spread_form = f;
                double t = 0.0;
                if ((stt = timed(t)) != NFFTGP_OK) break;
                if (t < best) {
                    best = t;
                    best_F = f;
                }
            }
            if (stt != NFFTGP_OK) break;
            G.spread_form = best_F;
        }
        // 2b) 3-D: waves sharing a spreading tile (4 by rule, or 2)
        if (G.g.d == 3) {
            const int cur_W = G.spread_W;
            G.spread_W = cur_W == 2 ? 0 : 2;
            double t = 0.0;
            if ((stt = timed(t)) != NFFTGP_OK) break;
            if (t < best)
                best = t;
            else
                G.spread_W = cur_W;
        }
        // 3) interpolation variant: tile with 1 or 2 points per thread, whole
        //    padded tile or the rule's row window (3-D), or runs (the pair form
        //    is not a candidate: the tuner times applies with derivative outputs,
        //    and the pair form's K-only launches, which CG makes, are slower)
        const bool cur_run = G.use_run_interp, cur_adj = G.interp_adj, cur_slot = G.interp_slot;
        const bool cur_blk = G.interp_mfma;
        const int cur_pt = G.interp_pt, cur_rows = G.interp_rows;
        bool best_run = cur_run, best_adj = cur_adj, best_slot = cur_slot, best_blk = cur_blk;
        int best_pt = cur_pt, best_rows = cur_rows;
        struct Cand { bool run; int pt, rows; bool adj, slot, blk = false; };
        std::vector<Cand> cands;
        const int rr = interp_rows_rule(G.g, plan->m);
        for (int pt : {1, 2}) {
            cands.push_back({false, pt, rr, false, false});
            if (rr != G.g.pd) cands.push_back({false, pt, G.g.pd, false, false});
        }
        if (G.g.d == 3) {
            // one slot (one or two points of one cell) per thread
            cands.push_back({false, 2, rr, false, true});
            if (rr != G.g.pd) cands.push_back({false, 2, G.g.pd, false, true});
            // blocks of one cell on matrix cores (FP32, m = 4 or 6)
            if (plan->prec == NFFTGP_F32 && (plan->m == 4 || plan->m == 6)) {
                const int mr = interp_mfma_rows_rule(G.g, plan->m);
                cands.push_back({false, 1, mr, false, false, true});
                if (rr != mr) cands.push_back({false, 1, rr, false, false, true});
            }
        }
        // 2-D: blocks of one cell on matrix cores (FP32, m = 4 or 6)
        if (G.g.d == 2 && plan->prec == NFFTGP_F32 && (plan->m == 4 || plan->m == 6))
            cands.push_back({false, 1, G.g.pd, false, false, true});
        cands.push_back({true, cur_pt, cur_rows, cur_adj, cur_slot, cur_blk});
        for (const Cand &c : cands) {
            if (stt != NFFTGP_OK) break;
            if (c.run == cur_run && (c.run || (c.pt == cur_pt && c.rows == cur_rows && c.adj == cur_adj &&
                                               c.slot == cur_slot && c.blk == cur_blk)))
                continue;
            G.use_run_interp = c.run;
            G.interp_adj = c.adj;
            if (!c.run && (stt = build_interp_lists(plan, G, c.pt, c.rows, c.slot, c.blk)) != NFFTGP_OK) break;
            double t = 0.0;
            if ((stt = timed(t)) != NFFTGP_OK) break;
            if (t < best) {
                best = t;
                best_run = c.run;
                best_pt = c.pt;
                best_rows = c.rows;
                best_adj = c.adj;
                best_slot = c.slot;
                best_blk = c.blk;
            }
        }
        if (stt != NFFTGP_OK) break;
        G.use_run_interp = best_run;
        G.interp_adj = best_adj;
        if ((stt = build_interp_lists(plan, G, best_pt, best_rows, best_slot, best_blk)) != NFFTGP_OK) break;
        G.interp_adj = best_adj && !best_slot && !best_blk;
        std::string ivar = "run";
        if (!G.use_run_interp) {
            ivar = G.interp_mfma ? "matrix-core blocks of one cell"
                                 : (G.interp_slot ? "tile, same-cell point pairs"
                                                  : (G.interp_adj ? "tile, adjacent point pairs"
                                                                  : (G.interp_pt == 2 ? "tile, 2 points/thread" : "tile")));
            if (G.g.d == 3) ivar += ", " + std::to_string(G.interp_rows) + " of " + std::to_string(G.g.pd) + " rows";
        }
        char line[240];
        std::snprintf(line, sizeof(line), "group d=%d N=%d (%d windows): spread subproblem %d, vectors/group %s%s, "
                                          "interpolation %s; %.4f ms per apply\n",
                      G.g.d, G.g.N, G.nwin, G.sub_sp,
                      G.spread_R > 0 ? std::to_string(G.spread_R).c_str() : "rule",
                      (std::string(G.spread_form == 1 ? ", four-point form"
                                                      : (G.spread_form == 2 ? ", run form"
                                                                            : (G.spread_form == 3 ? ", matrix cores" : ""))) +
                       (G.spread_W == 2 ? ", 2 waves/tile" : "")).c_str(),
                      ivar.c_str(), best);
        rep += line;
    }
    plan->prof = prof;
    release();
    if (stt != NFFTGP_OK) return stt;
    if (report && report_len > 0) {
        std::strncpy(report, rep.c_str(), (size_t)report_len - 1);
        report[report_len - 1] = '\0';
    }
    return NFFTGP_OK;
}

nfftgp_status nfftgp_col_dots(nfftgp_plan plan, const void *A_dev, int64_t lda, const void *B_dev,
                              int64_t ldb, int64_t n, int32_t ncol, double *out_host)
{
    set_error("");
    if (!plan) return fail(NFFTGP_E_ARG, "plan is NULL");
    if (ncol < 1 || ncol > 64 || n < 0 || lda < ncol || ldb < ncol || !out_host)
        return fail(NFFTGP_E_ARG, "bad col_dots arguments");
    if (n > 0 && (!A_dev || !B_dev)) return fail(NFFTGP_E_ARG, "A or B is NULL");
    double *outd = plan->dot_part + kDotBlocks * 64;
    NFFTGP_HIP_TRY(launch_coldots(plan->prec, A_dev, lda, B_dev, ldb, n, ncol, plan->dot_part, outd,
                                  plan->stream));
    NFFTGP_HIP_TRY(hipMemcpyAsync(out_host, outd, ncol * sizeof(double), hipMemcpyDeviceToHost,
                                  plan->stream));
    NFFTGP_HIP_TRY(hipStreamSynchronize(plan->stream));
    return NFFTGP_OK;
}

nfftgp_status nfftgp_cg(nfftgp_plan plan, const void *B_dev, int32_t nrhs, void *X_dev, double tol,
                        int32_t maxit, int32_t check_every, int32_t *iters_host,
                        double *alpha_beta_host, double *resid_host)
{
    set_error("");
    if (!plan) return fail(NFFTGP_E_ARG, "plan is NULL");
    if (!plan->have_hyper) return fail(NFFTGP_E_STATE, "nfftgp_set_hyper has not been called");
    if (nrhs < 1 || nrhs > plan->max_nrhs) return fail(NFFTGP_E_ARG, "nrhs out of range 1..max_nrhs");
    if (maxit < 0 || !(tol >= 0.0)) return fail(NFFTGP_E_ARG, "bad tol or maxit");
    if (plan->n > 0 && (!B_dev || !X_dev)) return fail(NFFTGP_E_ARG, "B or X is NULL");
    if (alpha_beta_host && maxit > NFFTGP_MAX_CG_HISTORY)
        return fail(NFFTGP_E_ARG, "maxit exceeds NFFTGP_MAX_CG_HISTORY while the Lanczos history is asked for");
    if (check_every <= 0) check_every = 8;
    // coefficients pending from set_hyper are computed before the iteration is
    // enqueued or captured (a captured iteration never computes them)
    NFFTGP_HIP_TRY(resolve_coef(plan));
    const hipStream_t st = plan->stream;
    const int64_t n = plan->n;
    double *sc = plan->cg_scal;
    double *hist = alpha_beta_host ? plan->cg_hist : nullptr;
    PROF_LAUNCH(plan, NFFTGP_PROF_CG, launch_cg_init(plan->prec, n, nrhs, B_dev, X_dev, plan->cg_r, plan->cg_p, st));
    PROF_LAUNCH(plan, NFFTGP_PROF_CG, launch_coldots(plan->prec, plan->cg_r, nrhs, plan->cg_r, nrhs, n, nrhs,
                                                         plan->dot_part, sc + kRR * nrhs, st));
    PROF_LAUNCH(plan, NFFTGP_PROF_CG, launch_cg_start(nrhs, sc, st));
    // one iteration: apply, p^T Khat p, alpha, x/r update, r^T r, beta, p update
    // (enqueued on the plan's stream, or on the capture stream while capturing)
    auto iteration = [&]() -> nfftgp_status {
        const hipStream_t cs = plan->stream;
        nfftgp_status e = apply_impl(plan, plan->cg_p, nrhs, nrhs, plan->cg_ap, nullptr, nullptr, nullptr);
        if (e != NFFTGP_OK) return e;
        PROF_LAUNCH(plan, NFFTGP_PROF_CG, launch_dot_part(plan->prec, plan->cg_p, nrhs, plan->cg_ap, nrhs, n, nrhs,
                                                          plan->dot_part, cs));
        PROF_LAUNCH(plan, NFFTGP_PROF_CG, launch_cg_alpha(nrhs, plan->dot_part, sc, cs));
        PROF_LAUNCH(plan, NFFTGP_PROF_CG, launch_cg_xr(plan->prec, n, nrhs, sc, X_dev, plan->cg_r, plan->cg_p,
                                                       plan->cg_ap, plan->dot_part, cs));
        PROF_LAUNCH(plan, NFFTGP_PROF_CG, launch_cg_beta(nrhs, plan->dot_part, sc, tol, hist, cs));
        PROF_LAUNCH(plan, NFFTGP_PROF_CG, launch_cg_p(plan->prec, n, nrhs, sc, plan->cg_r, plan->cg_p, cs));
        return NFFTGP_OK;
    };
    // With NFFTGP_CG_GRAPH=1 the iterations between two convergence checks
    // (at most 16) are captured once into a graph and replayed (all their
    // arguments are fixed: the iteration index lives on the device); one graph
    // launch then covers gi iterations, and iterations left over at the end
    // run eagerly.  By default the iterations are enqueued eagerly: replaying
    // the graph was measured no faster (the host already runs ahead of the
    // device).  Never while profiling (events are per launch) or when n = 0.
    const char *ge = std::getenv("NFFTGP_CG_GRAPH");
    const bool use_graph = maxit > 0 && n > 0 && !plan->prof && ge && std::strcmp(ge, "1") == 0;
    const int gi = std::max(1, std::min({check_every, maxit, 16}));
    if (use_graph) {
        const bool hit = plan->cg_exec && plan->cg_key_nrhs == nrhs && plan->cg_key_x == X_dev &&
                         plan->cg_key_hist == hist && plan->cg_key_tol == tol &&
                         plan->cg_key_sf == plan->sigma_f && plan->cg_key_se == plan->sigma_eps &&
                         plan->cg_key_iters == gi;
        if (!hit) {
            if (plan->cg_exec) {
                NFFTGP_HIP_TRY(hipGraphExecDestroy(plan->cg_exec));
                plan->cg_exec = nullptr;
            }
            if (!plan->cap_stream)
                NFFTGP_HIP_TRY(hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking));
            hipGraph_t graph = nullptr;
            NFFTGP_HIP_TRY(hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeRelaxed));
            plan->stream = plan->cap_stream;
            nfftgp_status ce = NFFTGP_OK;
            for (int k = 0; k < gi && ce == NFFTGP_OK; ++k) ce = iteration();
            plan->stream = st;
            const hipError_t ee = hipStreamEndCapture(plan->cap_stream, &graph);
            if (ce != NFFTGP_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return ce;
            }
            NFFTGP_HIP_TRY(ee);
            const hipError_t ie = hipGraphInstantiate(&plan->cg_exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            NFFTGP_HIP_TRY(ie);
            plan->cg_key_nrhs = nrhs;
            plan->cg_key_x = X_dev;
            plan->cg_key_hist = hist;
            plan->cg_key_tol = tol;
            plan->cg_key_sf = plan->sigma_f;
            plan->cg_key_se = plan->sigma_eps;
            plan->cg_key_iters = gi;
        }
    }
    std::vector<double> act(nrhs);
    int it = 0;
    while (it < maxit) {
        // up to the next convergence check (or maxit): whole graph launches,
        // then single eager iterations
        const int stop = std::min(maxit, (it / check_every + 1) * check_every);
        while (it < stop) {
            if (use_graph && it + gi <= stop) {
                NFFTGP_HIP_TRY(hipGraphLaunch(plan->cg_exec, st));
                it += gi;
            } else {
                nfftgp_status e = iteration();
                if (e != NFFTGP_OK) return e;
                ++it;
            }
        }
        NFFTGP_HIP_TRY(hipMemcpyAsync(act.data(), sc + kActive * nrhs, nrhs * sizeof(double),
                                      hipMemcpyDeviceToHost, st));
        NFFTGP_HIP_TRY(hipStreamSynchronize(st));
        bool any = false;
        for (int c = 0; c < nrhs; ++c) any = any || act[c] != 0.0;
        if (!any) break;
    }
    std::vector<double> all((size_t)kCgSlots * nrhs);
    NFFTGP_HIP_TRY(hipMemcpyAsync(all.data(), sc, all.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    if (alpha_beta_host && maxit > 0) {
        std::memset(alpha_beta_host, 0, (size_t)maxit * nrhs * 2 * sizeof(double));
        if (it > 0)
            NFFTGP_HIP_TRY(hipMemcpyAsync(alpha_beta_host, hist, (size_t)it * nrhs * 2 * sizeof(double),
                                          hipMemcpyDeviceToHost, st));
    }
    NFFTGP_HIP_TRY(hipStreamSynchronize(st));
    bool notpd = false, noconv = false;
    for (int c = 0; c < nrhs; ++c) {
        double rr = all[kRR * nrhs + c], rr0 = all[kRR0 * nrhs + c];
        double rel = rr0 > 0.0 ? std::sqrt(rr / rr0) : 0.0;
        if (iters_host) iters_host[c] = (int32_t)all[kIters * nrhs + c];
        if (resid_host) resid_host[c] = rel;
        if (all[kNotPD * nrhs + c] != 0.0) notpd = true;
        else if (rel > tol) noconv = true;
    }
    if (notpd) return fail(NFFTGP_E_NOTPD, "CG met p^T Khat p <= 0 (operator not positive definite)");
    if (noconv) return fail(NFFTGP_E_NOCONV, "CG did not reach tol within maxit");
    return NFFTGP_OK;
}

nfftgp_status nfftgp_slq_logquad(const double *ab, const int32_t *iters, int32_t ncol, int32_t maxit,
                                 const double *znorm2, double *out)
{
    set_error("");
    if (!ab || !iters || !znorm2 || !out || ncol < 1 || maxit < 0)
        return fail(NFFTGP_E_ARG, "bad slq arguments");
    nfftgp_status status = NFFTGP_OK;
    for (int c = 0; c < ncol; ++c) {
        const int k = iters[c];
        if (k < 0 || k > maxit) return fail(NFFTGP_E_ARG, "iters out of range");
        if (k == 0) {
            out[c] = 0.0;
            continue;
        }
        // Lanczos tridiagonal from CG: T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
        // T_{j,j+1} = sqrt(beta_j)/alpha_j.
        std::vector<double> dg(k), e(k, 0.0), z(k, 0.0);
        for (int j = 0; j < k; ++j) {
            const double a = ab[((size_t)j * ncol + c) * 2];
            dg[j] = 1.0 / a;
            if (j > 0) {
                const double ap = ab[((size_t)(j - 1) * ncol + c) * 2];
                const double bp = ab[((size_t)(j - 1) * ncol + c) * 2 + 1];
                dg[j] += bp / ap;
                e[j - 1] = std::sqrt(bp) / ap;
            }
        }
        z[0] = 1.0;   // first row of the eigenvector matrix
        // implicit QL iteration with Wilkinson-type shifts on the symmetric
        // tridiagonal matrix (dg, e); rotations are applied to z.
        for (int l = 0; l < k; ++l) {
            int iter = 0, mm;
            do {
                for (mm = l; mm < k - 1; ++mm) {
                    double dd = std::fabs(dg[mm]) + std::fabs(dg[mm + 1]);
                    if (std::fabs(e[mm]) <= 1e-16 * dd) break;
                }
                if (mm != l) {
                    if (++iter > 200) return fail(NFFTGP_E_NOCONV, "tridiagonal eigen-solver did not converge");
                    double g = (dg[l + 1] - dg[l]) / (2.0 * e[l]);
                    double r = std::hypot(g, 1.0);
                    g = dg[mm] - dg[l] + e[l] / (g + (g >= 0 ? r : -r));
                    double s = 1.0, cc = 1.0, pp = 0.0;
                    int i;
                    bool early = false;
                    for (i = mm - 1; i >= l; --i) {
                        double f = s * e[i], b = cc * e[i];
                        r = std::hypot(f, g);
                        e[i + 1] = r;
                        if (r == 0.0) {
                            dg[i + 1] -= pp;
                            e[mm] = 0.0;
                            early = true;
                            break;
                        }
                        s = f / r;
                        cc = g / r;
                        g = dg[i + 1] - pp;
                        r = (dg[i] - g) * s + 2.0 * cc * b;
                        pp = s * r;
                        dg[i + 1] = g + pp;
                        g = cc * r - b;
                        double zf = z[i + 1];
                        z[i + 1] = s * z[i] + cc * zf;
                        z[i] = cc * z[i] - s * zf;
                    }
                    if (early) continue;
                    dg[l] -= pp;
                    e[l] = g;
                    e[mm] = 0.0;
                }
            } while (mm != l);
        }
        double acc = 0.0;
        for (int j = 0; j < k; ++j) {
            if (!(dg[j] > 0.0)) {
                status = NFFTGP_E_NOTPD;
                acc = NAN;
                break;
            }
            acc += z[j] * z[j] * std::log(dg[j]);
        }
        out[c] = znorm2[c] * acc;
    }
    if (status != NFFTGP_OK) set_error("Lanczos matrix has a non-positive eigenvalue");
    return status;
}

nfftgp_status nfftgp_get_window_info(nfftgp_plan plan, int32_t s, double *c0, double *c, int32_t *d,
                                     int32_t *N, double *min_b, double *min_bder)
{
    set_error("");
    if (!plan) return fail(NFFTGP_E_ARG, "plan is NULL");
    if (s < 0 || s >= plan->P) return fail(NFFTGP_E_ARG, "window index out of range");
    if (plan->minb_pending) {
        NFFTGP_HIP_TRY(resolve_coef(plan));
        for (const Group &G : plan->groups) NFFTGP_HIP_TRY(launch_coef_min(G, plan->minb_host, plan->stream));
        NFFTGP_HIP_TRY(hipStreamSynchronize(plan->stream));
        for (int k = 0; k < plan->P; ++k) {
            plan->win[k].min_b = plan->minb_host[2 * k];
            plan->win[k].min_bder = plan->minb_host[2 * k + 1];
        }
        plan->minb_pending = false;
    }
    const Window &w = plan->win[s];
    if (c0)
        for (int q = 0; q < w.g.d; ++q) c0[q] = w.c0[q];
    if (c) *c = w.c;
    if (d) *d = w.g.d;
    if (N) *N = w.g.N;
    if (min_b) *min_b = w.min_b;
    if (min_bder) *min_bder = w.min_bder;
    return NFFTGP_OK;
}

nfftgp_status nfftgp_get_workspace_bytes(nfftgp_plan plan, size_t *bytes)
{
    set_error("");
    if (!plan || !bytes) return fail(NFFTGP_E_ARG, "NULL argument");
    *bytes = plan->bytes;
    return NFFTGP_OK;
}

nfftgp_status nfftgp_describe(nfftgp_plan plan, int32_t nrhs, char *out, int64_t len)
{
    set_error("");
    if (!plan || !out) return fail(NFFTGP_E_ARG, "NULL argument");
    if (len < 1) return fail(NFFTGP_E_ARG, "len must be positive");
    if (nrhs < 1 || nrhs > plan->max_nrhs) return fail(NFFTGP_E_ARG, "nrhs out of range 1..max_nrhs");
    std::string rep;
    for (const Group &G : plan->groups) rep += describe_group(plan->prec, G, plan->m, nrhs);
    std::strncpy(out, rep.c_str(), (size_t)len - 1);
    out[len - 1] = '\0';
    return NFFTGP_OK;
}

nfftgp_status nfftgp_profile(nfftgp_plan plan, int32_t categories)
{
    set_error("");
    if (!plan) return fail(NFFTGP_E_ARG, "plan is NULL");
    plan->prof = (uint32_t)categories & ((1u << NFFTGP_PROF_COUNT) - 1u);
    plan->ev_used = 0;
    plan->prof_cat.clear();
    plan->prof_ev.clear();
    return NFFTGP_OK;
}

nfftgp_status nfftgp_profile_read(nfftgp_plan plan, double *ms_host, int32_t *count_host)
{
    set_error("");
    if (!plan || !ms_host || !count_host) return fail(NFFTGP_E_ARG, "NULL argument");
    NFFTGP_HIP_TRY(hipStreamSynchronize(plan->stream));
    for (int c = 0; c < NFFTGP_PROF_COUNT; ++c) {
        ms_host[c] = 0.0;
        count_host[c] = 0;
    }
    for (size_t r = 0; r < plan->prof_cat.size(); ++r) {
        float ms = 0.0f;
        int i = plan->prof_ev[r];
        NFFTGP_HIP_TRY(hipEventElapsedTime(&ms, plan->ev_pool[i], plan->ev_pool[i + 1]));
        ms_host[plan->prof_cat[r]] += ms;
        count_host[plan->prof_cat[r]] += 1;
    }
    return NFFTGP_OK;
}

void nfftgp_plan_destroy(nfftgp_plan plan) { free_plan(plan); }

}  // extern "C"
