// Internal declarations shared by the HIP translation units of libnfftgp.
// Everything here is private to the library; the public surface is
// include/nfftgp.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "nfftgp.h"

namespace nfftgp {

// Oversampling factor of the Kaiser-Bessel window (Appendix A): the FFT grid
// has 2N points per dimension, i.e. sigma = 2, and the window shape parameter
// is b = pi (2 - 1/sigma).
constexpr double kSigma = 2.0;
constexpr double kPi = 3.14159265358979323846264338327950288;
inline double kb_beta() { return kPi * (2.0 - 1.0 / kSigma); }

// Points handled by one interpolation work-group at most (one per thread).
constexpr int kInterpSubPoints = 256;
// 3-D matrix-core interpolation: blocks (at most 16 points of one cell) per
// subproblem, at most (the kernel form that keeps the points' weights in LDS
// takes at most kInterpSubBlocksLds)
constexpr int kInterpSubBlocks = 32;
constexpr int kInterpSubBlocksLds = 16;
// 2-D matrix-core interpolation: values staged per cell and pass (K and dK of
// half as many vectors with derivative outputs)
constexpr int kInterp2Values = 16;
// d <= 2 several-vector interpolation: points per subproblem by rule
constexpr int kInterpVbSubPoints = 2048;
// Points per wave in run-based interpolation.
constexpr int kRunSubPoints = 512;

// Geometry of one window's oversampled grid and its tiling.
struct WindowGeom {
    int d = 0;       // window dimension (1..3)
    int N = 0;       // bandwidth; index set I_N = [-N/2, N/2)^d
    int ng = 0;      // FFT grid edge 2N
    int tb = 0;      // tile (bin) edge in grid cells
    int nb = 0;      // bins per dimension = ng / tb
    int nbins = 0;   // nb^d
    int pd = 0;      // padded tile edge tb + 2m
    int pc = 0;      // padded tile cells pd^d
    int64_t cells = 0;  // ng^d
    int64_t dcells = 0; // (N+1)^d entries of the symmetrised diagonal
};

struct Window {
    WindowGeom g;
    int kernel = 0;
    int feat[3] = {0, 0, 0};
    double c0[3] = {0, 0, 0};
    double c = 1.0;
    double ell = 1.0;
    double min_b = 0.0, min_bder = 0.0;
    // device data (owned)
    void *rec = nullptr;        // per sorted point: d x 2m window weights (plan precision)
    int32_t *anchor = nullptr;  // per sorted point: packed cell floor(t); bit 31 = last of its run
    int32_t *lpos = nullptr;    // per sorted point: first-tap position in its padded tile
                                // (bits 0-19 offset, 20-26 first coordinate; bit 31 as anchor)
    int32_t *perm = nullptr;    // sorted position -> original point index
    int32_t *slots = nullptr;   // 3-D: interpolation slots in sorted order, each one point or
                                // two consecutive points of one cell (first point | pair << 31)
    int32_t *blocks = nullptr;  // 3-D: first point of each block (at most 16 consecutive points
                                // of one cell) in sorted order, then n
    int32_t *bin_sub_ptr = nullptr;  // tile -> spreading subproblems of its group (nbins + 1)
    void *Dk = nullptr;     // symmetrised diagonal for K_s (dcells, plan precision)
    void *Dder = nullptr;   // same for K_s^der
    // host copies used while the plan is built
    std::vector<int> h_bin_start;   // tile -> first sorted point (kept for re-tuning)
    std::vector<int> h_row_cnt;     // 3-D: points per (tile, first-axis cell row), nbins x tb
    std::vector<int> h_slot_start;  // 3-D: tile -> first slot (nbins + 1)
    std::vector<int> h_row_slots;   // 3-D: slots per (tile, first-axis cell row), nbins x tb
    std::vector<int> h_block_start; // 3-D: tile -> first block (nbins + 1)
    std::vector<int> h_row_blocks;  // 3-D: blocks per (tile, first-axis cell row), nbins x tb
};

// Per-window data a kernel needs, in device memory (one array per group).
struct WinDesc {
    const void *rec;
    const int32_t *anchor;
    const int32_t *lpos;
    const int32_t *perm;
    const int32_t *bin_sub_ptr;
    const void *Dk;
    const void *Dder;
    const int32_t *slots;
    const int32_t *blocks;
    int32_t s_global;   // window index in the plan
    int32_t pad_;
};

// Windows of equal dimension and bandwidth go through every apply kernel in
// one launch; their work lists are concatenated.
// Per-window parameters of one group's coefficient kernels (passed by value).
struct CoefParams {
    double ell[NFFTGP_MAX_WINDOWS];
    double c[NFFTGP_MAX_WINDOWS];
    int32_t kernel[NFFTGP_MAX_WINDOWS];
    int32_t nwin;
};

struct Group {
    WindowGeom g;
    int nwin = 0;
    std::vector<int> wins;       // plan window indices
    WinDesc *desc = nullptr;     // device, nwin entries
    int32_t *sub_win = nullptr, *sub_bin = nullptr, *sub_start = nullptr, *sub_count = nullptr;
    int nsub = 0;                // spreading subproblems (tile slots)
    int32_t *isub_win = nullptr, *isub_bin = nullptr, *isub_start = nullptr, *isub_count = nullptr;
    int nisub = 0;               // interpolation subproblems
    // d <= 2: the several-vector interpolation's own list, subproblems of up to
    // vsub_sp points of one tile (the tile is staged once per vector batch for
    // all of them)
    int32_t *vsub_win = nullptr, *vsub_bin = nullptr, *vsub_start = nullptr, *vsub_count = nullptr;
    int nvsub = 0, vsub_cap = 0, vsub_sp = 0;
    int nbins_used = 0;          // tiles holding at least one point
    // tunables (rule defaults at plan creation; nfftgp_autotune may change them)
    int sub_sp = 0;              // points per spreading subproblem
    int spread_R = 0;            // vectors per spreading work-group (0: rule)
    int spread_W = 0;            // 3-D: waves sharing a spreading tile (0: rule, 4; or 2)
    int spread_form = 0;         // spreading kernel: 0 rule (four-point form for one vector
                                 // per work-group, else run-ordered), 1 four-point, 2 run-ordered,
                                 // 3 matrix cores (FP32, d = 3)
    int spread_mfma_R = 4;       // vectors per matrix-core spreading work-group (4, or 2: two
                                 // work-groups per CU, a padded column block)
    // every window Gaussian: set_hyper only records theta (prm) and the next
    // apply computes the coefficients in extra work-groups of its fold launch
    bool sep = false;
    bool coef_pending = false;
    CoefParams prm{};
    int sub_cap = 0;             // capacity of the spreading list arrays
    int interp_pt = 1;           // points per thread of the tile interpolation (1, 2)
    bool interp_adj = false;     // 3-D, 2 points per thread: adjacent sorted points share tap reads
    bool interp_slot = false;    // 3-D: one slot per thread (two points of one cell share every tap read)
    bool interp_mfma = false;    // 3-D FP32: blocks of one cell on matrix cores (lists count blocks)
    int interp_sub_blocks = kInterpSubBlocksLds;   // blocks per matrix-core interpolation subproblem
    int fold_form = 0;           // 3-D fold: 0 by rule, 1 per cell, 2 by tiles
    int interp_mfma_waves = 8;   // waves per work-group of the matrix-core interpolation (8: weights
                                 // read from L2, two work-groups per CU; 16: weights in LDS)
    int interp_vb_lds = 80 << 10;   // d <= 2: LDS bytes for several vectors per staging (0: one vector)
    int interp_rows = 0;         // 3-D: first-axis rows of the padded tile staged per subproblem
    int isub_cap = 0;            // capacity of the interpolation list arrays
    int32_t *fb = nullptr;       // tiles split into several subproblems (window * nbins + tile)
    int nfb = 0;
    // interpolation by register-held runs (selectable; see use_run_interp):
    // contiguous ranges of at most kRunSubPoints sorted points
    bool use_run_interp = false;
    int32_t *rsub_win = nullptr, *rsub_start = nullptr, *rsub_count = nullptr;
    int nrsub = 0;
    double *cinv2 = nullptr;     // N+1 window factors 1 / c(k)^2 (same for the whole group)
    double *cw = nullptr;        // (N/2+1)^2 weights of the real coefficient transform
    double *coef_part = nullptr; // per-block minima of the coefficients (last set_hyper)
};

// ---------------------------------------------------------------- AAFN
// Windows the preconditioner handles at most (one derivative per window is
// carried in registers).
constexpr int kPcMaxWin = 16;
constexpr int kPcMaxRank = 512;
constexpr int kPcMaxBlock = 128;
// Application operators: M^-1 v, F^-T v, F v (M = F F^T).
enum { kPcMinv = 0, kPcFinvT = 1, kPcFac = 2 };

// Exact-kernel parameters of the preconditioner (passed by value).
struct PcKer {
    int32_t P, ptot;
    int32_t d[kPcMaxWin], off[kPcMaxWin], type[kPcMaxWin];
    double ell[kPcMaxWin];
    double sf, se;
};

// Additive AFN preconditioner state (FP64, all device arrays owned by the plan).
struct Precond {
    bool on = false;
    bool ready = false;          // factors of the current theta enqueued
    bool info_pending = false;   // log det / traces not yet copied to the host
    int k = 0;                   // landmarks
    int64_t np = 0;              // other points
    int f = 0;                   // Schur-complement block size
    int nblk = 0, nzpart = 0;
    int64_t zrows = 0;           // rows per partial sum of Y^T Y
    int per_window = 0, max_rank = 0, ptot = 0;
    double *X = nullptr;         // n x ptot window features, caller units
    int32_t *lm = nullptr;       // k landmark indices, ascending
    int32_t *ord = nullptr;      // np other points in block order
    double *K11 = nullptr, *dK11 = nullptr, *L11 = nullptr, *L11inv = nullptr, *K11inv = nullptr;
    double *V = nullptr, *Y = nullptr, *Wt = nullptr, *G = nullptr;   // np x k each
    double *LB = nullptr, *LBinv = nullptr;                             // nblk x f x f each
    double *part = nullptr;      // nblk x (P + 3): block log det and trace shares
    double *zpart = nullptr;     // nzpart x k x k
    double *Zk = nullptr, *Tk = nullptr;   // k x k scratch
    double *acc = nullptr;       // log det K11
    int *flag = nullptr;         // non-positive pivot met
    double *out_dev = nullptr;   // log det M, then P + 2 traces
    double *out_host = nullptr;  // pinned copy
    // application scratch (max_nrhs vectors)
    double *T1 = nullptr, *R1 = nullptr, *ABAR = nullptr, *W1 = nullptr;   // max_nrhs x k
    double *Q = nullptr;         // nblk x max_nrhs x k
    double *lmt = nullptr;       // max_nrhs x (P + 2)
    double *dqp = nullptr;       // nblk x max_nrhs x (P + 2)
    double *dq_dev = nullptr;    // (P + 2) x max_nrhs
    void *pz = nullptr;          // PCG z vectors (n x max_nrhs, plan precision)
    PcKer ker{};
};

}  // namespace nfftgp

struct nfftgp_plan_s {
    int64_t n = 0;
    int p = 0;
    int P = 0;
    int m = 0;
    int prec = 0;
    int max_nrhs = 0;
    int scale_mode = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    std::vector<nfftgp::Window> win;
    std::vector<nfftgp::Group> groups;
    bool have_hyper = false;
    double sigma_f = 0.0, sigma_eps = 0.0;
    // workspaces (owned)
    void *tilebuf = nullptr;     // spreading tiles
    size_t tile_cap = 0;         // tilebuf capacity in values per vector
    void *grid = nullptr;        // (windows of a group) x max_nrhs x cells complex values: the real
                                 // grid before the transforms, kernel + i derivative grid after
    void *hbuf = nullptr;        // P x n x max_nrhs per-window products
    double *coef = nullptr;      // set_hyper scratch (real coefficient transforms)
    double *minb_host = nullptr; // 2 x P smallest coefficients (pinned, written by the
                                 // coefficient kernel, read lazily)
    bool minb_pending = false;
    double *dot_part = nullptr;  // dot-product partials
    double *cg_scal = nullptr;   // CG per-column scalars
    double *cg_hist = nullptr;   // CG (alpha, beta) history, NFFTGP_MAX_CG_HISTORY x max_nrhs x 2
    void *cg_r = nullptr, *cg_p = nullptr, *cg_ap = nullptr;  // n x max_nrhs
    // one CG iteration captured as a graph, with the arguments it was captured for
    hipGraphExec_t cg_exec = nullptr;
    hipStream_t cap_stream = nullptr;   // capture only (the plan's stream may be the null stream)
    int cg_key_nrhs = 0;
    const void *cg_key_x = nullptr;
    const double *cg_key_hist = nullptr;
    double cg_key_tol = 0.0, cg_key_sf = 0.0, cg_key_se = 0.0;
    int cg_key_iters = 0;       // iterations the captured graph holds
    nfftgp::Precond pc;          // AAFN preconditioner (nfftgp_precond_attach)
    size_t bytes = 0;
    std::vector<void *> allocs;
    std::vector<void *> host_allocs;   // pinned host memory (hipHostFree)
    // kernel timing (nfftgp_profile)
    uint32_t prof = 0;           // bit c set: launches of category c are timed
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<int> prof_cat;   // one entry per recorded launch: category
    std::vector<int> prof_ev;    // index of its first event (second is +1)
};

namespace nfftgp {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
#define NFFTGP_HIP_TRY(expr)                                                       \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            ::nfftgp::set_error(std::string(#expr) + ": " + hipGetErrorString(e_)); \
            return NFFTGP_E_HIP;                                                   \
        }                                                                          \
    } while (0)

// ---------------------------------------------------------------- plan-time kernels
// Per-feature min / max over the n points of the given features (FP64 result,
// 2*d doubles: lo[0..d), hi[0..d)) and a NaN flag.  `part` is scratch of
// kPartBlocks * 2 * 3 doubles.
constexpr int kPartBlocks = 256;
hipError_t launch_minmax(int prec, const void *X, int64_t n, int64_t ldx, int d, const int *feat,
                         double *part, double *out, int *nanflag, hipStream_t s);

// Grid coordinates t = 2N c (x - c0) + N per window feature (SoA, d x n, plan
// precision), bin keys, and a flag set when a scaled coordinate leaves
// [-1/4, 1/4).
hipError_t launch_coords(int prec, const void *X, int64_t n, int64_t ldx, int d, const int *feat,
                         const double *c0, double c, const WindowGeom &g, void *t_out, int *keys,
                         int *boxflag, hipStream_t s);

// Stable counting sort of points by bin key.  hist: nbins * nblk ints;
// scan_tmp: scan scratch; perm / t_sorted: outputs; bin_start: nbins + 1 ints.
constexpr int kSortBlock = 4096;
int64_t scan_scratch_ints(int64_t len);
hipError_t launch_sort(int prec, int64_t n, int d, int nbins, const int *keys, const int *ids_in,
                       const void *t_in, int *hist, int *scan_tmp, int *perm, void *t_sorted,
                       int *bin_start, hipStream_t s);
hipError_t launch_bin_keys(int prec, const void *t, int64_t n, const WindowGeom &g, int *keys,
                           hipStream_t s);
// Window weights, packed cells and tile positions (with run-end flags) of the
// sorted points.
double kb_knorm(int m);
hipError_t launch_weights(int prec, const void *t, int64_t n, const WindowGeom &g, int m,
                          double knorm, void *rec, int *anchor, int *lpos, hipStream_t s);
// Points per (tile, first-axis cell row of the tile) of a 3-D window, from the
// packed cells; counts (nbins x tb ints) must be zero on entry.
hipError_t launch_row_counts(const int *anchor, int64_t n, const WindowGeom &g, int *counts,
                             hipStream_t s);

// ---------------------------------------------------------------- per-theta kernels
// Coefficients b_k, b^der_k of one window (FP64) and the symmetrised diagonals.
// Window factors 1 / c(k)^2 (N + 1) and the real-transform weights ((N/2+1)^2).
hipError_t launch_window_coef(int N, int m, double *cinv2, double *cw, hipStream_t s);
// Scratch (doubles) the coefficient kernel of a group needs.
int64_t coef_scratch_doubles(const WindowGeom &g, int nwin);

// ---------------------------------------------------------------- apply kernels
// Coefficients and diagonals of every window of a group (two launches); the
// per-block minima of the coefficients go to G.coef_part, from which
// launch_coef_min writes the smallest b_k, b^der_k of window s to minb[2 s],
// minb[2 s + 1] when they are asked for.
int64_t coef_part_doubles(const WindowGeom &g, int nwin);
hipError_t launch_coefficients(int prec, const Group &G, const CoefParams &prm, const double *cinv2,
                               double *scratch, hipStream_t s);
hipError_t launch_coef_min(const Group &G, double *minb, hipStream_t s);
hipError_t launch_spread(int prec, const Group &G, int m, const void *V, int64_t ldv, int nrhs,
                         void *tilebuf, hipStream_t s);
// with_coef: the fold launch also computes the group's (separable)
// coefficients, diagonals and block minima from G.prm.
hipError_t launch_fold(int prec, const Group &G, int m, int nrhs, void *tilebuf, void *grid,
                       bool with_coef, hipStream_t s);
// Pruned FFT pipeline of one group: forward transforms of axes d-1..1, then
// axis 0 forward + diagonal (and derivative diagonal) + axis 0 inverse, then
// inverse transforms of axes 1..d-1 over the K (and derivative) blocks.
hipError_t launch_fft_fwd(int prec, const Group &G, int m, void *grid, int nrhs, hipStream_t s);
hipError_t launch_fft_diag(int prec, const Group &G, int m, void *grid, int nrhs, bool with_der,
                           hipStream_t s);
hipError_t launch_fft_inv(int prec, const Group &G, int m, void *grid, int nrhs, bool with_der,
                          hipStream_t s);
hipError_t launch_interp(int prec, const Group &G, int m, int64_t n, int nrhs, const void *grid,
                         bool with_der, void *hbuf, void *dout, double dscale, hipStream_t s);
hipError_t launch_assemble(int prec, int64_t n, int nrhs, int P, const void *V, int64_t ldv,
                           const void *hbuf, double sf, double se, void *KV, void *dsf, void *dse,
                           hipStream_t s);
// One line naming the kernel forms an apply of nrhs vectors takes for group G.
std::string describe_group(int prec, const Group &G, int m, int nrhs);

// ---------------------------------------------------------------- CG / dots
constexpr int kDotBlocks = 120;
hipError_t launch_coldots(int prec, const void *A, int64_t lda, const void *B, int64_t ldb,
                          int64_t n, int ncol, double *part, double *out, hipStream_t s);
hipError_t launch_cg_init(int prec, int64_t n, int nrhs, const void *B, void *X, void *R, void *Pv,
                          hipStream_t s);
hipError_t launch_cg_start(int nrhs, double *scal, hipStream_t s);
// One CG iteration besides the apply: partials of p^T Khat p (launch_dot_part),
// their sum and alpha (launch_cg_alpha, also advances the iteration index),
// the x/r update with the partials of the new r^T r (launch_cg_xr), their sum,
// beta, the convergence test and the Lanczos history (launch_cg_beta), then p.
hipError_t launch_dot_part(int prec, const void *A, int64_t lda, const void *B, int64_t ldb, int64_t n,
                           int ncol, double *part, hipStream_t s);
hipError_t launch_cg_alpha(int nrhs, const double *part, double *scal, hipStream_t s);
hipError_t launch_cg_xr(int prec, int64_t n, int nrhs, const double *scal, void *X, void *R,
                        const void *Pv, const void *AP, double *part, hipStream_t s);
hipError_t launch_cg_beta(int nrhs, const double *part, double *scal, double tol, double *hist, hipStream_t s);
hipError_t launch_cg_p(int prec, int64_t n, int nrhs, const double *scal, const void *R, void *Pv,
                       hipStream_t s);

// AAFN preconditioner kernels (k_precond.hip).
hipError_t launch_pc_gather(int prec, const void *X, int64_t ldx, int64_t n, int ptot, const int *feat, double *Xw,
                            hipStream_t s);
hipError_t launch_pc_fps(const double *X, int64_t n, int ptot, const PcKer &kp, const double *centre, int kw,
                         double *mind, int *sel, hipStream_t s);
hipError_t launch_pc_keys(const double *X, int64_t n, int ptot, int d, int N, int tb, double c, const double *c0,
                          int64_t *key, hipStream_t s);
// factors of M at kp's theta, log det M and tr(M^-1 dM/dtheta_j) into pc.out_dev
hipError_t launch_pc_setup(const Precond &pc, const PcKer &kp, hipStream_t s);
// out = op(v) for nrhs vectors (n x nrhs, plan precision; out must not alias v)
hipError_t launch_pc_apply(int prec, const Precond &pc, int op, const void *v, int nrhs, void *out, hipStream_t s);
// out[j * nrhs + c] = w_c^T dM/dtheta_j w_c (device, FP64)
hipError_t launch_pc_dquad(int prec, const Precond &pc, const PcKer &kp, const void *w, int nrhs, double *out,
                           hipStream_t s);
hipError_t launch_pcg_start(int nrhs, double *scal, hipStream_t s);
hipError_t launch_pcg_beta(int nrhs, const double *prr, const double *prz, double *scal, double tol, double *hist,
                           hipStream_t s);

// Shared between the C ABI translation units (api.hip, precond_api.hip).
hipError_t resolve_coef(nfftgp_plan p);
nfftgp_status apply_impl(nfftgp_plan p, const void *V, int64_t ldv, int nrhs, void *KV, void *dell, void *dsf,
                         void *dse);
int prof_begin_cat(nfftgp_plan p, int cat);
void prof_end_cat(nfftgp_plan p, int cat, int i);
// Enqueue the preconditioner's factorisation at the plan's current theta.
nfftgp_status precond_refresh(nfftgp_plan p);

// Layout of the per-column CG scalar block (doubles, each an array of nrhs).
enum CgSlot {
    kRR = 0,      // current r^T r
    kRR0 = 1,     // b^T b
    kPAP = 2,     // p^T Khat p
    kAlpha = 3,
    kBeta = 4,
    kActive = 5,  // 1 while the column iterates
    kIters = 6,   // iterations done
    kNotPD = 7,   // 1 if p^T Khat p <= 0 was met
    kRRNew = 8,
    kStep = 9,    // iteration index (element 0 only)
    kCgSlots = 10
};

}  // namespace nfftgp
