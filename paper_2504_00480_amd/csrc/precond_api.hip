// C ABI of the AAFN preconditioner (Sec. 2.3) and preconditioned CG: attach
// (landmarks by farthest point sampling, block order), per-theta factors
// (enqueued by nfftgp_set_hyper), log det M and tr(M^-1 dM/dtheta_j), the
// operators M^-1, F, F^-T, the quadratic forms w^T dM/dtheta_j w, and PCG.
// See include/nfftgp.h for the contract of every entry point.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "nfftgp_impl.h"

using namespace nfftgp;

namespace {

nfftgp_status fail(nfftgp_status st, const std::string &m)
{
    set_error(m);
    return st;
}

nfftgp_status palloc(nfftgp_plan p, void **ptr, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    const hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        return fail(NFFTGP_E_NOMEM, "hipMalloc(" + std::to_string(bytes) + " bytes) failed: " + hipGetErrorString(e));
    }
    p->allocs.push_back(*ptr);
    p->bytes += bytes;
    return NFFTGP_OK;
}

#define PTRY(expr)                                       \
    do {                                                 \
        const nfftgp_status st_ = (expr);                \
        if (st_ != NFFTGP_OK) return st_;                \
    } while (0)

PcKer make_ker(const nfftgp_plan p)
{
    PcKer kp{};
    kp.P = p->P;
    int off = 0;
    for (int s = 0; s < p->P; ++s) {
        kp.d[s] = p->win[s].g.d;
        kp.off[s] = off;
        kp.type[s] = p->win[s].kernel;
        kp.ell[s] = p->win[s].ell;
        off += p->win[s].g.d;
    }
    kp.ptot = off;
    kp.sf = p->sigma_f;
    kp.se = p->sigma_eps;
    return kp;
}

// Temporary device buffers of attach, freed on every exit path.
struct Tmp {
    std::vector<void *> p;
    ~Tmp()
    {
        for (void *x : p) (void)hipFree(x);
    }
    hipError_t get(void **ptr, size_t bytes)
    {
        const hipError_t e = hipMalloc(ptr, bytes == 0 ? 256 : bytes);
        if (e == hipSuccess) p.push_back(*ptr);
        return e;
    }
};

#define PLAUNCH(plan_, expr_)                                              \
    do {                                                                   \
        const int pi_ = prof_begin_cat(plan_, NFFTGP_PROF_PRECOND);         \
        NFFTGP_HIP_TRY(expr_);                                             \
        prof_end_cat(plan_, NFFTGP_PROF_PRECOND, pi_);                      \
    } while (0)

}  // namespace

namespace nfftgp {

nfftgp_status precond_refresh(nfftgp_plan p)
{
    Precond &pc = p->pc;
    pc.ker = make_ker(p);
    PLAUNCH(p, launch_pc_setup(pc, pc.ker, p->stream));
    pc.ready = true;
    pc.info_pending = true;
    return NFFTGP_OK;
}

}  // namespace nfftgp

extern "C" {

nfftgp_status nfftgp_precond_attach(nfftgp_plan plan, const void *X_dev, int64_t ldx, int32_t per_window,
                                    int32_t max_rank, int32_t block)
{
    set_error("");
    if (!plan) return fail(NFFTGP_E_ARG, "plan is NULL");
    if (plan->pc.on) return fail(NFFTGP_E_STATE, "a preconditioner is already attached to this plan");
    const int64_t n = plan->n;
    if (n < 1) return fail(NFFTGP_E_ARG, "the preconditioner needs n >= 1");
    if (!X_dev || ldx < plan->p) return fail(NFFTGP_E_ARG, "X_dev is NULL or ldx < p");
    if (plan->P > kPcMaxWin) return fail(NFFTGP_E_DIM, "the preconditioner supports at most 16 windows");
    if (per_window < 1) return fail(NFFTGP_E_ARG, "per_window must be >= 1");
    if (max_rank < 1 || max_rank > kPcMaxRank) return fail(NFFTGP_E_ARG, "max_rank must be in 1..512");
    if (block < 1 || block > kPcMaxBlock) return fail(NFFTGP_E_ARG, "block must be in 1..128");
    Precond &pc = plan->pc;
    const hipStream_t st = plan->stream;
    const int P = plan->P;
    PcKer kp = make_ker(plan);
    const int ptot = kp.ptot;
    // feature copy (FP64, caller units) and window centres
    std::vector<int> feat(ptot);
    std::vector<double> cen(ptot);
    for (int s = 0; s < P; ++s)
        for (int q = 0; q < plan->win[s].g.d; ++q) {
            feat[kp.off[s] + q] = plan->win[s].feat[q];
            cen[kp.off[s] + q] = plan->win[s].c0[q];
        }
    Tmp tmp;
    int *dfeat = nullptr, *sel = nullptr;
    double *dcen = nullptr, *mind = nullptr;
    int64_t *keys = nullptr;
    const int kw = (int)std::min<int64_t>(per_window, n);
    NFFTGP_HIP_TRY(tmp.get((void **)&dfeat, ptot * sizeof(int)));
    NFFTGP_HIP_TRY(tmp.get((void **)&dcen, ptot * sizeof(double)));
    NFFTGP_HIP_TRY(tmp.get((void **)&mind, (size_t)P * n * sizeof(double)));
    NFFTGP_HIP_TRY(tmp.get((void **)&sel, (size_t)P * kw * sizeof(int)));
    NFFTGP_HIP_TRY(tmp.get((void **)&keys, (size_t)n * sizeof(int64_t)));
    PTRY(palloc(plan, (void **)&pc.X, (size_t)n * ptot * sizeof(double)));
    NFFTGP_HIP_TRY(hipMemcpyAsync(dfeat, feat.data(), ptot * sizeof(int), hipMemcpyHostToDevice, st));
    NFFTGP_HIP_TRY(hipMemcpyAsync(dcen, cen.data(), ptot * sizeof(double), hipMemcpyHostToDevice, st));
    NFFTGP_HIP_TRY(launch_pc_gather(plan->prec, X_dev, ldx, n, ptot, dfeat, pc.X, st));
    NFFTGP_HIP_TRY(launch_pc_fps(pc.X, n, ptot, kp, dcen, kw, mind, sel, st));
    const Window &w0 = plan->win[0];
    NFFTGP_HIP_TRY(launch_pc_keys(pc.X, n, ptot, w0.g.d, w0.g.N, w0.g.tb, w0.c, dcen, keys, st));
    std::vector<int> hsel((size_t)P * kw);
    std::vector<int64_t> hkey(n);
    NFFTGP_HIP_TRY(hipMemcpyAsync(hsel.data(), sel, hsel.size() * sizeof(int), hipMemcpyDeviceToHost, st));
    NFFTGP_HIP_TRY(hipMemcpyAsync(hkey.data(), keys, n * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    NFFTGP_HIP_TRY(hipStreamSynchronize(st));
    // merge: ranks of all windows in turn, duplicates skipped, up to max_rank
    std::vector<char> is_lm(n, 0);
    std::vector<int> lm;
    for (int r = 0; r < kw && (int)lm.size() < max_rank; ++r)
        for (int s = 0; s < P && (int)lm.size() < max_rank; ++s) {
            const int j = hsel[(size_t)s * kw + r];
            if (j >= 0 && !is_lm[j]) {
                is_lm[j] = 1;
                lm.push_back(j);
            }
        }
    std::sort(lm.begin(), lm.end());
    // the other points in window-0 cell order (ties by index)
    std::vector<int> ord;
    ord.reserve(n - lm.size());
    for (int64_t i = 0; i < n; ++i)
        if (!is_lm[i]) ord.push_back((int)i);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return hkey[a] < hkey[b]; });
    pc.k = (int)lm.size();
    pc.np = (int64_t)ord.size();
    pc.f = block;
    pc.nblk = (int)((pc.np + block - 1) / block);
    pc.zrows = std::max<int64_t>(2048, (pc.np + 255) / 256);
    pc.nzpart = (int)std::max<int64_t>(1, (pc.np + pc.zrows - 1) / pc.zrows);
    pc.per_window = per_window;
    pc.max_rank = max_rank;
    pc.ptot = ptot;
    const int k = pc.k, mr = plan->max_nrhs, np2 = P + 2;
    const size_t kk = (size_t)k * k, npk = (size_t)std::max<int64_t>(1, pc.np) * k;
    const size_t nb = std::max(1, pc.nblk);
    const size_t eb = plan->prec == NFFTGP_F32 ? 4 : 8;
    PTRY(palloc(plan, (void **)&pc.lm, k * sizeof(int)));
    PTRY(palloc(plan, (void **)&pc.ord, std::max<size_t>(1, ord.size()) * sizeof(int)));
    double **mats[] = {&pc.K11, &pc.L11, &pc.L11inv, &pc.K11inv, &pc.Zk, &pc.Tk};
    for (double **m : mats) PTRY(palloc(plan, (void **)m, kk * sizeof(double)));
    PTRY(palloc(plan, (void **)&pc.dK11, np2 * kk * sizeof(double)));
    double **rows[] = {&pc.V, &pc.Y, &pc.Wt, &pc.G};
    for (double **m : rows) PTRY(palloc(plan, (void **)m, npk * sizeof(double)));
    PTRY(palloc(plan, (void **)&pc.LB, nb * block * block * sizeof(double)));
    PTRY(palloc(plan, (void **)&pc.LBinv, nb * block * block * sizeof(double)));
    PTRY(palloc(plan, (void **)&pc.part, nb * (np2 + 1) * sizeof(double)));
    PTRY(palloc(plan, (void **)&pc.zpart, (size_t)pc.nzpart * kk * sizeof(double)));
    PTRY(palloc(plan, (void **)&pc.acc, sizeof(double)));
    PTRY(palloc(plan, (void **)&pc.flag, sizeof(int)));
    PTRY(palloc(plan, (void **)&pc.out_dev, (np2 + 1) * sizeof(double)));
    double **vecs[] = {&pc.T1, &pc.R1, &pc.ABAR, &pc.W1};
    for (double **m : vecs) PTRY(palloc(plan, (void **)m, (size_t)mr * k * sizeof(double)));
    PTRY(palloc(plan, (void **)&pc.Q, nb * mr * k * sizeof(double)));
    PTRY(palloc(plan, (void **)&pc.lmt, (size_t)mr * np2 * sizeof(double)));
    PTRY(palloc(plan, (void **)&pc.dqp, nb * mr * np2 * sizeof(double)));
    PTRY(palloc(plan, (void **)&pc.dq_dev, (size_t)mr * np2 * sizeof(double)));
    PTRY(palloc(plan, &pc.pz, (size_t)n * mr * eb));
    {
        void *h = nullptr;
        NFFTGP_HIP_TRY(hipHostMalloc(&h, (np2 + 1) * sizeof(double), hipHostMallocDefault));
        pc.out_host = (double *)h;
        plan->host_allocs.push_back(h);
    }
    NFFTGP_HIP_TRY(hipMemcpyAsync(pc.lm, lm.data(), k * sizeof(int), hipMemcpyHostToDevice, st));
    if (!ord.empty())
        NFFTGP_HIP_TRY(hipMemcpyAsync(pc.ord, ord.data(), ord.size() * sizeof(int), hipMemcpyHostToDevice, st));
    NFFTGP_HIP_TRY(hipMemsetAsync(pc.flag, 0, sizeof(int), st));
    NFFTGP_HIP_TRY(hipStreamSynchronize(st));
    pc.on = true;
    if (plan->have_hyper) return precond_refresh(plan);
    return NFFTGP_OK;
}

nfftgp_status nfftgp_precond_info(nfftgp_plan plan, int32_t *k, int32_t *nblocks, double *logdet, double *dlogdet)
{
    set_error("");
    if (!plan) return fail(NFFTGP_E_ARG, "plan is NULL");
    Precond &pc = plan->pc;
    if (!pc.on) return fail(NFFTGP_E_STATE, "no preconditioner is attached");
    if (k) *k = pc.k;
    if (nblocks) *nblocks = pc.nblk;
    if (!logdet && !dlogdet) return NFFTGP_OK;
    if (!pc.ready) return fail(NFFTGP_E_STATE, "nfftgp_set_hyper has not been called");
    int flag = 0;
    if (pc.info_pending) {
        NFFTGP_HIP_TRY(hipMemcpyAsync(pc.out_host, pc.out_dev, (plan->P + 3) * sizeof(double),
                                      hipMemcpyDeviceToHost, plan->stream));
        NFFTGP_HIP_TRY(hipMemcpyAsync(&flag, pc.flag, sizeof(int), hipMemcpyDeviceToHost, plan->stream));
        NFFTGP_HIP_TRY(hipStreamSynchronize(plan->stream));
        if (flag) return fail(NFFTGP_E_NOTPD, "preconditioner: a Cholesky pivot was not positive");
        pc.info_pending = false;
    }
    if (logdet) *logdet = pc.out_host[0];
    if (dlogdet)
        for (int j = 0; j < plan->P + 2; ++j) dlogdet[j] = pc.out_host[1 + j];
    return NFFTGP_OK;
}

nfftgp_status nfftgp_precond_landmarks(nfftgp_plan plan, int32_t *idx_host)
{
    set_error("");
    if (!plan || !idx_host) return fail(NFFTGP_E_ARG, "NULL argument");
    if (!plan->pc.on) return fail(NFFTGP_E_STATE, "no preconditioner is attached");
    NFFTGP_HIP_TRY(hipMemcpyAsync(idx_host, plan->pc.lm, plan->pc.k * sizeof(int), hipMemcpyDeviceToHost,
                                  plan->stream));
    NFFTGP_HIP_TRY(hipStreamSynchronize(plan->stream));
    return NFFTGP_OK;
}

nfftgp_status nfftgp_precond_apply(nfftgp_plan plan, int32_t op, const void *V_dev, int32_t nrhs, void *out_dev)
{
    set_error("");
    if (!plan) return fail(NFFTGP_E_ARG, "plan is NULL");
    if (!plan->pc.on) return fail(NFFTGP_E_STATE, "no preconditioner is attached");
    if (!plan->pc.ready) return fail(NFFTGP_E_STATE, "nfftgp_set_hyper has not been called");
    if (op != NFFTGP_PC_MINV && op != NFFTGP_PC_FINVT && op != NFFTGP_PC_F) return fail(NFFTGP_E_ARG, "bad op");
    if (nrhs < 1 || nrhs > plan->max_nrhs) return fail(NFFTGP_E_ARG, "nrhs out of range 1..max_nrhs");
    if (!V_dev || !out_dev || V_dev == out_dev) return fail(NFFTGP_E_ARG, "V and out must be distinct device buffers");
    const int kop = op == NFFTGP_PC_MINV ? kPcMinv : (op == NFFTGP_PC_FINVT ? kPcFinvT : kPcFac);
    PLAUNCH(plan, launch_pc_apply(plan->prec, plan->pc, kop, V_dev, nrhs, out_dev, plan->stream));
    return NFFTGP_OK;
}

nfftgp_status nfftgp_precond_dquad(nfftgp_plan plan, const void *W_dev, int32_t nrhs, double *out_host)
{
    set_error("");
    if (!plan || !out_host) return fail(NFFTGP_E_ARG, "NULL argument");
    if (!plan->pc.on) return fail(NFFTGP_E_STATE, "no preconditioner is attached");
    if (!plan->pc.ready) return fail(NFFTGP_E_STATE, "nfftgp_set_hyper has not been called");
    if (nrhs < 1 || nrhs > plan->max_nrhs || !W_dev) return fail(NFFTGP_E_ARG, "bad W or nrhs");
    Precond &pc = plan->pc;
    PLAUNCH(plan, launch_pc_dquad(plan->prec, pc, pc.ker, W_dev, nrhs, pc.dq_dev, plan->stream));
    NFFTGP_HIP_TRY(hipMemcpyAsync(out_host, pc.dq_dev, (size_t)(plan->P + 2) * nrhs * sizeof(double),
                                  hipMemcpyDeviceToHost, plan->stream));
    NFFTGP_HIP_TRY(hipStreamSynchronize(plan->stream));
    return NFFTGP_OK;
}

nfftgp_status nfftgp_pcg(nfftgp_plan plan, const void *B_dev, int32_t nrhs, void *X_dev, double tol, int32_t maxit,
                         int32_t check_every, int32_t *iters_host, double *alpha_beta_host, double *resid_host)
{
    set_error("");
    if (!plan) return fail(NFFTGP_E_ARG, "plan is NULL");
    if (!plan->have_hyper) return fail(NFFTGP_E_STATE, "nfftgp_set_hyper has not been called");
    if (!plan->pc.on) return fail(NFFTGP_E_STATE, "no preconditioner is attached");
    if (nrhs < 1 || nrhs > plan->max_nrhs) return fail(NFFTGP_E_ARG, "nrhs out of range 1..max_nrhs");
    if (maxit < 0 || !(tol >= 0.0)) return fail(NFFTGP_E_ARG, "bad tol or maxit");
    if (!B_dev || !X_dev) return fail(NFFTGP_E_ARG, "B or X is NULL");
    if (alpha_beta_host && maxit > NFFTGP_MAX_CG_HISTORY)
        return fail(NFFTGP_E_ARG, "maxit exceeds NFFTGP_MAX_CG_HISTORY while the Lanczos history is asked for");
    if (check_every <= 0) check_every = 8;
    NFFTGP_HIP_TRY(resolve_coef(plan));
    const hipStream_t st = plan->stream;
    const int64_t n = plan->n;
    const int prec = plan->prec;
    Precond &pc = plan->pc;
    double *sc = plan->cg_scal;
    double *hist = alpha_beta_host ? plan->cg_hist : nullptr;
    double *prz = plan->dot_part;                              // r^T z partials
    double *outd = plan->dot_part + kDotBlocks * 64;           // final sums
    double *prr = outd + 64;                                   // r^T r partials
    void *R = plan->cg_r, *Pv = plan->cg_p, *AP = plan->cg_ap, *Z = pc.pz;
    const size_t vb = (size_t)n * nrhs * (prec == NFFTGP_F32 ? 4 : 8);
    auto cglaunch = [&](hipError_t e) -> nfftgp_status {
        if (e != hipSuccess) return fail(NFFTGP_E_HIP, std::string("PCG launch: ") + hipGetErrorString(e));
        return NFFTGP_OK;
    };
    // r = b, x = 0, z = M^-1 r, p = z; ||b||^2 and r^T z
    PTRY(cglaunch(launch_cg_init(prec, n, nrhs, B_dev, X_dev, R, Pv, st)));
    PLAUNCH(plan, launch_pc_apply(prec, pc, kPcMinv, R, nrhs, Z, st));
    PTRY(cglaunch(launch_coldots(prec, R, nrhs, R, nrhs, n, nrhs, prz, sc + kRRNew * nrhs, st)));
    PTRY(cglaunch(launch_coldots(prec, R, nrhs, Z, nrhs, n, nrhs, prz, sc + kRR * nrhs, st)));
    PTRY(cglaunch(launch_pcg_start(nrhs, sc, st)));
    NFFTGP_HIP_TRY(hipMemcpyAsync(Pv, Z, vb, hipMemcpyDeviceToDevice, st));
    std::vector<double> act(nrhs);
    int it = 0;
    for (; it < maxit; ++it) {
        PTRY(apply_impl(plan, Pv, nrhs, nrhs, AP, nullptr, nullptr, nullptr));
        PTRY(cglaunch(launch_dot_part(prec, Pv, nrhs, AP, nrhs, n, nrhs, prz, st)));
        PTRY(cglaunch(launch_cg_alpha(nrhs, prz, sc, st)));
        PTRY(cglaunch(launch_cg_xr(prec, n, nrhs, sc, X_dev, R, Pv, AP, prr, st)));
        PLAUNCH(plan, launch_pc_apply(prec, pc, kPcMinv, R, nrhs, Z, st));
        PTRY(cglaunch(launch_dot_part(prec, R, nrhs, Z, nrhs, n, nrhs, prz, st)));
        PTRY(cglaunch(launch_pcg_beta(nrhs, prr, prz, sc, tol, hist, st)));
        PTRY(cglaunch(launch_cg_p(prec, n, nrhs, sc, Z, Pv, st)));
        if ((it + 1) % check_every == 0 || it + 1 == maxit) {
            NFFTGP_HIP_TRY(hipMemcpyAsync(act.data(), sc + kActive * nrhs, nrhs * sizeof(double),
                                          hipMemcpyDeviceToHost, st));
            NFFTGP_HIP_TRY(hipStreamSynchronize(st));
            bool any = false;
            for (int c = 0; c < nrhs; ++c) any = any || act[c] != 0.0;
            if (!any) {
                ++it;
                break;
            }
        }
    }
    std::vector<double> all((size_t)kCgSlots * nrhs);
    NFFTGP_HIP_TRY(hipMemcpyAsync(all.data(), sc, all.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    if (alpha_beta_host && maxit > 0) {
        std::memset(alpha_beta_host, 0, (size_t)maxit * nrhs * 2 * sizeof(double));
        if (it > 0)
            NFFTGP_HIP_TRY(hipMemcpyAsync(alpha_beta_host, hist, (size_t)it * nrhs * 2 * sizeof(double),
                                          hipMemcpyDeviceToHost, st));
    }
    int flag = 0;
    NFFTGP_HIP_TRY(hipMemcpyAsync(&flag, pc.flag, sizeof(int), hipMemcpyDeviceToHost, st));
    NFFTGP_HIP_TRY(hipStreamSynchronize(st));
    if (flag) return fail(NFFTGP_E_NOTPD, "preconditioner: a Cholesky pivot was not positive");
    bool notpd = false, noconv = false;
    for (int c = 0; c < nrhs; ++c) {
        const double rr = all[kRRNew * nrhs + c], rr0 = all[kRR0 * nrhs + c];
        const double rel = rr0 > 0.0 ? std::sqrt(rr / rr0) : 0.0;
        if (iters_host) iters_host[c] = (int32_t)all[kIters * nrhs + c];
        if (resid_host) resid_host[c] = rel;
        if (all[kNotPD * nrhs + c] != 0.0) notpd = true;
        else if (rel > tol) noconv = true;
    }
    if (notpd) return fail(NFFTGP_E_NOTPD, "PCG met p^T Khat p <= 0 (operator not positive definite)");
    if (noconv) return fail(NFFTGP_E_NOCONV, "PCG did not reach tol within maxit");
    return NFFTGP_OK;
}

}  // extern "C"
