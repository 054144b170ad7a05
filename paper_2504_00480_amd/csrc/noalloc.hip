// Allocation-free FP64 column dot products: the reduction of nfftgp_col_dots
// with its partial sums in a static device array instead of a plan workspace,
// for callers that cannot allocate (code under HIP graph capture, serving
// loops).  See nfftgp_col_dots_noalloc in include/nfftgp.h.
#include <mutex>
#include <string>

#include "nfftgp_impl.h"

namespace {

// Partial sums of one call: kDotBlocks per column, at most 64 columns.
constexpr int kScratchCols = 64;
constexpr size_t kScratchDoubles = (size_t)nfftgp::kDotBlocks * kScratchCols;

// One copy per device, held until the process ends.  Host code never passes
// this name to a kernel: it uses the device address obtained below.
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up once per device,
// with the device current).
hipError_t scratch_ptr(int dev, double **out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

nfftgp_status fail(nfftgp_status st, const std::string &m)
{
    nfftgp::set_error(m);
    return st;
}

}  // namespace

extern "C" nfftgp_status nfftgp_col_dots_noalloc(int32_t prec, const void *A_dev, int64_t lda,
                                                 const void *B_dev, int64_t ldb, int64_t n, int32_t ncol,
                                                 double *out_dev, void *stream)
{
    nfftgp::set_error("");
    if (prec != NFFTGP_F32 && prec != NFFTGP_F64) return fail(NFFTGP_E_ARG, "bad precision");
    if (ncol < 1 || ncol > kScratchCols)
        return fail(NFFTGP_E_ARG, "ncol must be in 1..64 (the static scratch holds the partial sums of 64 columns)");
    if (n < 0 || lda < ncol || ldb < ncol) return fail(NFFTGP_E_ARG, "bad col_dots_noalloc arguments");
    if (!out_dev) return fail(NFFTGP_E_ARG, "out_dev is NULL");
    if (n > 0 && (!A_dev || !B_dev)) return fail(NFFTGP_E_ARG, "A or B is NULL");
    int dev = 0;
    NFFTGP_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(NFFTGP_E_ARG, "device index beyond 63");
    double *part = nullptr;
    NFFTGP_HIP_TRY(scratch_ptr(dev, &part));
    // every partial slot the final sum reads is written by this launch, so the
    // scratch needs no clearing
    NFFTGP_HIP_TRY(nfftgp::launch_coldots(prec, A_dev, lda, B_dev, ldb, n, ncol, part, out_dev,
                                          (hipStream_t)stream));
    return NFFTGP_OK;
}
