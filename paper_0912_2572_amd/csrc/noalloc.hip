// noalloc.hip -- tsqr_factor_solve_noalloc: factor, least squares and
// optionally the thin Q and R of one matrix with no device allocation,
// for callers that cannot allocate (HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// The workspace of the factorization lives in `scratch`, a file-scope device
// array of kScratchBytes that every GPU the library runs on holds until the
// process ends.  Host code never uses the array's name as an address (that
// is a host-side stand-in): at the first call on a device, with the device
// current, its device address is looked up once with hipGetSymbolAddress and
// kept per device; the kernels receive that address as their workspace
// argument, exactly as they receive a caller's workspace.
//
// Every call on one GPU shares that GPU's array, which keeps the last call's
// contents: nothing in it needs to start at zero (the factorization writes
// every region before reading it, and the multi-panel R is cleared by a fill
// kernel).  Calls that overlap on one GPU race; callers order them (one
// stream, or events).
#include <hip/hip_runtime.h>

#include <mutex>

#include "handle.h"
#include "plan.h"

namespace {

constexpr size_t kScratchBytes = TSQR_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];   // device address of `scratch` on each device

// The current device's address of `scratch` (looked up once per device).
int scratch_for_current_device(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return -1000 - (int)e;
    if (dev < 0 || dev >= kMaxDevices) return TSQR_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return -1000 - (int)e;
        if (!p) return -1000 - (int)hipErrorInvalidSymbol;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return 0;
}

}  // namespace

extern "C" {

TSQR_API int tsqr_factor_solve_noalloc(int64_t m, int64_t n, const double *A, int64_t lda, const tsqr_opts *o,
                                       int64_t k, const double *B, int64_t ldb, double *X, int64_t ldx,
                                       double *resid, int32_t *dinfo, double *Q, int64_t ldq, double *R,
                                       int64_t ldr, void *stream) {
    tsqr_opts defaults;
    tsqr_default_opts(&defaults);
    if (!o) o = &defaults;
    tsqr::Plan plan;
    int rc = tsqr::make_plan(m, n, o, &plan);
    if (rc) return rc;
    if (!A) return -3;
    if (lda < m) return -4;
    if (o->prec != TSQR_F64 || o->domain_weights) return TSQR_ERR_UNSUPPORTED;
    if (!o->keep_q) return TSQR_ERR_STATE;
    if (plan.total > kScratchBytes) return TSQR_ERR_WORKSPACE;
    if (k < 1 || k > o->lsq_max_rhs) return -6;
    if (!B) return -7;
    if (ldb < m) return -8;
    if (!X) return -9;
    if (ldx < n) return -10;
    if (Q && ldq < m) return -14;
    if (R && ldr < n) return -16;
    void *ws = nullptr;
    rc = scratch_for_current_device(&ws);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    tsqr_factors_s f;   // on the stack: the handle lives for this call only
    rc = tsqr::factor_into(&f, m, n, A, lda, o, ws, kScratchBytes, st);
    if (rc) return rc;
    rc = tsqr_lsq_solve(&f, A, lda, k, B, ldb, X, ldx, resid, dinfo, stream);
    if (!rc && Q) rc = tsqr_form_q(&f, Q, ldq, stream);
    if (!rc && R) rc = tsqr_get_r(&f, R, ldr, stream);
    return rc;
}

}  // extern "C"
