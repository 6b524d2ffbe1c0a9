// handle.h -- the library's internal view of a factorization handle.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "plan.h"

// What tsqr_factors points to: the plan and the caller's workspace.
struct tsqr_factors_s {
    tsqr::Plan plan;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int keep_q = 1;
    int last_refine = 0;
    int64_t last_k = 0;   // right-hand sides of the last mixed solve
    int route_checked = 0;  // mixed: the condition estimate of routing has run
    double kappa_est = 0.0; // ... and its value
};

namespace tsqr {

// tsqr_factor into a handle the caller owns (nothing is allocated): plans the
// factorization, checks the arguments and the workspace, and enqueues the
// kernels on st.  Returns 0 or tsqr_factor's error codes.
int factor_into(tsqr_factors_s *f, int64_t m, int64_t n, const double *A, int64_t lda, const tsqr_opts *o,
                void *dwork, size_t work_bytes, hipStream_t st);

}  // namespace tsqr
