// Anchor choices other than the pivoted QR (remark in Sec. 3) and the bounding box used by the
// data-driven rank of Corollary tradeoff.
#pragma once

#include "krr_internal.h"

namespace krr {

// Farthest point sampling: S [dev] int64 k picks (S[0] = start), dsel [dev] k squared pick
// distances (dsel[0] = inf; may be NULL).  X [dev] n x d FP64 row-major.
void fps_select(const double* X, int64_t n, int d, int k, int64_t start, int64_t* S, double* dsel, hipStream_t s);

// Per-coordinate minimum and maximum of X [dev] n x d into host arrays of d values (synchronises).
void bounding_box(const double* X, int64_t n, int d, double* lo_host, double* hi_host, hipStream_t s);

}  // namespace krr
