// Anchor selection (Sec. 3, Algorithms 1-2): sketch and column-pivoted QR on the transposed sketch.
#pragma once

#include "krr_internal.h"

namespace krr {

// Algorithm 2 sketch written transposed: Yt[i, a] (l x n, row stride ldy), FP64 (prec FP64) or FP32.
void sketch_sparse_t(const double* X, int64_t n, int d, double eps, const int64_t* idx, const double* sign, int l,
                     int r, int prec, void* Yt, int64_t ldy, hipStream_t s);
// Y (n x l, FP64 row-major) <-> Yt (l x n, row stride ldy, FP64 or FP32 by prec)
void transpose_to_t(const double* Y, int64_t n, int l, int prec, void* Yt, int64_t ldy, hipStream_t s);
void transpose_from_t(const void* Yt, int64_t ldy, int64_t n, int l, int prec, double* Y, hipStream_t s);
// First k pivots of the column-pivoted QR of Yt (l x N): piv [dev] int64 k, rdiag [dev] k.
void qrcp_t(const void* Yt, int64_t ldy, int64_t N, int l, int k, int prec, int64_t* piv, double* rdiag,
            hipStream_t s);

}  // namespace krr
