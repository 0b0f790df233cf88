// Dense products of the preconditioner (Algorithms 3 and 4) on the FP64 matrix cores
// (v_mfma_f64_16x16x4_f64: exact FP64 products, FP64 sums).  All matrices are row-major.
//
//   gemm_tn:  C (ka x kb) = A^T B, A rows x ka, B rows x kb (the long dimension is the row count:
//             W^T W and W^T X over n points).  Rows are split over the grid and the partial tiles
//             are added in a fixed order, so the result does not depend on the launch.  The partial
//             tiles go to *ws when given (grown when too small; reused without allocating afterwards).
//   syrk_tn:  C (k x k) = A^T A; only the upper block triangle is computed, the result is exactly
//             symmetric.
//   gemm_nn:  C (m x nb) = A B, A m x k, B k x nb; optional epilogue C = (X - A B) diag(scale)
//             (the last step of Algorithm 4 for several right-hand sides).
// A may be FP32 (the rounded factor of FP32/mixed handles; its products are exact in FP64) or FP64.
#pragma once

#include "krr_internal.h"

namespace krr {

template <typename TA, typename TB>
void gemm_tn(const TA* A, int64_t lda, const TB* B, int64_t ldb, int64_t rows, int ka, int kb, double* C,
             int64_t ldc, hipStream_t s, DevBuf<double>* ws = nullptr);

template <typename TA>
void syrk_tn(const TA* A, int64_t lda, int64_t rows, int k, double* C, int64_t ldc, hipStream_t s);

// X, scale: nullptr for the plain product; else C[i, j] = (X[i, j] - (A B)[i, j]) * scale[j] (scale on device).
template <typename TA>
void gemm_nn(const TA* A, int64_t lda, const double* B, int64_t ldb, int64_t m, int k, int nb, double* C,
             int64_t ldc, const double* X, int64_t ldx, const double* scale, hipStream_t s);

}  // namespace krr
