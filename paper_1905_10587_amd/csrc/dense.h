// Small dense FP64 linear algebra for the preconditioner build (k x k with k up to a few
// thousand), all column-major: kernel blocks K(A, B), a one-sided Jacobi symmetric EVD, a
// Cholesky factorisation and a lower-triangular inverse.
#pragma once

#include "krr_internal.h"

namespace krr {

// out[a + b*ldo] = exp(-||A_a - B_b||^2 / eps)  (A: ma x d, B: nb x d, row-major); column-major out.
void kernel_block_colmajor(const double* A, int64_t ma, const double* B, int64_t nb, int d, double eps,
                           double* out, int64_t ldo, hipStream_t s);
// Row-major variant: out[a*ldo + b].
void kernel_block_rowmajor(const double* A, int64_t ma, const double* B, int64_t nb, int d, double eps,
                           double* out, int64_t ldo, hipStream_t s);
// out[a, :] = X[idx[a], :]
void gather_rows(const double* X, int64_t n, int d, const int64_t* idx, int64_t k, double* out, hipStream_t s);

// Symmetric positive semidefinite EVD by one-sided (Hestenes) Jacobi with a round-robin parallel
// ordering.  A (k x k, column-major) is overwritten by A V whose columns are orthogonal; V holds
// the eigenvectors and lam[i] = ||(A V)_i|| the eigenvalues (unsorted).  Returns sweeps used.
int jacobi_evd(double* A, double* V, double* lam, int k, hipStream_t s, int max_sweeps = 40);

// Lower Cholesky factor of the symmetric positive definite A (k x k, column-major, lower part
// read; A is overwritten).  L receives the factor (upper part zeroed).  Returns 0 on success or
// (j+1) for the first non-positive or non-finite pivot j.
int cholesky_lower(double* A, double* L, int k, hipStream_t s);

// X = L^{-1} for lower-triangular L (column-major); X is lower triangular.
void lower_inverse(const double* L, double* X, int k, hipStream_t s);

}  // namespace krr
