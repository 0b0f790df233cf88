// Small dense FP64 linear algebra for the preconditioner build (see dense.h).
#include "dense.h"
#include "kmv_kernels.h"   // exp_neg_f64

#include <cstring>

namespace krr {

// ------------------------------------------------------------------ kernel blocks, gather
__global__ void k_kernel_block(const double* __restrict__ A, int64_t ma, const double* __restrict__ B, int64_t nb,
                               int d, double inv_eps, double* __restrict__ out, int64_t ldo, int rowmajor) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ma * nb) return;
  int64_t a, b;
  if (rowmajor) { a = idx / nb; b = idx % nb; }
  else { a = idx % ma; b = idx / ma; }
  double d2 = 0;
  for (int k = 0; k < d; ++k) {
    const double df = A[a * d + k] - B[b * d + k];
    d2 = __builtin_fma(df, df, d2);
  }
  const double v = exp_neg_f64(d2 * inv_eps);
  if (rowmajor) out[a * ldo + b] = v;
  else out[a + b * ldo] = v;
}

void kernel_block_colmajor(const double* A, int64_t ma, const double* B, int64_t nb, int d, double eps,
                           double* out, int64_t ldo, hipStream_t s) {
  const int64_t tot = ma * nb;
  hipLaunchKernelGGL(k_kernel_block, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, A, ma, B, nb, d,
                     1.0 / eps, out, ldo, 0);
  KRR_LAUNCH_CHECK();
}

void kernel_block_rowmajor(const double* A, int64_t ma, const double* B, int64_t nb, int d, double eps,
                           double* out, int64_t ldo, hipStream_t s) {
  const int64_t tot = ma * nb;
  hipLaunchKernelGGL(k_kernel_block, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, A, ma, B, nb, d,
                     1.0 / eps, out, ldo, 1);
  KRR_LAUNCH_CHECK();
}

__global__ void k_gather_rows(const double* __restrict__ X, int64_t n, int d, const int64_t* __restrict__ idx,
                              int64_t k, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= k * d) return;
  const int64_t a = t / d;
  const int c = (int)(t % d);
  int64_t r = idx[a];
  r = r < 0 ? 0 : (r >= n ? n - 1 : r);   // indices are validated on the host path; clamp keeps reads in bounds
  out[t] = X[r * d + c];
}

void gather_rows(const double* X, int64_t n, int d, const int64_t* idx, int64_t k, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)ceil_div(k * d, 256)), dim3(256), 0, s, X, n, d, idx, k, out);
  KRR_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ block reduction helper
template <int NT>
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* red) {
  // red: 3*NT doubles of LDS; fixed-order tree
  red[threadIdx.x] = a;
  red[NT + threadIdx.x] = b;
  red[2 * NT + threadIdx.x] = c;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[threadIdx.x] += red[threadIdx.x + w];
      red[NT + threadIdx.x] += red[NT + threadIdx.x + w];
      red[2 * NT + threadIdx.x] += red[2 * NT + threadIdx.x + w];
    }
    __syncthreads();
  }
  a = red[0];
  b = red[NT];
  c = red[2 * NT];
}

// ------------------------------------------------------------------ one-sided Jacobi
// Round r of the circle-method tournament on K (even) players: slot 0 pairs (r, K-1), slot i > 0
// pairs ((r+i) mod (K-1), (r-i) mod (K-1)).  Over r = 0..K-2 every pair meets exactly once.
// Players >= k are byes (k odd).
__global__ __launch_bounds__(256) void k_jacobi_round(double* __restrict__ A, double* __restrict__ V, int k, int K,
                                                      int r, double rot_tol,
                                                      unsigned long long* __restrict__ offmax) {
  __shared__ double red[3 * 256];
  const int i = blockIdx.x;
  int p, q;
  if (i == 0) { p = r; q = K - 1; }
  else { p = (r + i) % (K - 1); q = (r - i + K - 1) % (K - 1); }
  if (p > q) { int t = p; p = q; q = t; }
  if (q >= k) return;
  double* ap = A + (int64_t)p * k;
  double* aq = A + (int64_t)q * k;
  double a = 0, b = 0, g = 0;
  for (int t = threadIdx.x; t < k; t += 256) {
    const double x = ap[t], y = aq[t];
    a = __builtin_fma(x, x, a);
    b = __builtin_fma(y, y, b);
    g = __builtin_fma(x, y, g);
  }
  block_sum3<256>(a, b, g, red);
  const double den = sqrt(a * b);
  const double off = den > 0 ? fabs(g) / den : 0.0;
  if (threadIdx.x == 0) atomicMax(offmax, (unsigned long long)__double_as_longlong(off));
  if (!(off > rot_tol)) return;
  const double zeta = (b - a) / (2.0 * g);
  const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double c = 1.0 / sqrt(1.0 + tt * tt);
  const double sn = c * tt;
  double* vp = V + (int64_t)p * k;
  double* vq = V + (int64_t)q * k;
  for (int t = threadIdx.x; t < k; t += 256) {
    const double x = ap[t], y = aq[t];
    ap[t] = c * x - sn * y;
    aq[t] = sn * x + c * y;
    const double u = vp[t], w = vq[t];
    vp[t] = c * u - sn * w;
    vq[t] = sn * u + c * w;
  }
}

__global__ void k_identity(double* __restrict__ V, int k) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)k * k) return;
  V[idx] = (idx % k) == (idx / k) ? 1.0 : 0.0;
}

__global__ __launch_bounds__(256) void k_col_norms(const double* __restrict__ A, int k, double* __restrict__ out) {
  __shared__ double red[3 * 256];
  const double* a = A + (int64_t)blockIdx.x * k;
  double s = 0, z0 = 0, z1 = 0;
  for (int t = threadIdx.x; t < k; t += 256) s = __builtin_fma(a[t], a[t], s);
  block_sum3<256>(s, z0, z1, red);
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt(s);
}

int jacobi_evd(double* A, double* V, double* lam, int k, hipStream_t s, int max_sweeps) {
  hipLaunchKernelGGL(k_identity, dim3((unsigned)ceil_div((int64_t)k * k, 256)), dim3(256), 0, s, V, k);
  KRR_LAUNCH_CHECK();
  if (k == 1) {
    hipLaunchKernelGGL(k_col_norms, dim3(1), dim3(256), 0, s, A, k, lam);
    KRR_LAUNCH_CHECK();
    return 0;
  }
  const int K = k + (k & 1);
  DevBuf<unsigned long long> off(1, s);
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    KRR_CHECK_HIP(hipMemsetAsync(off.p, 0, sizeof(unsigned long long), s));
    for (int r = 0; r < K - 1; ++r) {
      hipLaunchKernelGGL(k_jacobi_round, dim3(K / 2), dim3(256), 0, s, A, V, k, K, r, 1e-15, off.p);
    }
    KRR_LAUNCH_CHECK();
    unsigned long long h = 0;
    KRR_CHECK_HIP(hipMemcpyAsync(&h, off.p, sizeof(h), hipMemcpyDeviceToHost, s));
    KRR_CHECK_HIP(hipStreamSynchronize(s));
    double offv;
    std::memcpy(&offv, &h, sizeof(offv));
    if (offv <= 1e-13) { ++sweep; break; }
  }
  hipLaunchKernelGGL(k_col_norms, dim3(k), dim3(256), 0, s, A, k, lam);
  KRR_LAUNCH_CHECK();
  return sweep;
}

// ------------------------------------------------------------------ Cholesky (right-looking, one launch per column)
// Step j: L[i, j] = A[i, j] / sqrt(A[j, j]) for i >= j, and A[i, t] -= A[i, j] A[t, j] / A[j, j] for
// j < t <= i.  Column j of A is only read during step j, so L can be written without a race.
__global__ __launch_bounds__(256) void k_chol_step(double* __restrict__ A, double* __restrict__ L, int k, int j,
                                                   int* __restrict__ info) {
  if (*info != 0) return;
  const double ajj = A[(int64_t)j * k + j];
  if (!(ajj > 0.0) || !isfinite(ajj)) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && threadIdx.y == 0) *info = j + 1;
    return;
  }
  const double rs = 1.0 / sqrt(ajj);
  const int m = k - j - 1;                       // trailing size
  const int ii = blockIdx.x * 64 + threadIdx.x;  // 0..m-1 -> row j+1+ii
  const int tt = blockIdx.y * 4 + threadIdx.y;   // 0..m-1 -> col j+1+tt
  if (blockIdx.y == 0 && threadIdx.y == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) L[(int64_t)j * k + j] = ajj * rs;
    if (ii < m) L[(int64_t)j * k + j + 1 + ii] = A[(int64_t)j * k + j + 1 + ii] * rs;
  }
  if (ii >= m || tt >= m || tt > ii) return;
  const int64_t i = j + 1 + ii, t = j + 1 + tt;
  const double ai = A[(int64_t)j * k + i], at = A[(int64_t)j * k + t];
  A[t * k + i] -= ai * at / ajj;
}

int cholesky_lower(double* A, double* L, int k, hipStream_t s) {
  DevBuf<int> info(1, s);
  KRR_CHECK_HIP(hipMemsetAsync(info.p, 0, sizeof(int), s));
  KRR_CHECK_HIP(hipMemsetAsync(L, 0, sizeof(double) * (size_t)k * k, s));
  for (int j = 0; j < k; ++j) {
    const int m = std::max(k - j - 1, 1);
    hipLaunchKernelGGL(k_chol_step, dim3((unsigned)ceil_div(m, 64), (unsigned)ceil_div(m, 4)), dim3(64, 4), 0, s, A,
                       L, k, j, info.p);
  }
  KRR_LAUNCH_CHECK();
  int h = 0;
  KRR_CHECK_HIP(hipMemcpyAsync(&h, info.p, sizeof(int), hipMemcpyDeviceToHost, s));
  KRR_CHECK_HIP(hipStreamSynchronize(s));
  return h;
}

// ------------------------------------------------------------------ lower-triangular inverse
// Block j solves L x = e_j by column-oriented forward substitution with x in LDS.
__global__ __launch_bounds__(256) void k_lower_inverse_col(const double* __restrict__ L, double* __restrict__ X,
                                                           int k) {
  extern __shared__ double x[];
  const int j = blockIdx.x;
  for (int i = threadIdx.x; i < k; i += 256) x[i] = (i == j) ? 1.0 : 0.0;
  __syncthreads();
  for (int t = j; t < k; ++t) {
    const double xt = x[t] / L[(int64_t)t * k + t];
    __syncthreads();
    if (threadIdx.x == 0) x[t] = xt;
    for (int i = t + 1 + threadIdx.x; i < k; i += 256) x[i] -= xt * L[(int64_t)t * k + i];
    __syncthreads();
  }
  for (int i = threadIdx.x; i < k; i += 256) X[(int64_t)j * k + i] = i >= j ? x[i] : 0.0;
}

void lower_inverse(const double* L, double* X, int k, hipStream_t s) {
  KRR_REQUIRE((size_t)k * sizeof(double) <= 160 * 1024, "k too large for the LDS triangular inverse");
  hipLaunchKernelGGL(k_lower_inverse_col, dim3(k), dim3(256), (size_t)k * sizeof(double), s, L, X, k);
  KRR_LAUNCH_CHECK();
}

}  // namespace krr
