// Validation-loss gradient with respect to log eps and log beta by the adjoint method.
//
//   alpha  = (K + beta I)^{-1} y_tr                      (forward PCG)
//   r_v    = K_vt alpha - y_val,  L = 1/2 ||r_v||^2
//   lambda = (K + beta I)^{-1} K_vt^T r_v                (adjoint PCG, same operator and preconditioner)
//   dL/dlog eps  = r_v^T K'_vt alpha - lambda^T K' alpha, K' = eps dK/deps = (D^2/eps) K
//   dL/dlog beta = -beta lambda^T alpha
// K_vt alpha and K'_vt alpha come from one fused (K, K') product; K' alpha on the training set from
// a derivative-kernel product.  The two solves run in the working precision; these few products
// that assemble the loss and the gradient run in FP64 (the validation residual r_v is a small
// difference of large terms when the model fits well, so reduced-precision products would be
// amplified).  The preconditioner only changes how the solves converge.
#include "kmv.h"
#include "pcg.h"
#include "precond.h"

namespace krr {

void validate_common(int64_t m, int64_t n, int32_t d, double eps);
void validate_prec(int32_t prec);
void kernel_mv_raw(const double* Xt, int64_t m, const double* Xs, int64_t n, int d, double eps, const double* V,
                   int R, const double* shift, int deriv, int prec, double* U, int64_t ldu, hipStream_t s);

// out[0] = sum a*b (strided reads a[i*sa], b[i*sb]); single block, fixed order.
__global__ __launch_bounds__(1024) void k_dot1(const double* __restrict__ a, int sa, const double* __restrict__ b,
                                               int sb, int64_t n, double* __restrict__ out) {
  __shared__ double red[1024];
  double s = 0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) s = __builtin_fma(a[i * sa], b[i * sb], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// rv[i] = U[i, 0] - yv[i]
__global__ void k_val_residual(const double* __restrict__ U, const double* __restrict__ yv, int64_t m,
                               double* __restrict__ rv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) rv[i] = U[2 * i] - yv[i];
}

static double dot_dev(const double* a, int sa, const double* b, int sb, int64_t n, double* tmp, hipStream_t s) {
  hipLaunchKernelGGL(k_dot1, dim3(1), dim3(1024), 0, s, a, sa, b, sb, n, tmp);
  KRR_LAUNCH_CHECK();
  double h = 0;
  KRR_CHECK_HIP(hipMemcpyAsync(&h, tmp, sizeof(double), hipMemcpyDeviceToHost, s));
  KRR_CHECK_HIP(hipStreamSynchronize(s));
  return h;
}

}  // namespace krr

extern "C" int krr_grad(const double* Xtr, int64_t n, const double* ytr, const double* Xval, int64_t m,
                        const double* yval, int32_t d, double eps, double beta, const krr_precond* P, double tol,
                        int32_t maxit, int32_t replace_every, int32_t prec, double* loss, double* dloss_dlog_eps,
                        double* dloss_dlog_beta, double* alpha_out, double* lambda_out, krr_solve_stats* stats,
                        void* stream) {
  using namespace krr;
  return guarded([&] {
    validate_common(m, n, d, eps);
    validate_prec(prec);
    KRR_REQUIRE(Xtr && ytr && Xval && yval && loss && dloss_dlog_eps && dloss_dlog_beta, "null pointer argument");
    KRR_REQUIRE(beta > 0 && std::isfinite(beta), "beta must be positive and finite");
    KRR_REQUIRE(tol > 0 && maxit >= 0 && replace_every >= 0, "invalid solver settings");
    hipStream_t s = (hipStream_t)stream;
    check_finite_device(Xtr, n * (int64_t)d, "Xtr", s);
    check_finite_device(Xval, m * (int64_t)d, "Xval", s);
    check_finite_device(ytr, n, "ytr", s);
    check_finite_device(yval, m, "yval", s);
    DevBuf<double> alpha(n, s), lam(n, s), Uv(2 * m, s), rv(m, s), g(n, s), Kpa(n, s), tmp(1, s);
    KRR_CHECK_HIP(hipMemsetAsync(alpha.p, 0, sizeof(double) * n, s));
    KRR_CHECK_HIP(hipMemsetAsync(lam.p, 0, sizeof(double) * n, s));
    // forward solve
    const bool timing = stats != nullptr;
    PcgResult f = pcg_solve(Xtr, n, d, eps, ytr, 1, &beta, P, tol, maxit, replace_every, prec, alpha.p, timing, s);
    if (f.status < 0) return f.status;
    // [K_vt alpha, K'_vt alpha]
    kernel_mv_raw(Xval, m, Xtr, n, d, eps, alpha.p, 1, nullptr, 2, KRR_FP64, Uv.p, 2, s);
    hipLaunchKernelGGL(k_val_residual, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, s, Uv.p, yval, m, rv.p);
    KRR_LAUNCH_CHECK();
    const double L = 0.5 * dot_dev(rv.p, 1, rv.p, 1, m, tmp.p, s);
    const double t1 = dot_dev(rv.p, 1, Uv.p + 1, 2, m, tmp.p, s);    // r_v^T K'_vt alpha
    // g = K_vt^T r_v = K(Xtr, Xval) r_v
    kernel_mv_raw(Xtr, n, Xval, m, d, eps, rv.p, 1, nullptr, 0, KRR_FP64, g.p, 1, s);
    // adjoint solve
    PcgResult a = pcg_solve(Xtr, n, d, eps, g.p, 1, &beta, P, tol, maxit, replace_every, prec, lam.p, timing, s);
    if (a.status < 0) return a.status;
    // K' alpha on the training set
    kernel_mv_raw(Xtr, n, Xtr, n, d, eps, alpha.p, 1, nullptr, 1, KRR_FP64, Kpa.p, 1, s);
    const double t2 = dot_dev(lam.p, 1, Kpa.p, 1, n, tmp.p, s);      // lambda^T K' alpha
    const double t3 = dot_dev(lam.p, 1, alpha.p, 1, n, tmp.p, s);    // lambda^T alpha
    if (stats) {
      stats[0] = f.st;
      stats[1] = a.st;
    }
    *loss = L;
    *dloss_dlog_eps = t1 - t2;
    *dloss_dlog_beta = -beta * t3;
    if (alpha_out) KRR_CHECK_HIP(hipMemcpyAsync(alpha_out, alpha.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    if (lambda_out) KRR_CHECK_HIP(hipMemcpyAsync(lambda_out, lam.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    return (f.status != KRR_OK || a.status != KRR_OK) ? (int)KRR_ENOCONV : (int)KRR_OK;
  });
}
