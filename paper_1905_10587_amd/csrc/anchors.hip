// Other anchor choices named in the remark of Sec. 3 (random sampling, farthest point sampling)
// and the data-driven rank of Corollary tradeoff (Eq. condbound).
//
// Farthest point sampling: S[0] = start; step j adds the point, not yet chosen, whose squared
// distance to the nearest chosen point is largest (ties to the lowest index).  Two launches per
// step: every block lowers dmin[i] = min(dmin[i], ||x_i - x_{S[j-1]}||^2) over its rows and
// proposes its best row; a second, one-block launch picks the winner among the proposals,
// records it and marks it chosen (dmin = -1).  The distances are summed coordinate by
// coordinate with every operation rounded on its own, so the picks are reproducible exactly.
#include <algorithm>
#include <cmath>
#include <vector>

#include "anchors.h"

namespace krr {

constexpr int kFpsThreads = 256;
constexpr int kFpsMaxBlocks = 2048;

__device__ __forceinline__ double sqdist_unfused(const double* __restrict__ xi, const double* __restrict__ xs,
                                                 int d) {
#pragma clang fp contract(off)
  double acc = 0.0;
  for (int c = 0; c < d; ++c) {
    const double t = xi[c] - xs[c];
    acc = acc + t * t;
  }
  return acc;
}

// (v, i) beats (w, j): larger value, then lower index.
__device__ __forceinline__ bool fps_better(double v, int64_t i, double w, int64_t j) {
  return v > w || (v == w && i < j);
}

__global__ void k_fps_init(int64_t* __restrict__ S, double* __restrict__ dsel, int64_t start) {
  S[0] = start;
  if (dsel) dsel[0] = INFINITY;
}

// Block-wide argmax of (rv, ri) in LDS; the result ends in rv[0], ri[0].
__device__ __forceinline__ void fps_block_best(double* rv, int64_t* ri, int tid) {
  __syncthreads();
  for (int h = kFpsThreads / 2; h > 0; h >>= 1) {
    if (tid < h && fps_better(rv[tid + h], ri[tid + h], rv[tid], ri[tid])) {
      rv[tid] = rv[tid + h];
      ri[tid] = ri[tid + h];
    }
    __syncthreads();
  }
}

// Step j, first launch: lower dmin over the block's rows and propose the block's best row.
__global__ __launch_bounds__(kFpsThreads) void k_fps_update(const double* __restrict__ X, int64_t n, int d,
                                                            const int64_t* __restrict__ S, int j,
                                                            double* __restrict__ dmin, double* __restrict__ bval,
                                                            int64_t* __restrict__ bidx) {
  __shared__ double xs[KRR_MAX_D];
  __shared__ double rv[kFpsThreads];
  __shared__ int64_t ri[kFpsThreads];
  const int tid = threadIdx.x;
  const int64_t last = S[j - 1];
  const int64_t first = S[0];
  for (int c = tid; c < d; c += kFpsThreads) xs[c] = X[last * d + c];
  __syncthreads();
  double best = -INFINITY;
  int64_t bi = n;
  const int64_t stride = (int64_t)gridDim.x * kFpsThreads;
  for (int64_t i = (int64_t)blockIdx.x * kFpsThreads + tid; i < n; i += stride) {
    const double v = sqdist_unfused(X + i * d, xs, d);
    double nv;
    if (j == 1) {
      nv = i == first ? -1.0 : v;             // the start point is chosen
    } else {
      const double old = dmin[i];
      nv = old < 0.0 ? old : fmin(old, v);
    }
    dmin[i] = nv;
    if (nv > best) { best = nv; bi = i; }     // rows ascend within a thread: first maximum kept
  }
  rv[tid] = best;
  ri[tid] = bi;
  fps_block_best(rv, ri, tid);
  if (tid == 0) {
    bval[blockIdx.x] = rv[0];
    bidx[blockIdx.x] = ri[0];
  }
}

// Step j, second launch (one block): the best proposal becomes S[j]; it is marked chosen.
__global__ __launch_bounds__(kFpsThreads) void k_fps_pick(int nb, const double* __restrict__ bval,
                                                          const int64_t* __restrict__ bidx, int64_t n,
                                                          int64_t* __restrict__ S, double* __restrict__ dsel, int j,
                                                          double* __restrict__ dmin) {
  __shared__ double rv[kFpsThreads];
  __shared__ int64_t ri[kFpsThreads];
  const int tid = threadIdx.x;
  double best = -INFINITY;
  int64_t bi = n;
  for (int b = tid; b < nb; b += kFpsThreads)
    if (fps_better(bval[b], bidx[b], best, bi)) { best = bval[b]; bi = bidx[b]; }
  rv[tid] = best;
  ri[tid] = bi;
  fps_block_best(rv, ri, tid);
  if (tid == 0) {
    // k <= n leaves an unchosen point (dmin >= 0 > -1), so the winner is a real, new row
    const int64_t w = ri[0] < n ? ri[0] : 0;
    S[j] = w;
    if (dsel) dsel[j] = rv[0];
    dmin[w] = -1.0;
  }
}

void fps_select(const double* X, int64_t n, int d, int k, int64_t start, int64_t* S, double* dsel, hipStream_t s) {
  KRR_REQUIRE(k >= 1 && k <= n, "need 1 <= k <= n");
  KRR_REQUIRE(start >= 0 && start < n, "start must be in [0, n)");
  KRR_REQUIRE(d >= 1 && d <= KRR_MAX_D, "d must be in [1, KRR_MAX_D]");
  const int nb = (int)std::min<int64_t>(ceil_div(n, kFpsThreads), kFpsMaxBlocks);
  DevBuf<double> dmin(k > 1 ? n : 0, s), bval(nb, s);
  DevBuf<int64_t> bidx(nb, s);
  hipLaunchKernelGGL(k_fps_init, dim3(1), dim3(1), 0, s, S, dsel, start);
  KRR_LAUNCH_CHECK();
  for (int j = 1; j < k; ++j) {
    hipLaunchKernelGGL(k_fps_update, dim3((unsigned)nb), dim3(kFpsThreads), 0, s, X, n, d, S, j, dmin.p, bval.p,
                       bidx.p);
    hipLaunchKernelGGL(k_fps_pick, dim3(1), dim3(kFpsThreads), 0, s, nb, bval.p, bidx.p, n, S, dsel, j, dmin.p);
    KRR_LAUNCH_CHECK();
  }
}

// ------------------------------------------------------------------ bounding box
constexpr int64_t kBoxRows = 65536;   // rows per block

// lo/hi[slice * d + c] = min/max of X[i, c] over the rows of one slice.
__global__ __launch_bounds__(256) void k_bbox(const double* __restrict__ X, int64_t n, int d, double* __restrict__ lo,
                                              double* __restrict__ hi) {
  __shared__ double rl[256], rh[256];
  const int c = blockIdx.y;
  const int64_t i0 = (int64_t)blockIdx.x * kBoxRows;
  const int64_t i1 = std::min<int64_t>(i0 + kBoxRows, n);
  double a = INFINITY, b = -INFINITY;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
    const double v = X[i * d + c];
    a = fmin(a, v);
    b = fmax(b, v);
  }
  rl[threadIdx.x] = a;
  rh[threadIdx.x] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      rl[threadIdx.x] = fmin(rl[threadIdx.x], rl[threadIdx.x + h]);
      rh[threadIdx.x] = fmax(rh[threadIdx.x], rh[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    lo[(int64_t)blockIdx.x * d + c] = rl[0];
    hi[(int64_t)blockIdx.x * d + c] = rh[0];
  }
}

void bounding_box(const double* X, int64_t n, int d, double* lo_host, double* hi_host, hipStream_t s) {
  const int64_t ns = ceil_div(n, kBoxRows);
  DevBuf<double> lo(ns * d, s), hi(ns * d, s);
  hipLaunchKernelGGL(k_bbox, dim3((unsigned)ns, (unsigned)d), dim3(256), 0, s, X, n, d, lo.p, hi.p);
  KRR_LAUNCH_CHECK();
  std::vector<double> l(ns * d), h(ns * d);
  KRR_CHECK_HIP(hipMemcpyAsync(l.data(), lo.p, sizeof(double) * ns * d, hipMemcpyDeviceToHost, s));
  KRR_CHECK_HIP(hipMemcpyAsync(h.data(), hi.p, sizeof(double) * ns * d, hipMemcpyDeviceToHost, s));
  KRR_CHECK_HIP(hipStreamSynchronize(s));
  for (int c = 0; c < d; ++c) {
    double a = INFINITY, b = -INFINITY;
    for (int64_t t = 0; t < ns; ++t) {
      a = std::min(a, l[t * d + c]);
      b = std::max(b, h[t * d + c]);
    }
    lo_host[c] = a;
    hi_host[c] = b;
  }
}

}  // namespace krr

// ================================================================== C ABI
namespace krr {
void validate_common(int64_t m, int64_t n, int32_t d, double eps);
}

extern "C" int krr_fps(const double* X, int64_t n, int32_t d, int32_t k, int64_t start, int64_t* S, double* dsel,
                       void* stream) {
  return krr::guarded([&] {
    krr::validate_common(n, n, d, 1.0);
    KRR_REQUIRE(X && S, "null pointer argument");
    KRR_REQUIRE(k >= 1 && k <= n, "need 1 <= k <= n");
    KRR_REQUIRE(start >= 0 && start < n, "start must be in [0, n)");
    hipStream_t s = (hipStream_t)stream;
    krr::check_finite_device(X, n * (int64_t)d, "X", s);
    krr::fps_select(X, n, d, k, start, S, dsel, s);
    return (int)KRR_OK;
  });
}

extern "C" int krr_rank_for_cond(const double* X, int64_t n, int32_t d, double eps, double beta, double xi,
                                 double Mbar, double* gamma, double* k_bound, double* q_host, void* stream) {
  return krr::guarded([&] {
    krr::validate_common(n, n, d, eps);
    KRR_REQUIRE(X && gamma && k_bound, "null pointer argument");
    KRR_REQUIRE(beta > 0 && std::isfinite(beta), "beta must be positive and finite");
    KRR_REQUIRE(xi > 1 && std::isfinite(xi), "xi must be finite and > 1");
    const double Mb = Mbar > 0 ? Mbar : (double)n;
    KRR_REQUIRE(std::isfinite(Mb), "Mbar must be finite");
    const double arg = Mb * (double)n / (beta * (xi - 1.0));
    KRR_REQUIRE(arg > 1.0, "Mbar n / (beta (xi - 1)) must exceed 1 (delta < 1)");
    hipStream_t s = (hipStream_t)stream;
    krr::check_finite_device(X, n * (int64_t)d, "X", s);
    std::vector<double> lo(d), hi(d);
    krr::bounding_box(X, n, d, lo.data(), hi.data(), s);
    // Eq. condbound_gamma with h = sqrt(eps), evaluated in this order: h^{-2} ln(arg), root, 2/pi factor
    const double h = std::sqrt(eps);
    const double g = (2.0 / M_PI) * std::sqrt(std::pow(h, -2.0) * std::log(arg));
    double k = 1.0;
    for (int c = 0; c < d; ++c) {
      const double q = hi[c] - lo[c];
      if (q_host) q_host[c] = q;
      k *= std::floor(g * q) + 1.0;
    }
    *gamma = g;
    *k_bound = k;
    return (int)KRR_OK;
  });
}
