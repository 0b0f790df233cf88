// ID / Nystrom / Woodbury preconditioner (Sec. 3): build (Algorithms 1-3) and apply (Algorithm 4),
// plus the C ABI entry points krr_sketch, krr_qrcp, krr_build_precond and the handle accessors.
//
// Build, all on the device:
//   sketch Y (Algorithm 1: K Omega^T through the kernel MVM; Algorithm 2: sparse sketch kernel)
//   -> pivoted QR of Y^T -> anchors S (first k pivots)
//   -> K_SS = U^{-1} -> one-sided Jacobi EVD -> drop eigenvalues <= tau * max
//   -> C = K(X, X_S) -> W = C V_kept diag(lam_kept)^{-1/2}  (so W W^T = C U C^T)
//   -> M = W^T W (FP64) -> per beta: Cholesky L L^T = beta I + M (Eq. chol_factor), L^{-1},
//      G = (beta I + M)^{-1} = L^{-T} L^{-1}.
// For FP32/mixed handles W is also rounded to FP32 and a second core is built from exactly that
// rounded copy, so the applied operator is the Woodbury inverse of W32 W32^T + beta I.
// W = K(X, X_S) T is formed on the FP64 matrix cores without storing C (the kernel block is evaluated
// inside the product); M = W^T W, G = L^{-T} L^{-1} and the several-column Woodbury products are the
// library's own FP64 matrix-core GEMMs (gemm.hip).
#include <algorithm>
#include <cstdlib>
#include <chrono>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>

#include "anchors.h"
#include "dense.h"
#include "gemm.h"
#include "kmv.h"
#include "precond.h"
#include "sketch_qrcp.h"

namespace krr {

void validate_common(int64_t m, int64_t n, int32_t d, double eps);
void validate_prec(int32_t prec);
void kernel_mv_raw(const double* Xt, int64_t m, const double* Xs, int64_t n, int d, double eps, const double* V,
                   int R, const double* shift, int deriv, int prec, double* U, int64_t ldu, hipStream_t s);

// ------------------------------------------------------------------ small kernels
// T (k x kept, row-major) = V_kept diag(lam_kept)^{-1/2}; V column-major (eigenvector j at V + j k)
__global__ void k_make_T(const double* __restrict__ V, const double* __restrict__ lam, const int* __restrict__ idx,
                         int k, int kept, double* __restrict__ T) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)k * kept) return;
  const int r = (int)(t / kept), c = (int)(t % kept);
  const int j = idx[c];
  T[t] = V[(int64_t)j * k + r] / sqrt(lam[j]);
}

// out (row-major) = in (column-major) for a k x k matrix: out[r * k + c] = in[c * k + r]
__global__ void k_colmajor_to_rowmajor(const double* __restrict__ in, int k, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)k * k) return;
  const int r = (int)(t / k), c = (int)(t % k);
  out[t] = in[(int64_t)c * k + r];
}

__global__ void k_to_f32(const double* __restrict__ a, int64_t n, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}
__global__ void k_add_diag(const double* __restrict__ M, int k, double beta, double* __restrict__ A) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)k * k) return;
  A[t] = M[t] + ((t % k) == (t / k) ? beta : 0.0);
}

static unsigned nblk(int64_t n, int b = 256) { return (unsigned)ceil_div(n, b); }

// ------------------------------------------------------------------ Woodbury apply kernels (one column)
constexpr int kWRows = 256;   // rows per block in the W^T x pass (at most)

// Rows per block of the W^T x pass: kWRows, fewer for small n so that the pass still has a few hundred blocks
// (a multiple of 4, at least 16).
static int wt_rows(int64_t n) {
  return (int)std::min<int64_t>(kWRows, std::max<int64_t>(16, round_up(ceil_div(n, 256), 4)));
}

// partial[b, c] = sum_{i in row block b} W[i, c] x[i]  (products and sums in FP64; W read once).
// Grid: row blocks x column chunks of 256, so that the pass has several blocks per CU at n ~ 1e5.
template <typename TW>
__global__ __launch_bounds__(256) void k_wt_partial(const TW* __restrict__ W, int64_t n, int kept,
                                                    const double* __restrict__ x, int ldx, int rows,
                                                    double* __restrict__ partial) {
  const int64_t i0 = (int64_t)blockIdx.x * rows;
  const int64_t i1 = i0 + rows < n ? i0 + rows : n;
  const int c = blockIdx.y * 256 + threadIdx.x;
  if (c >= kept) return;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t i = i0;
  for (; i + 4 <= i1; i += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = __builtin_fma((double)W[(i + u) * kept + c], x[(i + u) * ldx], acc[u]);
  }
  for (; i < i1; ++i) acc[0] = __builtin_fma((double)W[i * kept + c], x[i * ldx], acc[0]);
  partial[(int64_t)blockIdx.x * kept + c] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// t[c] = sum_b partial[b, c]: one block per column, strided partial sums then a fixed-order LDS tree.
__global__ __launch_bounds__(256) void k_reduce_partials(const double* __restrict__ partial, int nb, int kept,
                                                         double* __restrict__ t) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double s = 0;
  for (int b = threadIdx.x; b < nb; b += 256) s += partial[(int64_t)b * kept + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) t[c] = red[0];
}

// z[i] = sum_c G[i, c] t[c]; G symmetric, one wave per row reading row i of G contiguously.
__global__ __launch_bounds__(256) void k_sym_gemv(const double* __restrict__ G, int kept, const double* __restrict__ t,
                                                  double* __restrict__ z) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= kept) return;
  double s = 0;
#pragma unroll 16   // the row's loads in flight together; the FMA chain keeps its order
  for (int c = lane; c < kept; c += 64) s = __builtin_fma(G[(int64_t)i * kept + c], t[c], s);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) z[i] = s;
}

// out[i] = (x[i] - sum_c W[i, c] z[c]) / beta; a wave takes RW rows at a time (their loads in flight
// together), lane l sums columns l, l + 64, ... of each row, then a butterfly over the wave; z staged in LDS.
template <typename TW, int kWzRows>
__global__ __launch_bounds__(256) void k_w_z(const TW* __restrict__ W, int64_t n, int kept,
                                             const double* __restrict__ z, const double* __restrict__ x, int ldx,
                                             double inv_beta, double* __restrict__ out, int ldo) {
  extern __shared__ double zs[];
  for (int c = threadIdx.x; c < kept; c += 256) zs[c] = z[c];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * 4 * kWzRows;
  for (int64_t i0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kWzRows; i0 < n; i0 += stride) {
    double sum[kWzRows];
    const TW* wr[kWzRows];
#pragma unroll
    for (int r = 0; r < kWzRows; ++r) {
      sum[r] = 0.0;
      wr[r] = W + (i0 + r < n ? i0 + r : n - 1) * kept;
    }
#pragma unroll 4
    for (int c = lane; c < kept; c += 64) {
      const double zc = zs[c];
#pragma unroll
      for (int r = 0; r < kWzRows; ++r) sum[r] = __builtin_fma((double)wr[r][c], zc, sum[r]);
    }
#pragma unroll
    for (int r = 0; r < kWzRows; ++r)
      for (int o = 32; o > 0; o >>= 1) sum[r] += __shfl_xor(sum[r], o);
#pragma unroll
    for (int r = 0; r < kWzRows; ++r)
      if (lane == r && i0 + r < n) out[(i0 + r) * ldo] = (x[(i0 + r) * ldx] - sum[r]) * inv_beta;
  }
}

// ------------------------------------------------------------------ block (R > 1) helpers
// Z[c, r] = Zall[bidx[r]][c, r]  (kept x R row-major blocks, one per beta)
__global__ void k_select_z(const double* __restrict__ Zall, int kept, int R, const int* __restrict__ bidx,
                           double* __restrict__ Z) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)kept * R) return;
  const int r = (int)(t % R);
  Z[t] = Zall[(int64_t)bidx[r] * kept * R + t];
}

int beta_index(const krr_precond& P, double beta) {
  for (size_t i = 0; i < P.betas.size(); ++i)
    if (P.betas[i] == beta) return (int)i;
  return -1;
}

// One column of Algorithm 4 with caller-provided buffers: x and out are columns of n x R row-major blocks
// (strides ldx, ldo); partial holds ceil(n / wt_rows(n)) x kept doubles (at most max(256, ceil(n / 256)) x kept),
// t and z kept doubles each.  Every slot of
// partial is written before it is read, so the buffers need no clearing.
static void woodbury_one_column(const krr_precond& P, const double* x, int ldx, int b, bool use32, double* out,
                                int ldo, double* partial, double* t, double* z, hipStream_t s) {
  const int kept = P.kept;
  const int64_t n = P.n;
  const double* G = use32 ? P.G32[b].p : P.G64[b].p;
  const int rows = wt_rows(n);
  const int nb = (int)ceil_div(n, rows);
  const dim3 gw((unsigned)nb, nblk(kept));
  if (use32)
    hipLaunchKernelGGL(k_wt_partial<float>, gw, dim3(256), 0, s, P.W32.p, n, kept, x, ldx, rows, partial);
  else
    hipLaunchKernelGGL(k_wt_partial<double>, gw, dim3(256), 0, s, P.W64.p, n, kept, x, ldx, rows, partial);
  hipLaunchKernelGGL(k_reduce_partials, dim3((unsigned)kept), dim3(256), 0, s, partial, nb, kept, t);
  hipLaunchKernelGGL(k_sym_gemv, dim3(nblk(kept, 4)), dim3(256), 0, s, G, kept, t, z);
  // two rows per wave and at most 2048 blocks (measured best among 1, 2, 4 rows and 1024-8192 blocks)
  const unsigned g = (unsigned)std::min<int64_t>(ceil_div(n, 8), 2048);
  const size_t lds = (size_t)kept * sizeof(double);
  if (use32)
    hipLaunchKernelGGL((k_w_z<float, 2>), dim3(g), dim3(256), lds, s, P.W32.p, n, kept, z, x, ldx,
                       1.0 / P.betas[b], out, ldo);
  else
    hipLaunchKernelGGL((k_w_z<double, 2>), dim3(g), dim3(256), lds, s, P.W64.p, n, kept, z, x, ldx,
                       1.0 / P.betas[b], out, ldo);
  KRR_LAUNCH_CHECK();
}

// Doubles of scratch one column of woodbury_one_column needs.
static int64_t woodbury_column_scratch(const krr_precond& P) {
  return ceil_div(P.n, wt_rows(P.n)) * (int64_t)P.kept + 2 * (int64_t)P.kept;
}

void WoodburyWork::prepare(const krr_precond& P, int R_, const int* bidx_host_, hipStream_t s) {
  R = R_;
  bidx_host.assign(bidx_host_, bidx_host_ + R);
  const int kept = P.kept;
  if (R == 1) {
    partial.alloc((size_t)ceil_div(P.n, wt_rows(P.n)) * kept, s);
    t.alloc(kept, s);
    z.alloc(kept, s);
    return;
  }
  const int nbeta = (int)P.betas.size();
  std::vector<double> ib(R);
  for (int r = 0; r < R; ++r) ib[r] = 1.0 / P.betas[bidx_host[r]];
  invb.alloc(R, s);
  bidx.alloc(R, s);
  KRR_CHECK_HIP(hipMemcpyAsync(invb.p, ib.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
  KRR_CHECK_HIP(hipMemcpyAsync(bidx.p, bidx_host.data(), sizeof(int) * R, hipMemcpyHostToDevice, s));
  KRR_CHECK_HIP(hipStreamSynchronize(s));   // the host vectors above are temporaries
  T.alloc((size_t)kept * R, s);
  Zall.alloc((size_t)nbeta * kept * R, s);
  Z.alloc((size_t)kept * R, s);
}

void woodbury_apply(const krr_precond& P, const double* x, WoodburyWork& w, bool use32, double* out,
                    hipStream_t s) {
  const int kept = P.kept;
  const int64_t n = P.n;
  const int R = w.R;
  KRR_REQUIRE(!use32 || P.W32.p, "preconditioner was built without an FP32 factor");
  if (R == 1) {
    woodbury_one_column(P, x, 1, w.bidx_host[0], use32, out, 1, w.partial.p, w.t.p, w.z.p, s);
    return;
  }
  // Block form (FP64 matrix cores; the FP32 factor's products are exact in FP64): T = W^T X, summed over row
  // splits in a fixed order; Z_b = G_b T for each beta; column r takes Z_{beta_r}; out = (X - W Z) diag(1/beta).
  const int nbeta = (int)P.betas.size();
  if (use32) gemm_tn<float, double>(P.W32.p, kept, x, R, n, kept, R, w.T.p, R, s, &w.tn);
  else gemm_tn<double, double>(P.W64.p, kept, x, R, n, kept, R, w.T.p, R, s, &w.tn);
  for (int b = 0; b < nbeta; ++b) {
    const double* G = use32 ? P.G32[b].p : P.G64[b].p;
    gemm_nn<double>(G, kept, w.T.p, R, kept, kept, R, w.Zall.p + (int64_t)b * kept * R, R, nullptr, 0, nullptr, s);
  }
  hipLaunchKernelGGL(k_select_z, dim3(nblk((int64_t)kept * R)), dim3(256), 0, s, w.Zall.p, kept, R, w.bidx.p, w.Z.p);
  KRR_LAUNCH_CHECK();
  if (use32) gemm_nn<float>(P.W32.p, kept, w.Z.p, R, n, kept, R, out, R, x, R, w.invb.p, s);
  else gemm_nn<double>(P.W64.p, kept, w.Z.p, R, n, kept, R, out, R, x, R, w.invb.p, s);
}

void woodbury_apply(const krr_precond& P, const double* x, int R, const int* bidx_host, bool use32, double* out,
                    hipStream_t s) {
  WoodburyWork w;
  w.prepare(P, R, bidx_host, s);
  woodbury_apply(P, x, w, use32, out, s);
}

// ------------------------------------------------------------------ build
static double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

static void validate_sketch_inputs(const double* omega, const int64_t* idx, const double* sign, int64_t n, int l,
                                   int r, hipStream_t s) {
  KRR_REQUIRE((omega != nullptr) != (idx != nullptr), "give exactly one of omega (Algorithm 1) or idx/sign (Algorithm 2)");
  if (idx) {
    KRR_REQUIRE(sign != nullptr, "sign is required with idx");
    KRR_REQUIRE(r >= 1, "r must be >= 1 for the sparse sketch");
    std::vector<int64_t> h((size_t)l * r);
    KRR_CHECK_HIP(hipMemcpyAsync(h.data(), idx, sizeof(int64_t) * h.size(), hipMemcpyDeviceToHost, s));
    KRR_CHECK_HIP(hipStreamSynchronize(s));
    for (int64_t v : h) KRR_REQUIRE(v >= 0 && v < n, "sketch index out of range [0, n)");
    check_finite_device(sign, (int64_t)l * r, "sign", s);
  } else {
    check_finite_device(omega, n * (int64_t)l, "omega", s);
  }
}

// Sketch into Yt (l x ldy) in the working precision wprec (FP64 or FP32).
// Algorithm 1 sketch Y = K Omega^T (omega and Y n x l row-major), in column chunks of at most 256
// (the widest block product).
void sketch_dense(const double* X, int64_t n, int d, double eps, const double* omega, int l, int prec, double* Y,
                  hipStream_t s) {
  constexpr int kChunk = 256;
  DevBuf<double> Oc(l > kChunk ? (size_t)n * kChunk : 0, s);
  for (int c0 = 0; c0 < l; c0 += kChunk) {
    const int rc = std::min(kChunk, l - c0);
    const double* V = omega;
    if (l > kChunk) {
      KRR_CHECK_HIP(hipMemcpy2DAsync(Oc.p, sizeof(double) * rc, omega + c0, sizeof(double) * l, sizeof(double) * rc,
                                     (size_t)n, hipMemcpyDeviceToDevice, s));
      V = Oc.p;
    }
    kernel_mv_raw(X, n, X, n, d, eps, V, rc, nullptr, 0, prec, Y + c0, l, s);
  }
}

static void make_sketch_t(const double* X, int64_t n, int d, double eps, const double* omega, const int64_t* idx,
                          const double* sign, int l, int r, int prec, int wprec, void* Yt, int64_t ldy,
                          double* keepY, hipStream_t s) {
  if (omega) {
    DevBuf<double> Y(n * l, s);
    sketch_dense(X, n, d, eps, omega, l, prec, Y.p, s);
    transpose_to_t(Y.p, n, l, wprec, Yt, ldy, s);
    if (keepY) KRR_CHECK_HIP(hipMemcpyAsync(keepY, Y.p, sizeof(double) * n * l, hipMemcpyDeviceToDevice, s));
  } else {
    sketch_sparse_t(X, n, d, eps, idx, sign, l, r, wprec, Yt, ldy, s);
    if (keepY) transpose_from_t(Yt, ldy, n, l, wprec, keepY, s);
  }
}

static void build_core(krr_precond& P, const double* M, std::vector<DevBuf<double>>& G,
                       std::vector<DevBuf<double>>* Ls, hipStream_t s) {
  const int kept = P.kept;
  const int64_t kk = (int64_t)kept * kept;
  for (double beta : P.betas) {
    DevBuf<double> A(kk, s), L(kk, s), Li(kk, s), Gb(kk, s);
    hipLaunchKernelGGL(k_add_diag, dim3(nblk(kk)), dim3(256), 0, s, M, kept, beta, A.p);
    KRR_LAUNCH_CHECK();
    const int info = cholesky_lower(A.p, L.p, kept, s);
    if (info != 0)
      throw Error{KRR_ENOTSPD, "Cholesky of beta I + W^T W failed at column " + std::to_string(info - 1) +
                                   " (beta = " + std::to_string(beta) + ")"};
    lower_inverse(L.p, Li.p, kept, s);
    // G = L^{-T} L^{-1} = A^T A with A = L^{-1} row-major (lower_inverse writes it column-major)
    hipLaunchKernelGGL(k_colmajor_to_rowmajor, dim3(nblk(kk)), dim3(256), 0, s, Li.p, kept, A.p);
    KRR_LAUNCH_CHECK();
    syrk_tn<double>(A.p, kept, kept, kept, Gb.p, kept, s);
    G.push_back(std::move(Gb));
    if (Ls) Ls->push_back(std::move(L));
  }
}

void build_from_anchors(krr_precond& P, const double* X, hipStream_t s);

void build_precond(krr_precond& P, const double* X, const double* omega, const int64_t* idx, const double* sign,
                   int flags, hipStream_t s) {
  using clk = std::chrono::steady_clock;
  const auto t_all = clk::now();
  const int64_t n = P.n;
  const int d = P.d, k = P.k, l = P.l;
  const int wprec = P.prec == KRR_FP64 ? KRR_FP64 : KRR_FP32;
  const size_t esz = wprec == KRR_FP64 ? sizeof(double) : sizeof(float);
  // 1. sketch (Algorithm 1 / 2)
  auto t0 = clk::now();
  const int64_t ldy = round_up(n, 256);
  DevBuf<char> Yt((size_t)l * ldy * esz, s);
  if (flags & KRR_KEEP_SKETCH) P.Ysk.alloc(n * l, s);
  make_sketch_t(X, n, d, P.eps, omega, idx, sign, l, P.r, P.prec, wprec, Yt.p, ldy,
                (flags & KRR_KEEP_SKETCH) ? P.Ysk.p : nullptr, s);
  KRR_CHECK_HIP(hipStreamSynchronize(s));
  P.t_build_ms[0] = ms_since(t0);
  // 2. pivoted QR of Y^T -> S
  t0 = clk::now();
  P.S.alloc(k, s);
  DevBuf<double> rdiag(k, s);
  qrcp_t(Yt.p, ldy, n, l, k, wprec, P.S.p, rdiag.p, s);
  Yt.release();
  P.S_host.resize(k);
  P.rdiag_host.resize(k);
  KRR_CHECK_HIP(hipMemcpyAsync(P.S_host.data(), P.S.p, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s));
  KRR_CHECK_HIP(hipMemcpyAsync(P.rdiag_host.data(), rdiag.p, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  KRR_CHECK_HIP(hipStreamSynchronize(s));
  P.t_build_ms[1] = ms_since(t0);
  build_from_anchors(P, X, s);
  P.t_build_ms[5] = ms_since(t_all);
}

// Algorithm 3 and the core factors for the anchors in P.S (device) / P.S_host: fills phases 2-4.
void build_from_anchors(krr_precond& P, const double* X, hipStream_t s) {
  using clk = std::chrono::steady_clock;
  const int64_t n = P.n;
  const int d = P.d, k = P.k;
  // 3. K_SS = U^{-1}, EVD, truncation
  auto t0 = clk::now();
  DevBuf<double> XS((size_t)k * d, s), Kss((size_t)k * k, s), V((size_t)k * k, s), lam(k, s);
  gather_rows(X, n, d, P.S.p, k, XS.p, s);
  kernel_block_colmajor(XS.p, k, XS.p, k, d, P.eps, Kss.p, k, s);
  P.jacobi_sweeps = jacobi_evd(Kss.p, V.p, lam.p, k, s);
  std::vector<double> lh(k);
  KRR_CHECK_HIP(hipMemcpyAsync(lh.data(), lam.p, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  KRR_CHECK_HIP(hipStreamSynchronize(s));
  const double lmax = *std::max_element(lh.begin(), lh.end());
  KRR_REQUIRE(lmax > 0 && std::isfinite(lmax), "anchor kernel block has no positive eigenvalue");
  std::vector<int> keep;
  for (int i = 0; i < k; ++i)
    if (lh[i] > P.tau * lmax) keep.push_back(i);
  P.kept = (int)keep.size();
  P.lam_host = lh;
  std::sort(P.lam_host.begin(), P.lam_host.end());
  DevBuf<int> keep_d(P.kept, s);
  KRR_CHECK_HIP(hipMemcpyAsync(keep_d.p, keep.data(), sizeof(int) * P.kept, hipMemcpyHostToDevice, s));
  DevBuf<double> T((size_t)k * P.kept, s);
  hipLaunchKernelGGL(k_make_T, dim3(nblk((int64_t)k * P.kept)), dim3(256), 0, s, V.p, lam.p, keep_d.p, k, P.kept,
                     T.p);
  KRR_LAUNCH_CHECK();
  KRR_CHECK_HIP(hipStreamSynchronize(s));
  P.t_build_ms[2] = ms_since(t0);
  // 4. W = K(X, X_S) T (= C V_kept diag(lam_kept)^{-1/2}, C never stored), M = W^T W
  t0 = clk::now();
  const int kept = P.kept;
  P.W64.alloc(n * kept, s);
  if (!kernel_times_matrix_f64(X, n, XS.p, k, d, P.eps, T.p, kept, kept, P.W64.p, kept, s)) {
    // widths above the FP64 matrix-core kernel's: the kernel block C is formed, then W = C T
    DevBuf<double> C(n * k, s);
    kernel_block_rowmajor(X, n, XS.p, k, d, P.eps, C.p, k, s);
    gemm_nn<double>(C.p, k, T.p, kept, n, k, kept, P.W64.p, kept, nullptr, 0, nullptr, s);
  }
  P.M64.alloc((size_t)kept * kept, s);
  syrk_tn<double>(P.W64.p, kept, n, kept, P.M64.p, kept, s);
  if (P.prec != KRR_FP64) {
    // the FP32 copy of W and a core built from exactly that copy (its products are exact in FP64)
    P.W32.alloc(n * kept, s);
    hipLaunchKernelGGL(k_to_f32, dim3(nblk(n * kept)), dim3(256), 0, s, P.W64.p, n * kept, P.W32.p);
    KRR_LAUNCH_CHECK();
    P.M32.alloc((size_t)kept * kept, s);
    syrk_tn<float>(P.W32.p, kept, n, kept, P.M32.p, kept, s);
  }
  KRR_CHECK_HIP(hipStreamSynchronize(s));
  P.t_build_ms[3] = ms_since(t0);
  // 5. per-beta core factors
  t0 = clk::now();
  build_core(P, P.M64.p, P.G64, &P.L64, s);
  if (P.prec != KRR_FP64) build_core(P, P.M32.p, P.G32, nullptr, s);
  KRR_CHECK_HIP(hipStreamSynchronize(s));
  P.t_build_ms[4] = ms_since(t0);
}

}  // namespace krr

namespace krr {
void* noalloc_scratch();
}

// ================================================================== C ABI
extern "C" int krr_init(void* stream) {
  return krr::guarded([&] {
    hipStream_t s = (hipStream_t)stream;
    // one tiny call of each dense product the build and the block Woodbury apply use (loads their code objects)
    krr::DevBuf<double> a(64, s), c(64, s);
    krr::DevBuf<float> af(64, s);
    KRR_CHECK_HIP(hipMemsetAsync(a.p, 0, 64 * sizeof(double), s));
    KRR_CHECK_HIP(hipMemsetAsync(af.p, 0, 64 * sizeof(float), s));
    krr::syrk_tn<double>(a.p, 8, 8, 8, c.p, 8, s);
    krr::syrk_tn<float>(af.p, 8, 8, 8, c.p, 8, s);
    krr::gemm_tn<float, double>(af.p, 8, a.p, 8, 8, 8, 8, c.p, 8, s);
    krr::gemm_nn<double>(a.p, 8, a.p, 8, 8, 8, 8, c.p, 8, nullptr, 0, nullptr, s);
    KRR_CHECK_HIP(hipStreamSynchronize(s));
    (void)krr::noalloc_scratch();   // this device's address of the no-allocation entry point's scratch
    return (int)KRR_OK;
  });
}

extern "C" int krr_sketch(const double* X, int64_t n, int32_t d, double eps, const double* omega, const int64_t* idx,
                          const double* sign, int32_t l, int32_t r, int32_t prec, double* Y, void* stream) {
  return krr::guarded([&] {
    krr::validate_common(n, n, d, eps);
    krr::validate_prec(prec);
    KRR_REQUIRE(X && Y, "null pointer argument");
    KRR_REQUIRE(l >= 1 && l <= 65535, "l must be in [1, 65535]");
    hipStream_t s = (hipStream_t)stream;
    krr::validate_sketch_inputs(omega, idx, sign, n, l, r, s);
    if (omega) {
      krr::sketch_dense(X, n, d, eps, omega, l, prec, Y, s);
    } else {
      const int wprec = prec == KRR_FP64 ? KRR_FP64 : KRR_FP32;
      const int64_t ldy = krr::round_up(n, 256);
      krr::DevBuf<char> Yt((size_t)l * ldy * (wprec == KRR_FP64 ? 8 : 4), s);
      krr::sketch_sparse_t(X, n, d, eps, idx, sign, l, r, wprec, Yt.p, ldy, s);
      krr::transpose_from_t(Yt.p, ldy, n, l, wprec, Y, s);
    }
    return (int)KRR_OK;
  });
}

extern "C" int krr_qrcp(const double* Y, int64_t n, int32_t l, int32_t k, int32_t prec, int64_t* piv, double* rdiag,
                        void* stream) {
  return krr::guarded([&] {
    krr::validate_prec(prec);
    KRR_REQUIRE(Y && piv && rdiag, "null pointer argument");
    KRR_REQUIRE(n >= 1 && l >= 1 && k >= 1 && k <= l && k <= n, "need 1 <= k <= l and k <= n");
    hipStream_t s = (hipStream_t)stream;
    const int wprec = prec == KRR_FP64 ? KRR_FP64 : KRR_FP32;
    const int64_t ldy = krr::round_up(n, 256);
    krr::DevBuf<char> Yt((size_t)l * ldy * (wprec == KRR_FP64 ? 8 : 4), s);
    krr::transpose_to_t(Y, n, l, wprec, Yt.p, ldy, s);
    krr::qrcp_t(Yt.p, ldy, n, l, k, wprec, piv, rdiag, s);
    return (int)KRR_OK;
  });
}

extern "C" int krr_build_precond(const double* X, int64_t n, int32_t d, double eps, const double* betas,
                                 int32_t nbeta, int32_t k, int32_t l, const double* omega, const int64_t* idx,
                                 const double* sign, int32_t r, double tau, int32_t prec, int32_t flags,
                                 krr_precond** out, void* stream) {
  return krr::guarded([&] {
    KRR_REQUIRE(out != nullptr, "out must not be NULL");
    *out = nullptr;
    krr::validate_common(n, n, d, eps);
    krr::validate_prec(prec);
    KRR_REQUIRE(X && betas, "null pointer argument");
    KRR_REQUIRE(nbeta >= 1 && nbeta <= 64, "nbeta must be in [1, 64]");
    for (int i = 0; i < nbeta; ++i) KRR_REQUIRE(betas[i] > 0 && std::isfinite(betas[i]), "beta must be positive and finite");
    KRR_REQUIRE(k >= 1 && k <= l && l <= n, "need 1 <= k <= l <= n");
    KRR_REQUIRE(l <= 65535, "l must be <= 65535");
    KRR_REQUIRE((size_t)k * sizeof(double) <= 160 * 1024, "k too large (at most 20480)");
    hipStream_t s = (hipStream_t)stream;
    krr::check_finite_device(X, n * (int64_t)d, "X", s);
    krr::validate_sketch_inputs(omega, idx, sign, n, l, r, s);
    auto P = std::make_unique<krr_precond>();
    P->n = n; P->d = d; P->k = k; P->l = l; P->r = omega ? 0 : r; P->eps = eps; P->prec = prec;
    P->tau = tau > 0 ? tau : 1e-12;
    P->betas.assign(betas, betas + nbeta);
    krr::build_precond(*P, X, omega, idx, sign, flags, s);
    *out = P.release();
    return (int)KRR_OK;
  });
}

extern "C" int krr_build_precond_anchors(const double* X, int64_t n, int32_t d, double eps, const double* betas,
                                         int32_t nbeta, const int64_t* S, int32_t k, int64_t fps_start, double tau,
                                         int32_t prec, krr_precond** out, void* stream) {
  return krr::guarded([&] {
    KRR_REQUIRE(out != nullptr, "out must not be NULL");
    *out = nullptr;
    krr::validate_common(n, n, d, eps);
    krr::validate_prec(prec);
    KRR_REQUIRE(X && betas, "null pointer argument");
    KRR_REQUIRE(nbeta >= 1 && nbeta <= 64, "nbeta must be in [1, 64]");
    for (int i = 0; i < nbeta; ++i) KRR_REQUIRE(betas[i] > 0 && std::isfinite(betas[i]), "beta must be positive and finite");
    KRR_REQUIRE(k >= 1 && k <= n, "need 1 <= k <= n");
    KRR_REQUIRE((size_t)k * sizeof(double) <= 160 * 1024, "k too large (at most 20480)");
    KRR_REQUIRE(S != nullptr || (fps_start >= 0 && fps_start < n), "fps_start must be in [0, n)");
    hipStream_t s = (hipStream_t)stream;
    krr::check_finite_device(X, n * (int64_t)d, "X", s);
    using clk = std::chrono::steady_clock;
    const auto t_all = clk::now();
    auto P = std::make_unique<krr_precond>();
    P->n = n; P->d = d; P->k = k; P->l = 0; P->r = 0; P->eps = eps; P->prec = prec;
    P->tau = tau > 0 ? tau : 1e-12;
    P->betas.assign(betas, betas + nbeta);
    P->S.alloc(k, s);
    P->S_host.resize(k);
    P->rdiag_host.assign(k, 0.0);
    const auto t0 = clk::now();
    if (S) {
      KRR_CHECK_HIP(hipMemcpyAsync(P->S_host.data(), S, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s));
      KRR_CHECK_HIP(hipStreamSynchronize(s));
      std::vector<int64_t> srt(P->S_host);
      std::sort(srt.begin(), srt.end());
      KRR_REQUIRE(srt.front() >= 0 && srt.back() < n, "anchor index out of range");
      KRR_REQUIRE(std::adjacent_find(srt.begin(), srt.end()) == srt.end(), "anchor indices must be distinct");
      KRR_CHECK_HIP(hipMemcpyAsync(P->S.p, S, sizeof(int64_t) * k, hipMemcpyDeviceToDevice, s));
    } else {
      krr::fps_select(X, n, d, k, fps_start, P->S.p, nullptr, s);
      KRR_CHECK_HIP(hipMemcpyAsync(P->S_host.data(), P->S.p, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s));
    }
    KRR_CHECK_HIP(hipStreamSynchronize(s));
    P->t_build_ms[1] = krr::ms_since(t0);
    krr::build_from_anchors(*P, X, s);
    P->t_build_ms[5] = krr::ms_since(t_all);
    *out = P.release();
    return (int)KRR_OK;
  });
}

extern "C" int krr_precond_info(const krr_precond* P, int64_t* S_host, int32_t* kept, double* lam_host,
                                double* rdiag_host, int32_t* k, int32_t* nbeta) {
  return krr::guarded([&] {
    KRR_REQUIRE(P != nullptr, "null handle");
    if (S_host) std::copy(P->S_host.begin(), P->S_host.end(), S_host);
    if (kept) *kept = P->kept;
    if (lam_host) std::copy(P->lam_host.begin(), P->lam_host.end(), lam_host);
    if (rdiag_host) std::copy(P->rdiag_host.begin(), P->rdiag_host.end(), rdiag_host);
    if (k) *k = P->k;
    if (nbeta) *nbeta = (int32_t)P->betas.size();
    return (int)KRR_OK;
  });
}

extern "C" int krr_precond_timings(const krr_precond* P, double* ms, int32_t* sweeps) {
  return krr::guarded([&] {
    KRR_REQUIRE(P != nullptr && ms != nullptr, "null argument");
    for (int i = 0; i < 6; ++i) ms[i] = P->t_build_ms[i];
    if (sweeps) *sweeps = P->jacobi_sweeps;
    return (int)KRR_OK;
  });
}

extern "C" int krr_precond_get(const krr_precond* P, int32_t what, int32_t bidx, void* dst, size_t bytes,
                               void* stream) {
  return krr::guarded([&] {
    KRR_REQUIRE(P != nullptr && dst != nullptr, "null argument");
    hipStream_t s = (hipStream_t)stream;
    const void* src = nullptr;
    size_t need = 0;
    const size_t kk = (size_t)P->kept * P->kept;
    switch (what) {
      case 0: src = P->W64.p; need = P->W64.bytes(); break;
      case 1: src = P->W32.p; need = P->W32.bytes(); break;
      case 2:
        KRR_REQUIRE(bidx >= 0 && bidx < (int)P->L64.size(), "beta index out of range");
        src = P->L64[bidx].p; need = kk * sizeof(double); break;
      case 3: src = P->Ysk.p; need = P->Ysk.bytes(); break;
      case 4: src = P->M64.p; need = P->M64.bytes(); break;
      default: KRR_REQUIRE(false, "unknown buffer id");
    }
    KRR_REQUIRE(src != nullptr, "buffer not present in this handle");
    KRR_REQUIRE(bytes >= need, "destination too small");
    KRR_CHECK_HIP(hipMemcpyAsync(dst, src, need, hipMemcpyDeviceToDevice, s));
    return (int)KRR_OK;
  });
}

extern "C" int krr_precond_apply(const krr_precond* P, const double* x, int32_t R, const double* betas, int32_t prec,
                                 double* out, void* stream) {
  return krr::guarded([&] {
    KRR_REQUIRE(P && x && out && betas, "null argument");
    krr::validate_prec(prec);
    KRR_REQUIRE(R >= 1 && R <= 4096, "R must be in [1, 4096]");
    std::vector<int> bidx(R);
    for (int r = 0; r < R; ++r) {
      bidx[r] = krr::beta_index(*P, betas[r]);
      KRR_REQUIRE(bidx[r] >= 0, "beta not among the preconditioner's betas");
    }
    krr::woodbury_apply(*P, x, R, bidx.data(), prec != KRR_FP64, out, (hipStream_t)stream);
    return (int)KRR_OK;
  });
}

// ------------------------------------------------------------------ apply without device allocation
// For callers that cannot allocate device memory (HIP graph capture, serving loops): the Woodbury apply
// one column at a time with its scratch (the W^T x partial sums, t and z) in a file-scope device array.
// Every GPU the library runs on holds its own copy until the process ends; its address is looked up once
// per device (hipGetSymbolAddress) and only that address is passed to kernels.  Calls that overlap on one
// GPU share the array and race.
namespace krr {
namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) char scratch[kScratchBytes];
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device ordinal -> address of that device's copy of `scratch`
}  // namespace

// Address of this device's scratch array (looked up once per device with that device current).
void* noalloc_scratch() {
  int dev = 0;
  KRR_CHECK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* p = nullptr;
  KRR_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  KRR_REQUIRE(p != nullptr, "hipGetSymbolAddress returned no address for the scratch array");
  g_scratch_ptr[dev] = p;
  return p;
}

size_t noalloc_scratch_bytes() { return kScratchBytes; }
}  // namespace krr

extern "C" int krr_precond_apply_noalloc(const krr_precond* P, const double* x, int32_t R, const double* betas,
                                         int32_t prec, double* out, void* stream) {
  return krr::guarded([&] {
    KRR_REQUIRE(P && x && out && betas, "null argument");
    krr::validate_prec(prec);
    KRR_REQUIRE(R >= 1 && R <= 4096, "R must be in [1, 4096]");
    const bool use32 = prec != KRR_FP64;
    KRR_REQUIRE(!use32 || P->W32.p, "preconditioner was built without an FP32 factor");
    std::vector<int> bidx(R);
    for (int r = 0; r < R; ++r) {
      bidx[r] = krr::beta_index(*P, betas[r]);
      KRR_REQUIRE(bidx[r] >= 0, "beta not among the preconditioner's betas");
    }
    const int64_t need = krr::woodbury_column_scratch(*P);
    KRR_REQUIRE((size_t)need * sizeof(double) <= krr::noalloc_scratch_bytes(),
                "krr_precond_apply_noalloc: this preconditioner needs " + std::to_string(need * 8) +
                    " bytes of scratch (ceil(n / rows) * kept + 2 * kept doubles, rows = min(256, max(16, ~n / 256))); the library's scratch holds " +
                    std::to_string(krr::noalloc_scratch_bytes()) + " bytes");
    double* base = static_cast<double*>(krr::noalloc_scratch());
    double* partial = base;
    double* t = partial + krr::ceil_div(P->n, krr::wt_rows(P->n)) * P->kept;
    double* z = t + P->kept;
    hipStream_t s = (hipStream_t)stream;
    for (int r = 0; r < R; ++r) krr::woodbury_one_column(*P, x + r, R, bidx[r], use32, out + r, R, partial, t, z, s);
    return (int)KRR_OK;
  });
}

extern "C" void krr_precond_free(krr_precond* P) { delete P; }
