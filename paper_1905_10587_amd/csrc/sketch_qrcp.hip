// Anchor selection (Sec. 3, Algorithms 1-2): the sketch Y and the column-pivoted QR of Y^T.
//
// Layout: the sketch is kept transposed, Yt = Y^T (l rows x N columns, row stride ldy = padded N),
// so that the QR's per-step pass r = q^T Yt reads each row coalesced.
//
// Pivoted QR (left-looking, classical Gram-Schmidt applied twice): with Q_j = [q_0 .. q_{j-1}]
// orthonormal (l x j, FP64) and nrm2[c] the squared residual norm of column c,
//   p      = argmax_c nrm2[c] over unselected columns (lowest index on ties)
//   w      = Yt[:, p];  w -= Q_j (Q_j^T w) twice;  q_j = w / ||w||
//   r[c]   = q_j^T Yt[:, c];  nrm2[c] -= r[c]^2 (clamped at 0)
// This selects the same pivots as Householder QR with column pivoting in exact arithmetic
// (the residual norms are those of the trailing columns), without forming R or T (Sec. 2.3:
// only the permutation is needed).
#include "kmv_kernels.h"
#include "sketch_qrcp.h"

namespace krr {

// ------------------------------------------------------------------ sparse sketch (Algorithm 2)
// Yt[i, a] = sum_s sign[i, s] k(x_a, x_{idx[i, s]}).  Block: 256 targets a (one per thread) x kSkCols
// sketch columns; the r source points of a column are wave-uniform (scalar loads).  DM is the
// compile-time bound on d (coordinates held in registers).
constexpr int kSkCols = 8;

template <int DM, bool F64>
__global__ __launch_bounds__(256) void k_sketch_sparse(const double* __restrict__ X, int64_t n, int d,
                                                       const int64_t* __restrict__ idx,
                                                       const double* __restrict__ sign, int l, int r,
                                                       double inv_eps, float scale, void* __restrict__ Ytv,
                                                       int64_t ldy) {
  const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = a < n;
  const int64_t ar = live ? a : 0;
  double xa[DM];
#pragma unroll
  for (int k = 0; k < DM; ++k) xa[k] = k < d ? X[ar * d + k] : 0.0;
  for (int ci = 0; ci < kSkCols; ++ci) {
    const int i = blockIdx.y * kSkCols + ci;
    if (i >= l) return;
    double acc = 0.0;
    float accf = 0.0f;
    for (int s = 0; s < r; ++s) {
      int64_t j = idx[(int64_t)i * r + s];
      j = j < 0 ? 0 : (j >= n ? n - 1 : j);
      const double w = sign[(int64_t)i * r + s];
      if (F64) {
        double d2 = 0.0;
#pragma unroll
        for (int k = 0; k < DM; ++k) {
          if (k < d) {
            const double df = xa[k] - X[j * d + k];
            d2 = __builtin_fma(df, df, d2);
          }
        }
        acc = __builtin_fma(w, exp_neg_f64(d2 * inv_eps), acc);
      } else {
        float d2 = 0.0f;
#pragma unroll
        for (int k = 0; k < DM; ++k) {
          if (k < d) {
            const float df = (float)(xa[k] - X[j * d + k]) * scale;   // difference taken in FP64
            d2 = __builtin_fmaf(df, df, d2);
          }
        }
        accf = __builtin_fmaf((float)w, __builtin_amdgcn_exp2f(-d2), accf);
      }
    }
    if (live) {
      if (F64) ((double*)Ytv)[(int64_t)i * ldy + a] = acc;
      else ((float*)Ytv)[(int64_t)i * ldy + a] = accf;
    }
  }
}

template <bool F64>
static void sketch_go(int dm, dim3 grid, hipStream_t s, const double* X, int64_t n, int d, const int64_t* idx,
                      const double* sign, int l, int r, double inv_eps, float scale, void* Yt, int64_t ldy) {
#define KRR_SK(DM) \
  hipLaunchKernelGGL((k_sketch_sparse<DM, F64>), grid, dim3(256), 0, s, X, n, d, idx, sign, l, r, inv_eps, scale, Yt, ldy)
  if (dm <= 4) KRR_SK(4);
  else if (dm <= 8) KRR_SK(8);
  else if (dm <= 16) KRR_SK(16);
  else if (dm <= 32) KRR_SK(32);
  else if (dm <= 64) KRR_SK(64);
  else KRR_SK(128);
#undef KRR_SK
}

void sketch_sparse_t(const double* X, int64_t n, int d, double eps, const int64_t* idx, const double* sign, int l,
                     int r, int prec, void* Yt, int64_t ldy, hipStream_t s) {
  dim3 grid((unsigned)ceil_div(n, 256), (unsigned)ceil_div(l, kSkCols));
  const float scale = (float)std::sqrt(kLog2e / eps);
  if (prec == KRR_FP64) sketch_go<true>(d, grid, s, X, n, d, idx, sign, l, r, 1.0 / eps, scale, Yt, ldy);
  else sketch_go<false>(d, grid, s, X, n, d, idx, sign, l, r, 1.0 / eps, scale, Yt, ldy);
  KRR_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ transposes
template <typename T>
__global__ void k_transpose_to(const double* __restrict__ Y, int64_t n, int l, T* __restrict__ Yt, int64_t ldy) {
  // Y n x l row-major -> Yt l x n (row stride ldy)
  __shared__ double tile[32][33];
  const int64_t a0 = (int64_t)blockIdx.x * 32;
  const int i0 = blockIdx.y * 32;
  for (int t = threadIdx.y; t < 32; t += 8) {
    const int64_t a = a0 + t;
    const int i = i0 + threadIdx.x;
    tile[t][threadIdx.x] = (a < n && i < l) ? Y[a * l + i] : 0.0;
  }
  __syncthreads();
  for (int t = threadIdx.y; t < 32; t += 8) {
    const int i = i0 + t;
    const int64_t a = a0 + threadIdx.x;
    if (i < l && a < n) Yt[(int64_t)i * ldy + a] = (T)tile[threadIdx.x][t];
  }
}

template <typename T>
__global__ void k_transpose_from(const T* __restrict__ Yt, int64_t ldy, int64_t n, int l, double* __restrict__ Y) {
  __shared__ double tile[32][33];
  const int64_t a0 = (int64_t)blockIdx.x * 32;
  const int i0 = blockIdx.y * 32;
  for (int t = threadIdx.y; t < 32; t += 8) {
    const int i = i0 + t;
    const int64_t a = a0 + threadIdx.x;
    tile[t][threadIdx.x] = (i < l && a < n) ? (double)Yt[(int64_t)i * ldy + a] : 0.0;
  }
  __syncthreads();
  for (int t = threadIdx.y; t < 32; t += 8) {
    const int64_t a = a0 + t;
    const int i = i0 + threadIdx.x;
    if (a < n && i < l) Y[a * l + i] = tile[threadIdx.x][t];
  }
}

void transpose_to_t(const double* Y, int64_t n, int l, int prec, void* Yt, int64_t ldy, hipStream_t s) {
  dim3 grid((unsigned)ceil_div(n, 32), (unsigned)ceil_div(l, 32));
  if (prec == KRR_FP64)
    hipLaunchKernelGGL(k_transpose_to<double>, grid, dim3(32, 8), 0, s, Y, n, l, (double*)Yt, ldy);
  else
    hipLaunchKernelGGL(k_transpose_to<float>, grid, dim3(32, 8), 0, s, Y, n, l, (float*)Yt, ldy);
  KRR_LAUNCH_CHECK();
}

void transpose_from_t(const void* Yt, int64_t ldy, int64_t n, int l, int prec, double* Y, hipStream_t s) {
  dim3 grid((unsigned)ceil_div(n, 32), (unsigned)ceil_div(l, 32));
  if (prec == KRR_FP64)
    hipLaunchKernelGGL(k_transpose_from<double>, grid, dim3(32, 8), 0, s, (const double*)Yt, ldy, n, l, Y);
  else
    hipLaunchKernelGGL(k_transpose_from<float>, grid, dim3(32, 8), 0, s, (const float*)Yt, ldy, n, l, Y);
  KRR_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ pivoted QR kernels
// (value, index) argmax with ties to the lower index; -1 marks selected columns.
struct ArgMax {
  double v;
  int64_t i;
};
__device__ __forceinline__ ArgMax amax(ArgMax a, ArgMax b) {
  if (b.v > a.v || (b.v == a.v && b.i < a.i)) return b;
  return a;
}

constexpr int kQrBlock = 256;

// Partial column sums over one slab of rows [i0, i0 + slab): part[slab, c] = sum_i q_i Yt[i, c] (MODE 0)
// or sum_i Yt[i, c]^2 (MODE 1).  2-D grid (column blocks x row slabs) so that a pass over Yt fills the
// chip even when n / 256 is small; one column per thread, rows unrolled by 4 for memory-level parallelism.
template <typename T, int MODE>
__global__ __launch_bounds__(kQrBlock) void k_qr_slab(const T* __restrict__ Yt, int64_t ldy, int64_t N, int l,
                                                      int slab, const double* __restrict__ q,
                                                      double* __restrict__ part) {
  const int64_t c = (int64_t)blockIdx.x * kQrBlock + threadIdx.x;
  const int i0 = blockIdx.y * slab;
  const int i1 = i0 + slab < l ? i0 + slab : l;
  if (c >= N) return;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int i = i0;
  for (; i + 4 <= i1; i += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double y = (double)Yt[(int64_t)(i + u) * ldy + c];
      acc[u] = MODE == 1 ? __builtin_fma(y, y, acc[u]) : __builtin_fma(q[i + u], y, acc[u]);
    }
  }
  for (; i < i1; ++i) {
    const double y = (double)Yt[(int64_t)i * ldy + c];
    acc[0] = MODE == 1 ? __builtin_fma(y, y, acc[0]) : __builtin_fma(q[i], y, acc[0]);
  }
  part[(int64_t)blockIdx.y * N + c] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// Column update after a pass, summing the slab partials in slab order: mode 1 sets nrm2[c] to the sum
// (initial squared norms); mode 0 downdates nrm2[c] -= r_c^2 for unselected columns (clamped at 0).
// Writes the per-block argmax of the updated norms.
__global__ __launch_bounds__(kQrBlock) void k_qr_update(const double* __restrict__ part, int nslab, int64_t N,
                                                        int mode, double* __restrict__ nrm2,
                                                        ArgMax* __restrict__ amax_part) {
  __shared__ ArgMax red[kQrBlock];
  const int64_t c = (int64_t)blockIdx.x * kQrBlock + threadIdx.x;
  ArgMax best{-2.0, INT64_MAX};
  if (c < N) {
    double r = 0.0;
    for (int sl = 0; sl < nslab; ++sl) r += part[(int64_t)sl * N + c];
    if (mode == 1) {
      nrm2[c] = r;
      best = ArgMax{r, c};
    } else {
      double v = nrm2[c];
      if (v >= 0.0) {
        v -= r * r;
        v = v > 0.0 ? v : 0.0;
        nrm2[c] = v;
        best = ArgMax{v, c};
      }
    }
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int w = kQrBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = amax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) amax_part[blockIdx.x] = red[0];
}

// Final argmax over block partials -> pivot; gathers w = Yt[:, p] and records piv / rdiag.
template <typename T>
__global__ __launch_bounds__(1024) void k_qr_pick(const ArgMax* __restrict__ part, int nparts,
                                                  const T* __restrict__ Yt, int64_t ldy, int l, int j,
                                                  double* __restrict__ nrm2, int64_t* __restrict__ piv,
                                                  double* __restrict__ rdiag, double* __restrict__ w,
                                                  int64_t* __restrict__ pcur) {
  __shared__ ArgMax red[1024];
  ArgMax best{-2.0, INT64_MAX};
  for (int t = threadIdx.x; t < nparts; t += 1024) best = amax(best, part[t]);
  red[threadIdx.x] = best;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = amax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const ArgMax b = red[0];
  const int64_t p = b.i == INT64_MAX ? 0 : b.i;
  if (threadIdx.x == 0) {
    piv[j] = p;
    rdiag[j] = sqrt(b.v > 0 ? b.v : 0.0);
    *pcur = p;
    nrm2[p] = -1.0;   // selected
  }
  for (int i = threadIdx.x; i < l; i += 1024) w[i] = (double)Yt[(int64_t)i * ldy + p];
}

// t[c] = Q[c, :] . w for c < j  (Q stored k x l row-major: row c is q_c)
__global__ __launch_bounds__(256) void k_qr_proj_dots(const double* __restrict__ Q, int l, int j,
                                                      const double* __restrict__ w, double* __restrict__ t) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  if (c >= j) return;
  double s = 0;
  for (int i = threadIdx.x; i < l; i += 256) s = __builtin_fma(Q[(int64_t)c * l + i], w[i], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) t[c] = red[0];
}

// w[i] -= sum_c t[c] Q[c, i]: a block of 256 threads covers 32 rows, 8 threads per row splitting the
// c range; partials combined in LDS in a fixed order.
__global__ __launch_bounds__(256) void k_qr_proj_sub(const double* __restrict__ Q, int l, int j,
                                                     const double* __restrict__ t, double* __restrict__ w) {
  __shared__ double red[256];
  const int rl = threadIdx.x & 31, sl = threadIdx.x >> 5;
  const int i = blockIdx.x * 32 + rl;
  double s = 0;
  if (i < l)
    for (int c = sl; c < j; c += 8) s = __builtin_fma(t[c], Q[(int64_t)c * l + i], s);
  red[threadIdx.x] = s;
  __syncthreads();
  if (sl == 0 && i < l) {
    double tot = 0;
    for (int u = 0; u < 8; ++u) tot += red[u * 32 + rl];
    w[i] -= tot;
  }
}

// q_j = w / ||w|| (single block)
__global__ __launch_bounds__(1024) void k_qr_normalize(const double* __restrict__ w, int l, int j,
                                                       double* __restrict__ Q) {
  __shared__ double red[1024];
  double s = 0;
  for (int i = threadIdx.x; i < l; i += 1024) s = __builtin_fma(w[i], w[i], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double nrm = sqrt(red[0]);
  const double inv = nrm > 0 ? 1.0 / nrm : 0.0;
  for (int i = threadIdx.x; i < l; i += 1024) Q[(int64_t)j * l + i] = w[i] * inv;
}

template <typename T>
static void qrcp_impl(const T* Yt, int64_t ldy, int64_t N, int l, int k, int64_t* piv, double* rdiag,
                      hipStream_t s) {
  const int64_t nblk = ceil_div(N, (int64_t)kQrBlock);
  // Split the l rows into slabs so that a pass launches about 4096 blocks (at least 16 rows per slab).
  const int want = (int)std::min<int64_t>(std::max<int64_t>(1, ceil_div((int64_t)4096, nblk)), ceil_div(l, 16));
  const int slab = (int)ceil_div(l, want);
  const int nslab = (int)ceil_div(l, slab);
  DevBuf<double> nrm2(N, s), Q((size_t)k * l, s), w(l, s), t(std::max(k, 1), s), part((size_t)nslab * N, s);
  DevBuf<ArgMax> am(nblk, s);
  DevBuf<int64_t> pcur(1, s);
  const dim3 g2((unsigned)nblk, (unsigned)nslab);
  hipLaunchKernelGGL((k_qr_slab<T, 1>), g2, dim3(kQrBlock), 0, s, Yt, ldy, N, l, slab, (const double*)nullptr,
                     part.p);
  hipLaunchKernelGGL(k_qr_update, dim3((unsigned)nblk), dim3(kQrBlock), 0, s, (const double*)part.p, nslab, N, 1,
                     nrm2.p, am.p);
  KRR_LAUNCH_CHECK();
  for (int j = 0; j < k; ++j) {
    hipLaunchKernelGGL(k_qr_pick<T>, dim3(1), dim3(1024), 0, s, (const ArgMax*)am.p, (int)nblk, Yt, ldy, l, j,
                       nrm2.p, piv, rdiag, w.p, pcur.p);
    if (j > 0) {
      for (int pass = 0; pass < 2; ++pass) {   // Gram-Schmidt twice
        hipLaunchKernelGGL(k_qr_proj_dots, dim3(j), dim3(256), 0, s, Q.p, l, j, w.p, t.p);
        hipLaunchKernelGGL(k_qr_proj_sub, dim3((unsigned)ceil_div(l, 32)), dim3(256), 0, s, Q.p, l, j, t.p, w.p);
      }
    }
    hipLaunchKernelGGL(k_qr_normalize, dim3(1), dim3(1024), 0, s, w.p, l, j, Q.p);
    if (j + 1 < k) {
      hipLaunchKernelGGL((k_qr_slab<T, 0>), g2, dim3(kQrBlock), 0, s, Yt, ldy, N, l, slab,
                         (const double*)(Q.p + (int64_t)j * l), part.p);
      hipLaunchKernelGGL(k_qr_update, dim3((unsigned)nblk), dim3(kQrBlock), 0, s, (const double*)part.p, nslab, N,
                         0, nrm2.p, am.p);
    }
    KRR_LAUNCH_CHECK();
  }
}

void qrcp_t(const void* Yt, int64_t ldy, int64_t N, int l, int k, int prec, int64_t* piv, double* rdiag,
            hipStream_t s) {
  KRR_REQUIRE(k >= 1 && k <= l && k <= N, "pivoted QR needs 1 <= k <= min(l, n)");
  if (prec == KRR_FP64) qrcp_impl<double>((const double*)Yt, ldy, N, l, k, piv, rdiag, s);
  else qrcp_impl<float>((const float*)Yt, ldy, N, l, k, piv, rdiag, s);
}

}  // namespace krr
