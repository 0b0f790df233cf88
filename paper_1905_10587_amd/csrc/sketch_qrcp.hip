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
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "kmv_kernels.h"
#include "radix_sort.h"
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
static void qrcp_full(const T* Yt, int64_t ldy, int64_t N, int l, int k, int64_t* piv, double* rdiag,
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

// ------------------------------------------------------------------ candidate-set pivoting
// Residual norms never grow, so a norm computed at step j0 is an upper bound at every later step.
// After a refresh (all norms brought up to date), the T columns with the largest norms become
// candidates; their norms are kept exact step by step (T dot products per step), the others stay
// stale.  The best candidate is the true argmax as long as its norm exceeds tau, the largest stale
// norm outside the set; otherwise (and at least every kQrBatch steps) the norms are refreshed with one
// pass over Yt that applies all pending directions q_{j0} .. q_{j-1}, and the candidates are chosen
// again.  The pivots are those of the one-pass-per-step algorithm (up to rounding in the norms).
constexpr int kQrCand = 1024;    // candidates
constexpr int kQrBatch = 32;     // pending directions per refresh pass at most

// nrm2[c] -= (q_t^T Yt[:, c])^2 for t = 0 .. b-1 in order (clamped at 0), q_t = QT[:, j0 + t] (QT: l x ldq,
// row-major, zero beyond the computed columns).  A block covers 64 columns; its four waves each sum a
// quarter of the rows (lane = column) and the quarters are added in a fixed order through LDS.  Each wave
// stages its q rows through its own LDS buffer in chunks of kQrChunk rows (coalesced loads, the next chunk
// in registers while the current one is used; broadcast reads), and loads its Yt rows one chunk ahead.
// Selected columns (nrm2 < 0) are left as they are.
constexpr int kQrChunk = 16;

template <typename T, int B>
__global__ __launch_bounds__(256) void k_qr_refresh(const T* __restrict__ Yt, int64_t ldy, int64_t N, int l,
                                                    const double* __restrict__ QT, int ldq, int j0, int b,
                                                    double* __restrict__ nrm2) {
  constexpr int QPL = kQrChunk * B / 64;   // q values per lane per chunk
  static_assert(QPL >= 1 && (kQrChunk * B) % 64 == 0, "chunk must fill the wave");
  __shared__ double qs[4][kQrChunk * B];
  __shared__ double part[3][B][64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t c = (int64_t)blockIdx.x * 64 + lane;
  const int64_t cr = c < N ? c : N - 1;
  const int lq = (l + 3) / 4;
  const int i0 = wave * lq < l ? wave * lq : l;
  const int i1 = i0 + lq < l ? i0 + lq : l;
  double* qw = qs[wave];
  double acc[B];
#pragma unroll
  for (int t = 0; t < B; ++t) acc[t] = 0.0;
  const T* yp = Yt + cr;
  // chunk 0 into registers
  double qn[QPL];
  T yn[kQrChunk];
#pragma unroll
  for (int u = 0; u < QPL; ++u) {
    const int e = lane + 64 * u, r = e / B, t = e % B;
    qn[u] = i0 + r < i1 ? QT[(int64_t)(i0 + r) * ldq + j0 + t] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kQrChunk; ++u) yn[u] = i0 + u < i1 ? yp[(int64_t)(i0 + u) * ldy] : (T)0;
  for (int i = i0; i < i1; i += kQrChunk) {
    // current chunk: q into LDS, y into registers; then start loading the next chunk
#pragma unroll
    for (int u = 0; u < QPL; ++u) qw[lane + 64 * u] = qn[u];
    T ycur[kQrChunk];
#pragma unroll
    for (int u = 0; u < kQrChunk; ++u) ycur[u] = yn[u];
    const int inx = i + kQrChunk;
#pragma unroll
    for (int u = 0; u < QPL; ++u) {
      const int e = lane + 64 * u, r = e / B, t = e % B;
      qn[u] = inx + r < i1 ? QT[(int64_t)(inx + r) * ldq + j0 + t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kQrChunk; ++u) yn[u] = inx + u < i1 ? yp[(int64_t)(inx + u) * ldy] : (T)0;
#pragma unroll
    for (int u = 0; u < kQrChunk; ++u) {
      const double y = (double)ycur[u];   // rows past i1 hold zeros in both y and q
#pragma unroll
      for (int t = 0; t < B; ++t) acc[t] = __builtin_fma(qw[u * B + t], y, acc[t]);
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int t = 0; t < B; ++t) part[wave - 1][t][lane] = acc[t];
  }
  __syncthreads();
  if (wave > 0 || c >= N) return;
  double v = nrm2[c];
  if (v < 0.0) return;
#pragma unroll
  for (int t = 0; t < B; ++t) {
    if (t < b) {
      const double r = ((acc[t] + part[0][t][lane]) + part[1][t][lane]) + part[2][t][lane];
      v -= r * r;
      v = v > 0.0 ? v : 0.0;
    }
  }
  nrm2[c] = v;
}

// Sort keys: larger norm first, selected columns last (ascending order of the key).
__global__ void k_qr_keys(const double* __restrict__ nrm2, int64_t N, uint64_t* __restrict__ key,
                          int64_t* __restrict__ idx) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= N) return;
  const double v = nrm2[c];
  key[c] = v < 0.0 ? ~0ull : 0x7FFFFFFFFFFFFFFFull - (uint64_t)__double_as_longlong(v);
  idx[c] = c;
}

// Candidate t: its column gathered into Yc[t, :] (FP64, row stride l), its norm into cnrm[t]
// (-1 past the unselected columns); tau = norm of the first column after the candidates (-1 if none).
template <typename T>
__global__ __launch_bounds__(256) void k_qr_gather(const T* __restrict__ Yt, int64_t ldy, int l,
                                                   const int64_t* __restrict__ sidx,
                                                   const uint64_t* __restrict__ skey, int64_t N, int Tc,
                                                   const double* __restrict__ nrm2, int64_t* __restrict__ cidx,
                                                   double* __restrict__ cnrm, double* __restrict__ Yc,
                                                   double* __restrict__ tau) {
  const int t = blockIdx.x;
  const bool live = t < N && skey[t] != ~0ull;
  const int64_t c = live ? sidx[t] : 0;
  if (threadIdx.x == 0) {
    cidx[t] = live ? c : INT64_MAX;
    cnrm[t] = live ? nrm2[c] : -1.0;
    if (t == 0) *tau = (Tc < N && skey[Tc] != ~0ull) ? nrm2[sidx[Tc]] : -1.0;
  }
  for (int i = threadIdx.x; i < l; i += 256) Yc[(int64_t)t * l + i] = live ? (double)Yt[(int64_t)i * ldy + c] : 0.0;
}

// Step j's pivot among the candidates.  ok: 1 while the steps of this batch are valid; a pick whose
// norm does not exceed tau (unless the candidates are fresh) clears it and records the step in *fail,
// and every later kernel of the batch does nothing.
template <typename T>
__global__ __launch_bounds__(1024) void k_qr_cpick(const double* __restrict__ cnrm, const int64_t* __restrict__ cidx,
                                                   int Tc, const double* __restrict__ tau, int fresh,
                                                   const T* __restrict__ Yt, int64_t ldy, int l, int j,
                                                   double* __restrict__ nrm2, int64_t* __restrict__ piv,
                                                   double* __restrict__ rdiag, double* __restrict__ w,
                                                   int* __restrict__ ok, int* __restrict__ fail) {
  __shared__ ArgMax red[1024];
  __shared__ int go;
  if (*ok == 0) return;
  ArgMax best{-2.0, INT64_MAX};
  for (int t = threadIdx.x; t < Tc; t += 1024) {
    const double v = cnrm[t];
    if (v >= 0.0) best = amax(best, ArgMax{v, cidx[t]});
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = amax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const ArgMax b = red[0];
    go = b.i != INT64_MAX && (fresh || b.v > *tau);
    if (go) {
      piv[j] = b.i;
      rdiag[j] = sqrt(b.v > 0 ? b.v : 0.0);
      nrm2[b.i] = -1.0;   // selected
    } else {
      *ok = 0;
      *fail = j;
    }
  }
  __syncthreads();
  if (!go) return;
  const int64_t p = red[0].i;
  for (int i = threadIdx.x; i < l; i += 1024) w[i] = (double)Yt[(int64_t)i * ldy + p];
}

// t[c] = Q[c, :] . w for c < j (one block per c), skipped when the batch is stopped.
__global__ __launch_bounds__(256) void k_qr_cdots(const double* __restrict__ Q, int l, int j,
                                                  const double* __restrict__ w, double* __restrict__ t,
                                                  const int* __restrict__ ok) {
  __shared__ double red[256];
  if (*ok == 0) return;
  const int c = blockIdx.x;
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

// w[i] -= sum_{c<j} t[c] QT[i, c]: one wave per row i reading row i of QT contiguously.
__global__ __launch_bounds__(256) void k_qr_csub(const double* __restrict__ QT, int ldq, int l, int j,
                                                 const double* __restrict__ t, double* __restrict__ w,
                                                 const int* __restrict__ ok) {
  if (*ok == 0) return;
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= l) return;
  double s = 0;
  for (int c = lane; c < j; c += 64) s = __builtin_fma(t[c], QT[(int64_t)i * ldq + c], s);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) w[i] -= s;
}

// q_j = w / ||w|| into Q[j, :] and QT[:, j]; then the candidates' norms are downdated with q_j
// (one wave per candidate; every block recomputes ||w|| from w, block 0 stores q_j).
__global__ __launch_bounds__(256) void k_qr_cupdate(const double* __restrict__ w, int l, int j,
                                                    double* __restrict__ Q, double* __restrict__ QT, int ldq,
                                                    const double* __restrict__ Yc, const int64_t* __restrict__ cidx,
                                                    int Tc, const int64_t* __restrict__ piv,
                                                    double* __restrict__ cnrm, const int* __restrict__ ok) {
  __shared__ double red[256];
  __shared__ double qs[4096];
  if (*ok == 0) return;
  double s = 0;
  for (int i = threadIdx.x; i < l; i += 256) s = __builtin_fma(w[i], w[i], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double nrm = sqrt(red[0]);
  const double inv = nrm > 0 ? 1.0 / nrm : 0.0;
  for (int i = threadIdx.x; i < l; i += 256) {
    const double q = w[i] * inv;
    qs[i] = q;
    if (blockIdx.x == 0) {
      Q[(int64_t)j * l + i] = q;
      QT[(int64_t)i * ldq + j] = q;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= Tc) return;
  if (cidx[t] == piv[j]) {
    if (lane == 0) cnrm[t] = -1.0;   // the pivot itself
    return;
  }
  const double v = cnrm[t];
  if (v < 0.0) return;
  double r = 0;
  for (int i = lane; i < l; i += 64) r = __builtin_fma(qs[i], Yc[(int64_t)t * l + i], r);
  for (int o = 32; o > 0; o >>= 1) r += __shfl_xor(r, o);
  if (lane == 0) {
    const double nv = v - r * r;
    cnrm[t] = nv > 0.0 ? nv : 0.0;
  }
}

__global__ void k_qr_reset_ok(int* ok) { *ok = 1; }

template <typename T>
static void refresh_pass(const T* Yt, int64_t ldy, int64_t N, int l, const double* QT, int ldq, int j0, int b,
                         double* nrm2, hipStream_t s) {
  const dim3 g((unsigned)ceil_div(N, 64));
#define KRR_QRF(B) hipLaunchKernelGGL((k_qr_refresh<T, B>), g, dim3(256), 0, s, Yt, ldy, N, l, QT, ldq, j0, b, nrm2)
  if (b <= 4) KRR_QRF(4);
  else if (b <= 8) KRR_QRF(8);
  else if (b <= 16) KRR_QRF(16);
  else KRR_QRF(32);
#undef KRR_QRF
  KRR_LAUNCH_CHECK();
}

template <typename T>
static void qrcp_cand(const T* Yt, int64_t ldy, int64_t N, int l, int k, int64_t* piv, double* rdiag, hipStream_t s) {
  const int64_t nblk = ceil_div(N, (int64_t)kQrBlock);
  const int want = (int)std::min<int64_t>(std::max<int64_t>(1, ceil_div((int64_t)4096, nblk)), ceil_div(l, 16));
  const int slab = (int)ceil_div(l, want);
  const int nslab = (int)ceil_div(l, slab);
  const int Tc = (int)std::min<int64_t>(kQrCand, N);
  const int ldq = k + kQrBatch;   // QT columns past k stay zero (read by the widest refresh form)
  DevBuf<double> nrm2(N, s), Q((size_t)k * l, s), QT((size_t)l * ldq, s), w(l, s), t(std::max(k, 1), s),
      part((size_t)nslab * N, s), Yc((size_t)Tc * l, s), cnrm(Tc, s), tau(1, s);
  DevBuf<ArgMax> am(nblk, s);
  DevBuf<uint64_t> key(N, s), skey(N, s);
  DevBuf<int64_t> idx(N, s), sidx(N, s), cidx(Tc, s);
  DevBuf<int> flags(2, s);   // ok, fail step
  int* ok = flags.p;
  int* fail = flags.p + 1;
  KRR_CHECK_HIP(hipMemsetAsync(QT.p, 0, QT.bytes(), s));
  RadixSortWork rsw;
  rsw.reserve(N, s);
  // initial squared norms
  const dim3 g2((unsigned)nblk, (unsigned)nslab);
  hipLaunchKernelGGL((k_qr_slab<T, 1>), g2, dim3(kQrBlock), 0, s, Yt, ldy, N, l, slab, (const double*)nullptr,
                     part.p);
  hipLaunchKernelGGL(k_qr_update, dim3((unsigned)nblk), dim3(kQrBlock), 0, s, (const double*)part.p, nslab, N, 1,
                     nrm2.p, am.p);
  KRR_LAUNCH_CHECK();
  int j = 0, j0 = 0;
  const bool verbose = std::getenv("KRR_QR_VERBOSE") != nullptr;
  int refreshes = 0;
  while (j < k) {
    // refresh: bring every norm up to date with q_{j0} .. q_{j-1}, choose the candidates
    if (j > j0) refresh_pass(Yt, ldy, N, l, QT.p, ldq, j0, j - j0, nrm2.p, s);
    j0 = j;
    ++refreshes;
    hipLaunchKernelGGL(k_qr_keys, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s, (const double*)nrm2.p, N,
                       key.p, idx.p);
    KRR_LAUNCH_CHECK();
    radix_sort_pairs(key.p, skey.p, idx.p, sidx.p, N, 64, rsw, s);
    hipLaunchKernelGGL(k_qr_gather<T>, dim3((unsigned)Tc), dim3(256), 0, s, Yt, ldy, l, (const int64_t*)sidx.p,
                       (const uint64_t*)skey.p, N, Tc, (const double*)nrm2.p, cidx.p, cnrm.p, Yc.p, tau.p);
    hipLaunchKernelGGL(k_qr_reset_ok, dim3(1), dim3(1), 0, s, ok);
    KRR_LAUNCH_CHECK();
    // a batch of steps on the candidates, stopped on the device at the first invalid pick
    const int jend = std::min(k, j0 + kQrBatch);
    for (int jj = j0; jj < jend; ++jj) {
      hipLaunchKernelGGL(k_qr_cpick<T>, dim3(1), dim3(1024), 0, s, (const double*)cnrm.p, (const int64_t*)cidx.p, Tc,
                         (const double*)tau.p, jj == j0 ? 1 : 0, Yt, ldy, l, jj, nrm2.p, piv, rdiag, w.p, ok,
                         fail);
      if (jj > 0) {
        for (int pass = 0; pass < 2; ++pass) {   // Gram-Schmidt twice
          hipLaunchKernelGGL(k_qr_cdots, dim3(jj), dim3(256), 0, s, (const double*)Q.p, l, jj, (const double*)w.p,
                             t.p, (const int*)ok);
          hipLaunchKernelGGL(k_qr_csub, dim3((unsigned)ceil_div(l, 4)), dim3(256), 0, s, (const double*)QT.p, ldq, l,
                             jj, (const double*)t.p, w.p, (const int*)ok);
        }
      }
      hipLaunchKernelGGL(k_qr_cupdate, dim3((unsigned)ceil_div(Tc, 4)), dim3(256), 0, s, (const double*)w.p, l, jj,
                         Q.p, QT.p, ldq, (const double*)Yc.p, (const int64_t*)cidx.p, Tc, (const int64_t*)piv,
                         cnrm.p, (const int*)ok);
      KRR_LAUNCH_CHECK();
    }
    int hf[2];
    KRR_CHECK_HIP(hipMemcpyAsync(hf, flags.p, sizeof(hf), hipMemcpyDeviceToHost, s));
    KRR_CHECK_HIP(hipStreamSynchronize(s));
    KRR_REQUIRE(hf[0] || hf[1] > j0, "pivoted QR: no valid pivot on fresh candidates");
    j = hf[0] ? jend : hf[1];
  }
  if (verbose) std::fprintf(stderr, "krr qrcp: %d steps, %d candidate refreshes\n", k, refreshes);
}

void qrcp_t(const void* Yt, int64_t ldy, int64_t N, int l, int k, int prec, int64_t* piv, double* rdiag,
            hipStream_t s) {
  KRR_REQUIRE(k >= 1 && k <= l && k <= N, "pivoted QR needs 1 <= k <= min(l, n)");
  // KRR_QR_FULL: one pass over Yt per step (also used for l > 4096, beyond the candidate kernels' LDS,
  // and for more than 2^31 - 1 columns)
  const bool full = std::getenv("KRR_QR_FULL") != nullptr || l > 4096 || N > INT32_MAX;   // sort counts are int
  if (prec == KRR_FP64) {
    if (full) qrcp_full<double>((const double*)Yt, ldy, N, l, k, piv, rdiag, s);
    else qrcp_cand<double>((const double*)Yt, ldy, N, l, k, piv, rdiag, s);
  } else {
    if (full) qrcp_full<float>((const float*)Yt, ldy, N, l, k, piv, rdiag, s);
    else qrcp_cand<float>((const float*)Yt, ldy, N, l, k, piv, rdiag, s);
  }
}

}  // namespace krr
