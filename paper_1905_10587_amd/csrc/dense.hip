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

// Block form of the same tournament: the k columns are cut into blocks of W, and round r pairs the blocks
// (P, Q) by the circle method.  A workgroup copies the 2W columns S of its pair into LDS, forms their Gram
// matrix G = S^T S afresh, and runs `inner` sweeps of two-sided Jacobi rotations on G (rounds of W
// disjoint rotations, G <- R^T G R in a column phase and a row phase, the rotated 2x2 block set by the
// stable formulas G_pp - t G_pq, G_qq + t G_pq and 0), accumulating J = prod R.  It then writes S J back to A and V J to V.  The rotation of a pair (p, q) is the one the
// scalar algorithm would take from the same a = G_pp, b = G_qq, g = G_pq.  The convergence measure is
// taken from the fresh Gram (every pair of the 2W columns), so the outer loop stops on columns that are
// orthogonal as stored.  Columns >= k (partial last block, bye block) are zero and never rotate.
template <int W>
__global__ __launch_bounds__(256) void k_jacobi_blockpair(double* __restrict__ A, double* __restrict__ V, int k,
                                                          int NB, int r, double rot_tol, int inner,
                                                          unsigned long long* __restrict__ offmax) {
  constexpr int C2 = 2 * W;
  static_assert(C2 * C2 <= 256 && W * C2 <= 256, "one thread per Gram entry");
  constexpr int NEB = (C2 / 4) * (C2 / 4);   // 4 x 4 blocks of the Gram matrix
  constexpr int RGW = 64 / NEB;              // row groups per wave
  extern __shared__ double sa[];   // C2 columns of length k, column stride ks (odd: conflict-free)
  __shared__ double G[C2][C2 + 1];
  __shared__ double gred[4][NEB][16];
  __shared__ double J[C2][C2 + 1];
  __shared__ double rc[W], rs[W], rt[W], rg[W], ra[W], rb[W];
  __shared__ int rp[W], rq[W], ron[W];
  __shared__ double offw[4];
  const int tid = threadIdx.x;
  const int i = blockIdx.x;
  int P, Q;
  if (i == 0) { P = r; Q = NB - 1; }
  else { P = (r + i) % (NB - 1); Q = (r - i + NB - 1) % (NB - 1); }
  if (P > Q) { const int t = P; P = Q; Q = t; }
  // a pair with the bye block has nothing to rotate across, except in the first round of a sweep, where
  // it is that block's only chance to rotate its own column pairs (the bye's columns read as zeros)
  if ((int64_t)Q * W >= k && r != 0) return;
  auto gcol = [&](int lc) { return lc < W ? P * W + lc : Q * W + (lc - W); };
  const int ks = k | 1;
  // Rows per thread: at most RMAX (k <= 256 RMAX, which the host guarantees for each W).  All of a
  // thread's A loads are issued before the first LDS store; its V rows are loaded into registers right
  // after, so their latency is hidden behind the Gram matrix and the rotations.
  constexpr int RMAX = W == 8 ? 5 : 9;
  {
    double row[RMAX][C2];
#pragma unroll
    for (int u = 0; u < RMAX; ++u) {
      const int t = tid + 256 * u;
#pragma unroll
      for (int lc = 0; lc < C2; ++lc) {
        const int g = gcol(lc);
        row[u][lc] = (t < k && g < k) ? A[(int64_t)g * k + t] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < RMAX; ++u) {
      const int t = tid + 256 * u;
      if (t < k) {
#pragma unroll
        for (int lc = 0; lc < C2; ++lc) sa[lc * ks + t] = row[u][lc];
      }
    }
  }
  // W = 8 applies the rotation on the FP64 matrix cores: wave w takes the 16-row tiles w, w + 4, ...
  // (at most TPW of them), and lane l holds rows 16 tile + l % 16 of columns 4 kc + l / 16 (kc = 0..3):
  // its B-operand elements.  Its V values are loaded here in that layout.  W = 4: rows tid + 256 u.
  constexpr bool kMfmaApply = C2 == 16;
  constexpr int TPW = (256 * RMAX / 16 + 3) / 4;
  const int alane = tid & 63, awave = tid >> 6, ar16 = alane & 15, akq = alane >> 4;
  double vpre[kMfmaApply ? TPW : RMAX][kMfmaApply ? 4 : C2];
  if constexpr (kMfmaApply) {
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
      const int t = (awave + 4 * tt) * 16 + ar16;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const int g = gcol(4 * kc + akq);
        vpre[tt][kc] = (t < k && g < k) ? V[(int64_t)g * k + t] : 0.0;
      }
    }
  } else {
#pragma unroll
    for (int u = 0; u < RMAX; ++u) {
      const int t = tid + 256 * u;
#pragma unroll
      for (int lc = 0; lc < C2; ++lc) {
        const int g = gcol(lc);
        vpre[u][lc] = (t < k && g < k) ? V[(int64_t)g * k + t] : 0.0;
      }
    }
  }
  __syncthreads();
  // fresh Gram G = S^T S: lane (row group, 4 x 4 block) accumulates its block over the rows of its group,
  // the row groups of a wave are combined by butterflies, the four waves in a fixed order.  Block (bi, bj)
  // and (bj, bi) use the same products in the same order, so G is exactly symmetric.
  {
    const int lane = tid & 63, wave = tid >> 6;
    const int eb = lane % NEB, rgl = lane / NEB;
    const int bi = eb / (C2 / 4), bj = eb % (C2 / 4);
    const int rg = wave * RGW + rgl, nrg = 4 * RGW;
    double acc[4][4];
#pragma unroll
    for (int e1 = 0; e1 < 4; ++e1)
#pragma unroll
      for (int e2 = 0; e2 < 4; ++e2) acc[e1][e2] = 0.0;
    for (int t = rg; t < k; t += nrg) {
      double x[4], y[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        x[e] = sa[(4 * bi + e) * ks + t];
        y[e] = sa[(4 * bj + e) * ks + t];
      }
#pragma unroll
      for (int e1 = 0; e1 < 4; ++e1)
#pragma unroll
        for (int e2 = 0; e2 < 4; ++e2) acc[e1][e2] = __builtin_fma(x[e1], y[e2], acc[e1][e2]);
    }
#pragma unroll
    for (int e1 = 0; e1 < 4; ++e1)
#pragma unroll
      for (int e2 = 0; e2 < 4; ++e2)
        for (int o = NEB; o < 64; o <<= 1) acc[e1][e2] += __shfl_xor(acc[e1][e2], o);
    if (rgl == 0) {
#pragma unroll
      for (int e1 = 0; e1 < 4; ++e1)
#pragma unroll
        for (int e2 = 0; e2 < 4; ++e2) gred[wave][eb][e1 * 4 + e2] = acc[e1][e2];
    }
  }
  __syncthreads();
  if (tid < C2 * C2) {
    const int gi = tid / C2, gj = tid % C2;
    const int eb = (gi / 4) * (C2 / 4) + gj / 4, e = (gi % 4) * 4 + gj % 4;
    G[gi][gj] = ((gred[0][eb][e] + gred[1][eb][e]) + gred[2][eb][e]) + gred[3][eb][e];
    J[gi][gj] = gi == gj ? 1.0 : 0.0;
  }
  __syncthreads();
  double off_local = 0.0;
  if (tid < C2 * C2) {
    const int gi = tid / C2, gj = tid % C2;
    if (gi < gj) {
      const double den = sqrt(G[gi][gi] * G[gj][gj]);
      off_local = den > 0 ? fabs(G[gi][gj]) / den : 0.0;
    }
  }
  // The first round of an outer sweep meets every block once: it runs the full circle over the 2W columns
  // (pairs inside P and inside Q included); later rounds run only the W x W cross pairs, in W rounds of W
  // disjoint pairs (p, W + (p + ir) mod W), which every outer sweep meets exactly once.
  const bool full = r == 0;
  const int nround = full ? C2 - 1 : W;
  for (int sw = 0; sw < inner; ++sw) {
    for (int ir = 0; ir < nround; ++ir) {
      if (tid < W) {   // rotation parameters of slot tid
        int p, q;
        if (!full) { p = tid; q = W + (tid + ir) % W; }
        else if (tid == 0) { p = ir; q = C2 - 1; }
        else { p = (ir + tid) % (C2 - 1); q = (ir - tid + C2 - 1) % (C2 - 1); }
        if (p > q) { const int t = p; p = q; q = t; }
        const double a = G[p][p], b = G[q][q], g = G[p][q];
        const double den = sqrt(a * b);
        const double off = den > 0 ? fabs(g) / den : 0.0;
        const int on = off > rot_tol;
        double c = 1.0, sn = 0.0, tt = 0.0;
        if (on) {
          const double zeta = (b - a) / (2.0 * g);
          tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          c = 1.0 / sqrt(1.0 + tt * tt);
          sn = c * tt;
        }
        rp[tid] = p; rq[tid] = q; ron[tid] = on;
        rc[tid] = c; rs[tid] = sn; rt[tid] = tt; rg[tid] = g; ra[tid] = a; rb[tid] = b;
      }
      __syncthreads();
      const int sl = tid / C2, e = tid % C2;   // W slots x C2 rows/columns
      if (tid < W * C2 && ron[sl]) {         // column phase: G <- G R, J <- J R
        const int p = rp[sl], q = rq[sl];
        const double c = rc[sl], sn = rs[sl];
        const double x = G[e][p], y = G[e][q];
        G[e][p] = c * x - sn * y;
        G[e][q] = sn * x + c * y;
        const double u = J[e][p], w = J[e][q];
        J[e][p] = c * u - sn * w;
        J[e][q] = sn * u + c * w;
      }
      __syncthreads();
      if (tid < W * C2 && ron[sl]) {         // row phase: G <- R^T G
        const int p = rp[sl], q = rq[sl];
        const double c = rc[sl], sn = rs[sl];
        const double x = G[p][e], y = G[q][e];
        G[p][e] = c * x - sn * y;
        G[q][e] = sn * x + c * y;
      }
      __syncthreads();
      if (tid < W && ron[tid]) {             // the rotated 2x2 block, stable formulas
        const int p = rp[tid], q = rq[tid];
        G[p][p] = ra[tid] - rt[tid] * rg[tid];
        G[q][q] = rb[tid] + rt[tid] * rg[tid];
        G[p][q] = 0.0;
        G[q][p] = 0.0;
      }
      __syncthreads();
    }
  }
  if constexpr (kMfmaApply) {
    // A <- S J, V <- V J as (S J)^T = J^T S^T on v_mfma_f64_16x16x4_f64: the A operand is J^T (lane l
    // holds J[4 kc + l / 16][l % 16]), the B operand S^T or V^T of a 16-row tile, and result element e of
    // lane l is column 4 e + l / 16 at row 16 tile + l % 16, so each store instruction writes four runs
    // of 16 consecutive rows.
    double ja[4];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) ja[kc] = J[4 * kc + akq][ar16];
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) {
      const int t = (awave + 4 * tt) * 16 + ar16;
      if ((awave + 4 * tt) * 16 >= k) break;   // wave-uniform
      f64x4 da = {0.0, 0.0, 0.0, 0.0}, dv = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const double sb = t < k ? sa[(4 * kc + akq) * ks + t] : 0.0;
        da = __builtin_amdgcn_mfma_f64_16x16x4f64(ja[kc], sb, da, 0, 0, 0);
        dv = __builtin_amdgcn_mfma_f64_16x16x4f64(ja[kc], vpre[tt][kc], dv, 0, 0, 0);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int g = gcol(4 * e + akq);
        if (t < k && g < k) {
          A[(int64_t)g * k + t] = da[e];
          V[(int64_t)g * k + t] = dv[e];
        }
      }
    }
  } else {
  // A <- S J, V <- V J on the 2W columns, one row per thread at a time (V from the prefetched rows)
#pragma unroll
  for (int u = 0; u < RMAX; ++u) {
    const int t = tid + 256 * u;
    if (t >= k) break;
    double so[C2];
#pragma unroll
    for (int m = 0; m < C2; ++m) so[m] = sa[m * ks + t];
#pragma unroll 1
    for (int lc = 0; lc < C2; ++lc) {   // J is read from LDS here (not hoisted into registers)
      const int g = gcol(lc);
      if (g >= k) continue;
      double xa = 0.0, xv = 0.0;
#pragma unroll
      for (int m = 0; m < C2; ++m) {
        xa = __builtin_fma(so[m], J[m][lc], xa);
        xv = __builtin_fma(vpre[u][m], J[m][lc], xv);
      }
      A[(int64_t)g * k + t] = xa;
      V[(int64_t)g * k + t] = xv;
    }
  }
  }
  // block maximum of the off-diagonal measure -> one atomic
  for (int o = 32; o > 0; o >>= 1) {
    const double t = __shfl_xor(off_local, o);
    off_local = t > off_local ? t : off_local;
  }
  if ((tid & 63) == 0) offw[tid >> 6] = off_local;
  __syncthreads();
  if (tid == 0) {
    double m = offw[0];
    for (int w = 1; w < 4; ++w) m = offw[w] > m ? offw[w] : m;
    atomicMax(offmax, (unsigned long long)__double_as_longlong(m));
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
  const int kInner = 1;   // sweeps over a block pair's Gram matrix per visit
  // block form when a pair of column blocks fits in LDS (2W columns of k doubles <= 141 KB)
  const int W = k >= 64 && k <= 1100 ? 8 : (k >= 64 && k <= 2200 ? 4 : 0);
  const size_t lds = (size_t)2 * W * (k | 1) * sizeof(double);
  int NB = 0;
  if (W) {
    NB = (int)ceil_div(k, W);
    NB += NB & 1;
    if (W == 8)
      KRR_CHECK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_jacobi_blockpair<8>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    else
      KRR_CHECK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_jacobi_blockpair<4>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  }
  DevBuf<unsigned long long> off(1, s);
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    KRR_CHECK_HIP(hipMemsetAsync(off.p, 0, sizeof(unsigned long long), s));
    if (W == 8) {
      for (int r = 0; r < NB - 1; ++r)
        hipLaunchKernelGGL(k_jacobi_blockpair<8>, dim3(NB / 2), dim3(256), lds, s, A, V, k, NB, r, 1e-15, kInner,
                           off.p);
    } else if (W == 4) {
      for (int r = 0; r < NB - 1; ++r)
        hipLaunchKernelGGL(k_jacobi_blockpair<4>, dim3(NB / 2), dim3(256), lds, s, A, V, k, NB, r, 1e-15, kInner,
                           off.p);
    } else {
      for (int r = 0; r < K - 1; ++r)
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
