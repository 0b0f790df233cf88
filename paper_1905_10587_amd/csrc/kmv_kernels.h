// Kernel templates of the exact Gaussian kernel MVM (included by one translation unit per
// precision so the instantiations compile in parallel).  See kmv.hip for the overview.
#pragma once

#include "kmv.h"

namespace krr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ FP64 exp(-t), t >= 0
// exp(-t) = 2^{-n} exp(r), n = rint(t / ln 2), r = n ln2 - t in [-ln2/2, ln2/2] (Cody-Waite with a
// two-part ln 2 whose high part has 42 significant bits, so n * LN2_HI is exact), exp(r) by its
// Taylor series to degree 12 (truncation below 2e-16 relative on the reduced interval).
__device__ __forceinline__ double exp_neg_f64(double t) {
  constexpr double LN2_HI = 0x1.62e42fefa3800p-1;
  constexpr double LN2_LO = 0x1.ef35793c76730p-45;
  const double n = __builtin_rint(t * kLog2e);
  double r = __builtin_fma(n, LN2_HI, -t);
  r = __builtin_fma(n, LN2_LO, r);
  double p = 2.08767569878681e-09;            // 1/12!
  p = __builtin_fma(p, r, 2.505210838544172e-08);
  p = __builtin_fma(p, r, 2.755731922398589e-07);
  p = __builtin_fma(p, r, 2.7557319223985893e-06);
  p = __builtin_fma(p, r, 2.48015873015873e-05);
  p = __builtin_fma(p, r, 0.0001984126984126984);
  p = __builtin_fma(p, r, 0.001388888888888889);
  p = __builtin_fma(p, r, 0.008333333333333333);
  p = __builtin_fma(p, r, 0.041666666666666664);
  p = __builtin_fma(p, r, 0.16666666666666666);
  p = __builtin_fma(p, r, 0.5);
  p = __builtin_fma(p, r, 1.0);
  p = __builtin_fma(p, r, 1.0);
  const double res = __builtin_ldexp(p, -(int)n);
  return t < 708.0 ? res : 0.0;
}

// ------------------------------------------------------------------ direct kernels (FP64 / FP32)
// Block: 256 threads, each owns TM targets (strided by 256) and RC columns.  Sources stream through
// LDS in tiles of TS points (coalesced cooperative loads); every wave then reads a source's
// coordinates and weights with one wave-uniform (broadcast) LDS access.  grid.y splits the sources,
// grid.z the column chunks.
template <int D>
struct DirectTile {
  static constexpr int TS = D <= 16 ? 256 : (D <= 32 ? 128 : 64);
};

template <int D, int TM, int RC, int DV>
__global__ __launch_bounds__(256) void k_kmv_f64(const double* __restrict__ xt, const double* __restrict__ xs,
                                                 const double* __restrict__ v, int Rp, int64_t src_len,
                                                 int64_t n_src, double inv_eps, double* __restrict__ part,
                                                 int64_t mpad, int Rout) {
  constexpr int NO = DV == 2 ? 2 : 1;
  constexpr int TS = DirectTile<D>::TS;
  __shared__ double sx[TS * D];
  __shared__ double sv[TS * RC];
  const int64_t ibase = (int64_t)blockIdx.x * (256 * TM) + threadIdx.x;
  const int c0 = blockIdx.z * RC;
  const int64_t jb = (int64_t)blockIdx.y * src_len;
  const int64_t je = jb + src_len < n_src ? jb + src_len : n_src;
  double xi[TM][D];
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int k = 0; k < D; ++k) xi[t][k] = xt[(ibase + t * 256) * D + k];
  double acc[TM][RC][NO];
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int c = 0; c < RC; ++c)
#pragma unroll
      for (int o = 0; o < NO; ++o) acc[t][c][o] = 0.0;
  for (int64_t jt = jb; jt < je; jt += TS) {
    __syncthreads();
    for (int u = threadIdx.x; u < TS * D; u += 256) sx[u] = xs[jt * D + u];
    for (int u = threadIdx.x; u < TS * RC; u += 256) sv[u] = v[(jt + u / RC) * Rp + c0 + u % RC];
    __syncthreads();
#pragma unroll 2
    for (int j = 0; j < TS; ++j) {
      double xj[D], vj[RC];
#pragma unroll
      for (int k = 0; k < D; ++k) xj[k] = sx[j * D + k];
#pragma unroll
      for (int c = 0; c < RC; ++c) vj[c] = sv[j * RC + c];
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        double d2 = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          const double df = xi[t][k] - xj[k];
          d2 = __builtin_fma(df, df, d2);
        }
        const double tt = d2 * inv_eps;
        const double e = exp_neg_f64(tt);
        if (DV == 0 || DV == 2) {
#pragma unroll
          for (int c = 0; c < RC; ++c) acc[t][c][0] = __builtin_fma(e, vj[c], acc[t][c][0]);
        }
        if (DV >= 1) {
          const double ed = tt * e;
#pragma unroll
          for (int c = 0; c < RC; ++c) acc[t][c][NO - 1] = __builtin_fma(ed, vj[c], acc[t][c][NO - 1]);
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < TM; ++t) {
    const int64_t i = ibase + t * 256;
    double* prow = part + ((int64_t)blockIdx.y * mpad + i) * Rout;
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      prow[c0 + c] = acc[t][c][0];
      if (DV == 2) prow[Rp + c0 + c] = acc[t][c][1];
    }
  }
}

// FP32 form: coordinates pre-scaled so that q = -||t'-s'||^2 is the exp2 argument.  Per pair: D subs,
// D FMAs, one v_exp_f32, RC FMAs.  FP32 partial sums are folded into FP64 once per 256 sources.
template <int D, int TM, int RC, int DV>
__global__ __launch_bounds__(256) void k_kmv_f32(const float* __restrict__ xt, const float* __restrict__ xs,
                                                 const float* __restrict__ v, int Rp, int64_t src_len,
                                                 int64_t n_src, double* __restrict__ part, int64_t mpad,
                                                 int Rout) {
  constexpr int NO = DV == 2 ? 2 : 1;
  constexpr int TS = 256;
  __shared__ float sx[TS * D];
  __shared__ float sv[TS * RC];
  const int64_t ibase = (int64_t)blockIdx.x * (256 * TM) + threadIdx.x;
  const int c0 = blockIdx.z * RC;
  const int64_t jb = (int64_t)blockIdx.y * src_len;
  const int64_t je = jb + src_len < n_src ? jb + src_len : n_src;
  float xi[TM][D];
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int k = 0; k < D; ++k) xi[t][k] = xt[(ibase + t * 256) * D + k];
  double acc[TM][RC][NO];
#pragma unroll
  for (int t = 0; t < TM; ++t)
#pragma unroll
    for (int c = 0; c < RC; ++c)
#pragma unroll
      for (int o = 0; o < NO; ++o) acc[t][c][o] = 0.0;
  constexpr float kLn2f = 0.69314718055994531f;
  for (int64_t jt = jb; jt < je; jt += TS) {
    __syncthreads();
    for (int u = threadIdx.x; u < TS * D; u += 256) sx[u] = xs[jt * D + u];
    for (int u = threadIdx.x; u < TS * RC; u += 256) sv[u] = v[(jt + u / RC) * Rp + c0 + u % RC];
    __syncthreads();
    float a32[TM][RC][NO];
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
      for (int c = 0; c < RC; ++c)
#pragma unroll
        for (int o = 0; o < NO; ++o) a32[t][c][o] = 0.0f;
#pragma unroll 2
    for (int j = 0; j < TS; ++j) {
      float xj[D], vj[RC];
#pragma unroll
      for (int k = 0; k < D; ++k) xj[k] = sx[j * D + k];
#pragma unroll
      for (int c = 0; c < RC; ++c) vj[c] = sv[j * RC + c];
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        float d2 = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          const float df = xi[t][k] - xj[k];
          d2 = __builtin_fmaf(df, df, d2);
        }
        const float e = __builtin_amdgcn_exp2f(-d2);
        if (DV == 0 || DV == 2) {
#pragma unroll
          for (int c = 0; c < RC; ++c) a32[t][c][0] = __builtin_fmaf(e, vj[c], a32[t][c][0]);
        }
        if (DV >= 1) {
          const float ed = d2 * e * kLn2f;   // (D^2/eps) K = (ln 2) q K with q = log2(e) D^2/eps
#pragma unroll
          for (int c = 0; c < RC; ++c) a32[t][c][NO - 1] = __builtin_fmaf(ed, vj[c], a32[t][c][NO - 1]);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
      for (int c = 0; c < RC; ++c)
#pragma unroll
        for (int o = 0; o < NO; ++o) acc[t][c][o] += (double)a32[t][c][o];
  }
#pragma unroll
  for (int t = 0; t < TM; ++t) {
    const int64_t i = ibase + t * 256;
    double* prow = part + ((int64_t)blockIdx.y * mpad + i) * Rout;
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      prow[c0 + c] = acc[t][c][0];
      if (DV == 2) prow[Rp + c0 + c] = acc[t][c][1];
    }
  }
}

// ------------------------------------------------------------------ MIXED (MFMA) kernel, one column
// Block: 4 waves; wave w owns 16*NF consecutive targets as NF A-fragments (16 rows x 32*NCH K).
// For each group of 16 sources the wave loads one B-fragment per chunk and issues NF*NCH MFMAs;
// lane l then holds q for targets (l/16)*4+e of each fragment against source l%16, applies
// v_exp_f32 and one FMA with v.  Partial sums are folded into FP64 every 256 sources and finally
// reduced over the 16 lanes that share a target row.
template <int NCH, int NF, int DV>
__global__ __launch_bounds__(256) void k_kmv_mixed(const uint4* __restrict__ A, const uint4* __restrict__ B,
                                                   const float* __restrict__ v, int Rp, int col,
                                                   int64_t src_len, int64_t n_src, double* __restrict__ part,
                                                   int64_t mpad, int Rout, int out_col) {
  constexpr int NO = DV == 2 ? 2 : 1;
  constexpr int KV = NCH * 4;   // uint4 (8 bf16) units per point
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * NF);
  const int64_t jb = (int64_t)blockIdx.y * src_len;
  const int64_t je = jb + src_len < n_src ? jb + src_len : n_src;
  const int r16 = lane & 15;
  const int kq = lane >> 4;

  bf16x8 a[NF][NCH];
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
      a[f][ch] = __builtin_bit_cast(bf16x8, A[(row0 + 16 * f + r16) * KV + ch * 4 + kq]);

  double acc[NF][4][NO];
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int o = 0; o < NO; ++o) acc[f][e][o] = 0.0;
  constexpr float kNegLn2f = -0.69314718055994531f;

  bf16x8 bn[NCH];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) bn[ch] = __builtin_bit_cast(bf16x8, B[(jb + r16) * KV + ch * 4 + kq]);
  float vn = v[(jb + r16) * Rp + col];
  for (int64_t j0 = jb; j0 < je; j0 += 256) {
    float a32[NF][4][NO];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int o = 0; o < NO; ++o) a32[f][e][o] = 0.0f;
    for (int64_t j = j0; j < j0 + 256; j += 16) {
      // the fragment for j was loaded one step ahead; issue the load for j + 16 now
      bf16x8 b[NCH];
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) b[ch] = bn[ch];
      const float vj = vn;
      const int64_t jn = j + 16 < je ? j + 16 : j;
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) bn[ch] = __builtin_bit_cast(bf16x8, B[(jn + r16) * KV + ch * 4 + kq]);
      vn = v[(jn + r16) * Rp + col];
      f32x4 q[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        q[f] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) q[f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f][ch], b[ch], q[f], 0, 0, 0);
      }
#pragma unroll
      for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float ex = __builtin_amdgcn_exp2f(q[f][e]);
          if (DV == 0 || DV == 2) a32[f][e][0] = __builtin_fmaf(ex, vj, a32[f][e][0]);
          if (DV >= 1) a32[f][e][NO - 1] = __builtin_fmaf(q[f][e] * ex, kNegLn2f * vj, a32[f][e][NO - 1]);
        }
      }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int o = 0; o < NO; ++o) acc[f][e][o] += (double)a32[f][e][o];
  }
  // reduce over the 16 lanes (sources mod 16) sharing each target row
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int o = 0; o < NO; ++o) {
        double x = acc[f][e][o];
        x += __shfl_xor(x, 8);
        x += __shfl_xor(x, 4);
        x += __shfl_xor(x, 2);
        x += __shfl_xor(x, 1);
        acc[f][e][o] = x;
      }
  if (r16 == 0) {
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = row0 + 16 * f + kq * 4 + e;
        double* prow = part + ((int64_t)blockIdx.y * mpad + i) * Rout;
        prow[out_col] = acc[f][e][0];
        if (DV == 2) prow[Rp + out_col] = acc[f][e][1];
      }
  }
}


}  // namespace krr
