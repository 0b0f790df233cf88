// Kernel templates of the exact Gaussian kernel MVM (included by one translation unit per
// precision so the instantiations compile in parallel).  See kmv.hip for the overview.
#pragma once

#include "kmv.h"

#include <type_traits>

namespace krr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ FP64 2^q, q <= 0
// 2^q = 2^n * 2^f with n = rint(q) and f = q - n (exact, |f| <= 1/2); 2^f by a degree-10
// near-minimax polynomial (Chebyshev fit in 50-digit arithmetic, coefficients rounded to double;
// worst relative error 3.1e-16 on [-1/2, 1/2]; derived by gen_exp2_poly.py).  CLAMP: q is clamped at
// -1020 so ldexp stays in the normal range and a q of -inf cannot give NaN; values below 2^-1020 come out
// as ~1e-307 instead of 0.  Without it (for callers that know q >= -1020 and finite) one operation less.
template <bool CLAMP = true>
__device__ __forceinline__ double exp2_neg_f64(double q) {
  if (CLAMP) q = q > -1020.0 ? q : -1020.0;
  const double n = __builtin_rint(q);
  const double f = q - n;
  double p = 0x1.e6063f7217bc6p-28;
  p = __builtin_fma(p, f, 0x1.b675bca4eeebbp-24);
  p = __builtin_fma(p, f, 0x1.62bfd47773353p-20);
  p = __builtin_fma(p, f, 0x1.ffcb54062e698p-17);
  p = __builtin_fma(p, f, 0x1.430913096fd9fp-13);
  p = __builtin_fma(p, f, 0x1.5d87fe9d7a584p-10);
  p = __builtin_fma(p, f, 0x1.3b2ab6fba1ddap-7);
  p = __builtin_fma(p, f, 0x1.c6b08d703ce49p-5);
  p = __builtin_fma(p, f, 0x1.ebfbdff82c598p-3);
  p = __builtin_fma(p, f, 0x1.62e42fefa3a19p-1);
  p = __builtin_fma(p, f, 1.0);
  return __builtin_ldexp(p, (int)n);
}

// exp(-t) for t >= 0
__device__ __forceinline__ double exp_neg_f64(double t) { return exp2_neg_f64(-t * kLog2e); }

// ------------------------------------------------------------------ direct kernels (FP64 / FP32)
// Block: 256 threads, each owns TM targets (strided by 256) and RC columns.  Sources stream through
// LDS in tiles of TS points (coalesced cooperative loads); every wave then reads a source's
// coordinates and weights with one wave-uniform (broadcast) LDS access.  grid.y splits the sources,
// grid.z the column chunks.
template <int D>
struct DirectTile {
  static constexpr int TS = D <= 16 ? 256 : (D <= 32 ? 128 : 64);
};

// TSX != 0: source tiles of TSX points (the short-split form for small products, whose source splits are
// multiples of TSX rather than of 256).
template <int D, int TM, int RC, int DV, int TSX = 0>
__global__ __launch_bounds__(256) void k_kmv_f64(const double* __restrict__ xt, const double* __restrict__ xs,
                                                 const double* __restrict__ v, int Rp, int64_t src_len,
                                                 int64_t n_src, double neg_c, double* __restrict__ part,
                                                 int64_t mpad, int Rout) {
  // neg_c = -log2(e) / eps: the exponent q = neg_c * D^2 is the base-2 exponent of the kernel value
  constexpr int NO = DV == 2 ? 2 : 1;
  constexpr int TS = TSX ? TSX : DirectTile<D>::TS * 8 / (RC > 8 ? RC : 8);   // wide column chunks: shorter tiles
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
        const double q = d2 * neg_c;
        const double e = exp2_neg_f64(q);
        if (DV == 0 || DV == 2) {
#pragma unroll
          for (int c = 0; c < RC; ++c) acc[t][c][0] = __builtin_fma(e, vj[c], acc[t][c][0]);
        }
        if (DV >= 1) {
          const double ed = -kLn2 * q * e;   // (D^2/eps) K = -ln(2) q K
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

typedef double f64x4 __attribute__((ext_vector_type(4)));

// FP64 product with many right-hand sides on the FP64 matrix cores (v_mfma_f64_16x16x4_f64, A 16 x 4,
// B 4 x 16, exact FP64 products and sums).  A block covers 64 targets (wave w: targets row0 + 16 w ..) and
// 16 * NRG columns.  At each 4-source step lane l evaluates the one pair (target l % 16, source l / 16) in
// FP64 direct differences, which is its A-operand element, and the NRG MFMAs contract it with the V rows of
// the four sources: the kernel value of a pair is evaluated once for all 16 * NRG columns.  The source tiles
// (16 sources: coordinates and V rows) move into LDS by direct global->LDS loads one tile ahead (double
// buffered, 38 KB per block at D = 6 and 128 columns), one barrier per tile, so the loads of the next tile
// overlap the products of this one.  A V row of the block (16 NRG doubles) is one wave instruction, its
// lanes past 8 NRG idle.  The last column block may be partly filled: the lanes whose 16 bytes fall in its
// dead column groups load nothing, and those groups' products read stale LDS values and are not stored (a
// branch around their MFMAs would cost more than the wasted products).
template <int D, int NRG>
__global__ __launch_bounds__(256) void k_kmv_f64_mfma_db(const double* __restrict__ xt,
                                                         const double* __restrict__ xs,
                                                         const double* __restrict__ v, int Rp, int64_t src_len,
                                                         int64_t n_src, double neg_c, double* __restrict__ part,
                                                         int64_t mpad, int Rout, int64_t m_store, int n_store) {
  constexpr int TS = 16;
  constexpr int RCH = 16 * NRG;
  constexpr int VS = RCH + 16;      // LDS row stride (doubles): consecutive rows start 128 bytes apart in the banks
  constexpr int NXU = TS * D / 2;   // 16-byte units of a tile's source coordinates
  __shared__ __align__(16) double sx0[TS * D], sx1[TS * D];
  __shared__ __align__(16) double sv0[TS * VS], sv1[TS * VS];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r16 = lane & 15;
  const int kq = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * 64 + wave * 16;
  const int c0 = blockIdx.z * RCH;
  const int ng = (Rp - c0) / 16 < NRG ? (Rp - c0) / 16 : NRG;   // live column groups of this block
  const bool vlive = 2 * lane < 16 * ng;
  const int64_t jb = (int64_t)blockIdx.y * src_len;
  const int64_t je = jb + src_len < n_src ? jb + src_len : n_src;
  const int ntiles = (int)((je - jb) / TS);
  double xi[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xi[k] = xt[(row0 + r16) * D + k];
  f64x4 acc[NRG];
#pragma unroll
  for (int g = 0; g < NRG; ++g) acc[g] = f64x4{0.0, 0.0, 0.0, 0.0};

  // staging of the tile at source jt: V row r by wave r % 4 (one row of up to 1 KB per wave instruction),
  // the coordinates by the first NXU threads
  auto issue = [&](double* dx, double* dv, int64_t jt) {
    for (int r = wave; r < TS; r += 4)
      if (vlive) __builtin_amdgcn_global_load_lds(v + (jt + r) * Rp + c0 + 2 * lane, dv + r * VS, 16, 0, 0);
    if (tid < NXU) __builtin_amdgcn_global_load_lds(xs + jt * D + 2 * tid, dx + 128 * wave, 16, 0, 0);
  };

  if (ntiles > 0) issue(sx0, sv0, jb);
  for (int t = 0; t < ntiles; ++t) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();   // tile t staged by every wave; tile t - 1's buffers no longer read
    if (t + 1 < ntiles) {
      if (t & 1) issue(sx0, sv0, jb + (int64_t)(t + 1) * TS);
      else issue(sx1, sv1, jb + (int64_t)(t + 1) * TS);
    }
    const double* sx = (t & 1) ? sx1 : sx0;
    const double* sv = (t & 1) ? sv1 : sv0;
#pragma unroll
    for (int s4 = 0; s4 < TS; s4 += 4) {
      const int js = s4 + kq;
      double d2 = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const double df = xi[k] - sx[js * D + k];
        d2 = __builtin_fma(df, df, d2);
      }
      const double e = exp2_neg_f64(d2 * neg_c);
#pragma unroll
      for (int g = 0; g < NRG; ++g)
        acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(e, sv[js * VS + 16 * g + r16], acc[g], 0, 0, 0);
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t row = row0 + 4 * e + kq;
    double* prow = part + ((int64_t)blockIdx.y * mpad + row) * Rout + c0 + r16;
#pragma unroll
    for (int g = 0; g < NRG; ++g)
      if (g < ng && row < m_store && c0 + 16 * g + r16 < n_store) prow[16 * g] = acc[g][e];
  }
}

// Symmetric FP64 form for the square product u = K(X, X) v (one column), D even and <= 16.  Super-tiles
// and partial slots as in k_kmv_mixed_sym: block b owns one pair (r, c <= ...) of the upper triangle,
// evaluates the E x E tile once and writes its row sums to part[c][rows of r] and, off the diagonal, its
// column sums to part[r][rows of c].  Each thread owns TM targets (strided by 256 in a target tile).
// Sources stream through LDS in tiles of 256; a wave walks each 64-source sub-tile in rotated order
// (lane l takes source (l + k) mod 64 at step k), so at every step the 64 lanes touch 64 distinct
// sources: a lane's column contribution (its TM targets) is added to that source's per-wave LDS slot
// with an LDS atomic, and the four waves' slots are added in a fixed order at the end of the tile.
// Rows are stored with an odd number of 16-byte units so the rotated reads are bank-conflict free.
template <int D, int TM>
__global__ __launch_bounds__(256) void k_kmv_f64_sym(const double* __restrict__ X, const double* __restrict__ v,
                                                     int Rp, double neg_c, int E, int NS, int64_t npad,
                                                     double* __restrict__ part, int Rout) {
  static_assert(D % 2 == 0 && D <= 16, "even dimensions up to 16");
  constexpr int SD = 2 * ((D / 2) | 1);   // LDS row stride in doubles (odd number of 16-byte units)
  constexpr int TS = 256;
  constexpr int TT = 256 * TM;
  __shared__ double xs[TS * SD];
  __shared__ double vs[TS];
  __shared__ double cacc[4][TS];

  const int64_t nitems = (int64_t)NS * (NS + 1) / 2;
  const int64_t per = (nitems + 7) / 8;
  const int64_t item = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (item >= nitems) return;
  int c = (int)((sqrt(8.0 * (double)item + 1.0) - 1.0) / 2);
  if (c < 0) c = 0;
  if (c > NS - 1) c = NS - 1;
  auto col_start = [&](int64_t cc) { return cc * (cc + 1) / 2; };
  while (c > 0 && col_start(c) > item) --c;
  while (c + 1 < NS && col_start(c + 1) <= item) ++c;
  const int r = (int)(item - col_start(c));
  const bool diag = r == c;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t t0 = (int64_t)r * E, t1 = t0 + E < npad ? t0 + E : npad;
  const int64_t s0 = (int64_t)c * E, s1 = s0 + E < npad ? s0 + E : npad;
  const int ntile = (int)((s1 - s0) / TS);
  const int ntt = (int)((t1 - t0) / TT);

  auto run = [&](auto colflag) {
    constexpr bool COL = decltype(colflag)::value;
    for (int tt = 0; tt < ntt; ++tt) {
      const int64_t ib = t0 + (int64_t)tt * TT + tid;
      double xi[TM][D], vt[TM], acc[TM];
#pragma unroll
      for (int m = 0; m < TM; ++m) {
#pragma unroll
        for (int k = 0; k < D; ++k) xi[m][k] = X[(ib + m * 256) * D + k];
        vt[m] = COL ? v[(ib + m * 256) * Rp] : 0.0;
        acc[m] = 0.0;
      }
      for (int t = 0; t < ntile; ++t) {
        const int64_t jt = s0 + (int64_t)t * TS;
        double* dst = part + (int64_t)r * npad + jt + tid;   // one column: dense partials
        double prev = 0.0;
        if (COL && tt > 0) prev = *dst;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < D; ++k) xs[tid * SD + k] = X[(jt + tid) * D + k];
        vs[tid] = v[(jt + tid) * Rp];
        if (COL) {
#pragma unroll
          for (int u = 0; u < 4; ++u) cacc[wave][lane + 64 * u] = 0.0;
        }
        __syncthreads();
        for (int sub = 0; sub < 4; ++sub) {
#pragma unroll 2
          for (int k = 0; k < 64; ++k) {
            const int j = sub * 64 + ((lane + k) & 63);
            double xj[D];
#pragma unroll
            for (int u = 0; u < D; u += 2) {
              const double2 w = *reinterpret_cast<const double2*>(&xs[j * SD + u]);
              xj[u] = w.x;
              xj[u + 1] = w.y;
            }
            const double vj = vs[j];
            double cs = 0.0;
#pragma unroll
            for (int m = 0; m < TM; ++m) {
              double d2 = 0.0;
#pragma unroll
              for (int u = 0; u < D; ++u) {
                const double df = xi[m][u] - xj[u];
                d2 = __builtin_fma(df, df, d2);
              }
              const double e = exp2_neg_f64(d2 * neg_c);
              acc[m] = __builtin_fma(e, vj, acc[m]);
              if (COL) cs = __builtin_fma(e, vt[m], cs);
            }
            if (COL) __hip_atomic_fetch_add(&cacc[wave][j], cs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        }
        __syncthreads();
        if (COL) *dst = prev + (((cacc[0][tid] + cacc[1][tid]) + cacc[2][tid]) + cacc[3][tid]);
      }
#pragma unroll
      for (int m = 0; m < TM; ++m) part[(int64_t)c * npad + ib + m * 256] = acc[m];
    }
  };
  if (diag) run(std::false_type{});
  else run(std::true_type{});
}

// Symmetric FP64 form with the exponent's cross term on the FP64 matrix cores (v_mfma_f64_16x16x4f64, FP64
// products and sums): q = c'|x_i|^2 + c'|x_j|^2 - 2c' x_i.x_j (c' = neg_c).  When D + 2 fits the K padding
// (D = 2, 6: FOLD) the whole of q is the contraction of a_i = [x_i, c'|x_i|^2, 1] with b_j = [-2c' x_j, 1,
// c'|x_j|^2], and a pair costs the FP64 exp2 and the row and column FMAs on the VALU; otherwise the MFMA
// contracts x_i with b_j = -2c' x_j on top of the accumulator input c'|x_i|^2 (the lane's four result rows),
// and q = C + c'|x_j|^2 adds one VALU operation (an extra K chunk costs more than this, the MFMA work not
// being hidden behind the VALU work).  Either way the direct form's D subtractions, D FMAs and scaling are
// gone.  The cancellation leaves an error of up to about k u |c'| max|x|^2 in q (centred coordinates), a
// relative error ln2 times that in a kernel value: the norms 2(D + 1), the scaled b_j 2, and D accumulation
// steps on partial sums up to 3|c'| max|x|^2 plus the final addition 4 (k = 5D + 8), or with FOLD D + 2 steps
// on partial sums up to 4|c'| max|x|^2 (k = 6D + 12).
// Same super-tiles, triangle order and partial slots as k_kmv_f64_sym.  Block: 4 waves x NFR fragments of 16
// targets (64 NFR targets); source tiles of 256 points in LDS (b_j, or x_j and c'|x_j|^2), 16 sources per
// MFMA step.
// Lane l holds the pairs (target 4e + l/16 of a fragment, source l%16 of the step), e = 0..3: its row sums
// are added over the 16 lanes of its group at the end, its column sums over the four groups every step.
// CLAMP false: the caller guarantees q >= -1020 for every pair (c'|x_i - x_j|^2 bounded by the points' box),
// so the exp2 needs no clamp.
template <int D, int NFR, bool CLAMP>
__global__ __launch_bounds__(256) void k_kmv_f64_symm(const double* __restrict__ X, const double* __restrict__ v,
                                                      int Rp, double neg_c, int E, int NS, int64_t npad,
                                                      double* __restrict__ part, int Rout) {
  static_assert(D % 2 == 0 && D <= 16, "even dimensions up to 16");
  constexpr bool FOLD = D % 4 == 2;
  constexpr int KC = (D + (FOLD ? 2 : 0) + 3) / 4;   // K chunks of the contraction
  constexpr int SD = 4 * KC + 1;                     // LDS row stride of the source entries (doubles)
  constexpr int TS = 256;
  constexpr int TT = 4 * NFR * 16;                   // targets per target tile
  __shared__ double xs[TS * SD];
  __shared__ double vs[TS];
  __shared__ double ns[FOLD ? 1 : TS];               // c'|x_j|^2 (without FOLD)
  __shared__ double cacc[4][TS];
  const double m2c = -2.0 * neg_c;

  const int64_t nitems = (int64_t)NS * (NS + 1) / 2;
  const int64_t per = (nitems + 7) / 8;
  const int64_t item = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (item >= nitems) return;
  int c = (int)((sqrt(8.0 * (double)item + 1.0) - 1.0) / 2);
  if (c < 0) c = 0;
  if (c > NS - 1) c = NS - 1;
  auto col_start = [&](int64_t cc) { return cc * (cc + 1) / 2; };
  while (c > 0 && col_start(c) > item) --c;
  while (c + 1 < NS && col_start(c + 1) <= item) ++c;
  const int r = (int)(item - col_start(c));
  const bool diag = r == c;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int r16 = lane & 15;
  const int kq = lane >> 4;
  const int64_t t0 = (int64_t)r * E, t1 = t0 + E < npad ? t0 + E : npad;
  const int64_t s0 = (int64_t)c * E, s1 = s0 + E < npad ? s0 + E : npad;
  const int ntile = (int)((s1 - s0) / TS);
  const int ntt = (int)((t1 - t0) / TT);

  auto run = [&](auto colflag) {
    constexpr bool COL = decltype(colflag)::value;
    for (int tt = 0; tt < ntt; ++tt) {
      const int64_t rowf = t0 + (int64_t)tt * TT + (int64_t)wave * (16 * NFR);
      double a[NFR][KC], vt[NFR][4], acc[NFR][4];
      f64x4 an[NFR];   // the MFMA's accumulator input: c'|x|^2 of the lane's four result rows (FOLD: zero)
#pragma unroll
      for (int f = 0; f < NFR; ++f) {
        const int64_t ra = rowf + 16 * f + r16;   // the A operand's row of this lane
        if (FOLD) {
          double nn = 0.0;
#pragma unroll
          for (int k = 0; k < D; ++k) nn = __builtin_fma(X[ra * D + k], X[ra * D + k], nn);
#pragma unroll
          for (int kc = 0; kc < KC; ++kc) {
            const int k = 4 * kc + kq;
            a[f][kc] = k < D ? X[ra * D + k] : k == D ? neg_c * nn : k == D + 1 ? 1.0 : 0.0;
          }
          an[f] = f64x4{0.0, 0.0, 0.0, 0.0};
        } else {
#pragma unroll
          for (int kc = 0; kc < KC; ++kc) {
            const int k = 4 * kc + kq;
            a[f][kc] = k < D ? X[ra * D + k] : 0.0;
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) {   // c'|x|^2 of the result rows of this lane
            const int64_t row = rowf + 16 * f + 4 * e + kq;
            double nn = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) nn = __builtin_fma(X[row * D + k], X[row * D + k], nn);
            an[f][e] = neg_c * nn;
          }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          vt[f][e] = COL ? v[(rowf + 16 * f + 4 * e + kq) * Rp] : 0.0;
          acc[f][e] = 0.0;
        }
      }
      for (int t = 0; t < ntile; ++t) {
        const int64_t jt = s0 + (int64_t)t * TS;
        double* dst = part + (int64_t)r * npad + jt + tid;   // one column: dense partials
        double prev = 0.0;
        if (COL && tt > 0) prev = *dst;
        __syncthreads();
        {
          double nn = 0.0;
#pragma unroll
          for (int k = 0; k < D; ++k) {
            const double xv = X[(jt + tid) * D + k];
            xs[tid * SD + k] = m2c * xv;
            nn = __builtin_fma(xv, xv, nn);
          }
          if (FOLD) {
            xs[tid * SD + D] = 1.0;
            xs[tid * SD + D + 1] = neg_c * nn;
          } else {
            ns[tid] = neg_c * nn;
          }
#pragma unroll
          for (int k = D + (FOLD ? 2 : 0); k < 4 * KC; ++k) xs[tid * SD + k] = 0.0;
          vs[tid] = v[(jt + tid) * Rp];
        }
        __syncthreads();
#pragma unroll 1
        for (int st = 0; st < TS / 16; ++st) {
          const int j = st * 16 + r16;
          double b[KC];
#pragma unroll
          for (int kc = 0; kc < KC; ++kc) b[kc] = xs[j * SD + 4 * kc + kq];
          const double vj = vs[j];
          const double bn = FOLD ? 0.0 : ns[FOLD ? 0 : j];
          f64x4 C[NFR];
#pragma unroll
          for (int f = 0; f < NFR; ++f) {
            C[f] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[f][0], b[0], an[f], 0, 0, 0);
#pragma unroll
            for (int kc = 1; kc < KC; ++kc) C[f] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[f][kc], b[kc], C[f], 0, 0, 0);
          }
          double cs = 0.0;
#pragma unroll
          for (int f = 0; f < NFR; ++f)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const double q = FOLD ? C[f][e] : C[f][e] + bn;
              const double kv = exp2_neg_f64<CLAMP>(q);
              acc[f][e] = __builtin_fma(kv, vj, acc[f][e]);
              if (COL) cs = __builtin_fma(kv, vt[f][e], cs);
            }
          if (COL) {
            cs += __shfl_xor(cs, 16);
            cs += __shfl_xor(cs, 32);
            if (kq == 0) cacc[wave][j] = cs;
          }
        }
        __syncthreads();
        if (COL) *dst = prev + (((cacc[0][tid] + cacc[1][tid]) + cacc[2][tid]) + cacc[3][tid]);
      }
#pragma unroll
      for (int f = 0; f < NFR; ++f)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          double s = acc[f][e];
#pragma unroll
          for (int o = 1; o < 16; o <<= 1) s += __shfl_xor(s, o);
          if (r16 == 0) part[(int64_t)c * npad + rowf + 16 * f + 4 * e + kq] = s;
        }
    }
  };
  if (diag) run(std::false_type{});
  else run(std::true_type{});
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

  // per-lane pointers, advanced by 16 sources per step; the fragment for the next step is loaded one
  // step ahead (the staged source arrays carry 16 padding rows, so the last prefetch stays in bounds)
  const uint4* bp = B + (jb + r16) * KV + kq;
  const float* vp = v + (jb + r16) * Rp + col;
  const int64_t bstep = 16 * KV;
  const int64_t vstep = 16 * (int64_t)Rp;
  bf16x8 bn[NCH];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) bn[ch] = __builtin_bit_cast(bf16x8, bp[ch * 4]);
  float vn = *vp;
  for (int64_t j0 = jb; j0 < je; j0 += 256) {
    float a32[NF][4][NO];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int o = 0; o < NO; ++o) a32[f][e][o] = 0.0f;
    for (int step = 0; step < 16; ++step) {
      bf16x8 b[NCH];
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) b[ch] = bn[ch];
      const float vj = vn;
      bp += bstep;
      vp += vstep;
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) bn[ch] = __builtin_bit_cast(bf16x8, bp[ch * 4]);
      vn = *vp;
      // software pipeline, two fragments deep: the MFMA of fragment f+2 is issued before the exps of
      // fragment f, so the result of an MFMA is read 16 VALU instructions after its issue
      f32x4 q0 = f32x4{0.f, 0.f, 0.f, 0.f}, q1 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) q0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][ch], b[ch], q0, 0, 0, 0);
      if (NF > 1) {
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
          q1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[NF > 1 ? 1 : 0][ch], b[ch], q1, 0, 0, 0);
      }
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        f32x4 q2 = f32x4{0.f, 0.f, 0.f, 0.f};
        if (f + 2 < NF) {
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch)
            q2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f + 2 < NF ? f + 2 : 0][ch], b[ch], q2, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float ex = __builtin_amdgcn_exp2f(q0[e]);
          if (DV == 0 || DV == 2) a32[f][e][0] = __builtin_fmaf(ex, vj, a32[f][e][0]);
          if (DV >= 1) a32[f][e][NO - 1] = __builtin_fmaf(q0[e] * ex, kNegLn2f * vj, a32[f][e][NO - 1]);
        }
        q0 = q1;
        q1 = q2;
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


// Pipelined form of k_kmv_mixed (same arithmetic, same per-lane summation order, so the results are
// identical).  The MFMA stream runs two fragments ahead of the exp/FMA stream across step boundaries:
// while a wave evaluates the exps of fragment f it issues the MFMAs of fragment f + 2, which for the last
// two fragments of a step belong to the next step (source fragments are prefetched two steps ahead).
// Scheduling barriers interleave one MFMA with a group of VALU instructions, so the matrix core works
// under the wave's own exp/FMA work instead of in a separate burst.  NF >= 2.
template <int NCH, int NF, int DV>
__global__ __launch_bounds__(256) void k_kmv_mixed_pp(const uint4* __restrict__ A, const uint4* __restrict__ B,
                                                      const float* __restrict__ v, int Rp, int col,
                                                      int64_t src_len, int64_t n_src, double* __restrict__ part,
                                                      int64_t mpad, int Rout, int out_col) {
  static_assert(NF >= 2, "the cross-step pipeline needs two fragments per step");
  constexpr int NO = DV == 2 ? 2 : 1;
  constexpr int KV = NCH * 4;
  constexpr int VPER = (DV == 0 ? 8 : 14) / NCH;   // VALU instructions placed after each MFMA
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

  // b: fragment of the current step, bn: next step, bn2: two steps ahead (loaded at the top of a step).
  // The staged source arrays carry 32 padding rows, so the loads past the last step stay in bounds.
  const uint4* bp = B + (jb + r16) * KV + kq;
  const float* vp = v + (jb + r16) * Rp + col;
  const int64_t bstep = 16 * KV;
  const int64_t vstep = 16 * (int64_t)Rp;
  bf16x8 b[NCH], bn[NCH];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    b[ch] = __builtin_bit_cast(bf16x8, bp[ch * 4]);
    bn[ch] = __builtin_bit_cast(bf16x8, bp[bstep + ch * 4]);
  }
  float vj = vp[0], vn = vp[vstep];
  bp += 2 * bstep;
  vp += 2 * vstep;
  f32x4 q0 = f32x4{0.f, 0.f, 0.f, 0.f}, q1 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) q0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][ch], b[ch], q0, 0, 0, 0);
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) q1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][ch], b[ch], q1, 0, 0, 0);

  for (int64_t j0 = jb; j0 < je; j0 += 256) {
    float a32[NF][4][NO];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int o = 0; o < NO; ++o) a32[f][e][o] = 0.0f;
    for (int step = 0; step < 16; ++step) {
      bf16x8 bn2[NCH];
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) bn2[ch] = __builtin_bit_cast(bf16x8, bp[ch * 4]);
      const float vn2 = *vp;
      bp += bstep;
      vp += vstep;
      __builtin_amdgcn_sched_group_barrier(0x020, NCH + 1, 0);   // the prefetch loads go first
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        f32x4 q2 = f32x4{0.f, 0.f, 0.f, 0.f};
        if (f + 2 < NF) {
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch)
            q2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f + 2 < NF ? f + 2 : 0][ch], b[ch], q2, 0, 0, 0);
        } else {
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch)
            q2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f + 2 - NF >= 0 ? f + 2 - NF : 0][ch], bn[ch], q2, 0,
                                                         0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float ex = __builtin_amdgcn_exp2f(q0[e]);
          if (DV == 0 || DV == 2) a32[f][e][0] = __builtin_fmaf(ex, vj, a32[f][e][0]);
          if (DV >= 1) a32[f][e][NO - 1] = __builtin_fmaf(q0[e] * ex, kNegLn2f * vj, a32[f][e][NO - 1]);
        }
        q0 = q1;
        q1 = q2;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);      // one MFMA
          __builtin_amdgcn_sched_group_barrier(0x002, VPER, 0);   // then VALU work
        }
        __builtin_amdgcn_sched_barrier(0);   // keep fragments in order (MFMA results are consumed 2 later)
      }
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        b[ch] = bn[ch];
        bn[ch] = bn2[ch];
      }
      vj = vn;
      vn = vn2;
    }
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int o = 0; o < NO; ++o) acc[f][e][o] += (double)a32[f][e][o];
  }
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

// LDS-staged form of k_kmv_mixed_pp (same arithmetic and per-lane summation order: identical results).
// The four waves of a block share one copy of each source tile: TS sources of split vectors are moved
// from global memory into LDS by direct global->LDS loads (16 bytes per lane, fully coalesced), double
// buffered so that tile t+1 streams in while tile t is evaluated.  Rows are stored with one pad unit
// (stride KV + 1 units of 16 bytes, odd), so the per-step fragment reads (16 rows x 16 bytes per quarter
// wave) fall in distinct banks.  The weights v of the next tile go through a register into LDS.
template <int NCH, int NF, int DV>
__global__ __launch_bounds__(256) void k_kmv_mixed_lds(const uint4* __restrict__ A, const uint4* __restrict__ B,
                                                       const float* __restrict__ v, int Rp, int col,
                                                       int64_t src_len, int64_t n_src, double* __restrict__ part,
                                                       int64_t mpad, int Rout, int out_col) {
  static_assert(NF >= 2, "the pipeline needs two fragments per step");
  constexpr int NO = DV == 2 ? 2 : 1;
  constexpr int KV = NCH * 4;
  constexpr int RS = KV + 1;                 // LDS row stride in 16-byte units
  constexpr int TS = NCH <= 2 ? 256 : 128;   // sources per tile
  constexpr int SPT = TS / 16;               // steps per tile
  constexpr int NI = (TS * RS + 63) / 64;    // direct loads of 64 units per tile
  constexpr int SBU = NI * 64 + 16 * RS;     // + 16 rows read (and discarded) by the last step's look-ahead
  constexpr int VPER = (DV == 0 ? 8 : 14) / NCH;
  __shared__ uint4 sb0[SBU], sb1[SBU];
  __shared__ float sv0[TS + 16], sv1[TS + 16];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * NF);
  const int64_t jb = (int64_t)blockIdx.y * src_len;
  const int64_t je = jb + src_len < n_src ? jb + src_len : n_src;
  const int64_t ntile = (je - jb) / TS;
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
  float a32[NF][4][NO];
  auto clear32 = [&]() {
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int o = 0; o < NO; ++o) a32[f][e][o] = 0.0f;
  };
  auto fold = [&]() {
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int o = 0; o < NO; ++o) acc[f][e][o] += (double)a32[f][e][o];
    clear32();
  };
  constexpr float kNegLn2f = -0.69314718055994531f;

  // Tile j0 -> LDS: slot s of the tile holds unit u of source row r (s = r * RS + u); the pad unit and
  // the slots past TS * RS load a valid unit of the tile that is never read.
  auto issue = [&](uint4* dst, int64_t j0) {
    for (int i = wave; i < NI; i += 4) {
      const int slot = i * 64 + lane;
      int r = slot / RS, u = slot - r * RS;
      if (u == KV) u = 0;
      if (r >= TS) { r = 0; u = 0; }
      __builtin_amdgcn_global_load_lds(B + (j0 + r) * KV + u, dst + i * 64, 16, 0, 0);
    }
  };
  auto vload = [&](int64_t j0) -> float { return tid < TS ? v[(j0 + tid) * Rp + col] : 0.0f; };

  auto compute = [&](const uint4* sb, const float* sv) {
    bf16x8 b[NCH], bn[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) b[ch] = __builtin_bit_cast(bf16x8, sb[r16 * RS + ch * 4 + kq]);
    float vj = sv[r16];
    f32x4 q0 = f32x4{0.f, 0.f, 0.f, 0.f}, q1 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) q0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][ch], b[ch], q0, 0, 0, 0);
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) q1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][ch], b[ch], q1, 0, 0, 0);
#pragma unroll 1
    for (int st = 0; st < SPT; ++st) {
      // look-ahead fragment of the next step (for the last step: pad rows, results discarded)
      const int rn = (st + 1) * 16 + r16;
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) bn[ch] = __builtin_bit_cast(bf16x8, sb[rn * RS + ch * 4 + kq]);
      const float vn = sv[rn];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        f32x4 q2 = f32x4{0.f, 0.f, 0.f, 0.f};
        if (f + 2 < NF) {
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch)
            q2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f + 2 < NF ? f + 2 : 0][ch], b[ch], q2, 0, 0, 0);
        } else {
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch)
            q2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f + 2 - NF >= 0 ? f + 2 - NF : 0][ch], bn[ch], q2, 0,
                                                         0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float ex = __builtin_amdgcn_exp2f(q0[e]);
          if (DV == 0 || DV == 2) a32[f][e][0] = __builtin_fmaf(ex, vj, a32[f][e][0]);
          if (DV >= 1) a32[f][e][NO - 1] = __builtin_fmaf(q0[e] * ex, kNegLn2f * vj, a32[f][e][NO - 1]);
        }
        q0 = q1;
        q1 = q2;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x002, VPER, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) b[ch] = bn[ch];
      vj = vn;
    }
  };

  clear32();
  if (ntile > 0) {
    issue(sb0, jb);
    const float v0 = vload(jb);
    if (tid < TS) sv0[tid] = v0;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  for (int64_t t = 0; t < ntile; t += 2) {
    // tile t from buffer 0 while tile t + 1 streams into buffer 1
    const bool has1 = t + 1 < ntile;
    float vr = 0.0f;
    if (has1) {
      issue(sb1, jb + (t + 1) * TS);
      vr = vload(jb + (t + 1) * TS);
    }
    compute(sb0, sv0);
    if (TS == 256) fold();
    if (has1 && tid < TS) sv1[tid] = vr;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (!has1) break;
    // tile t + 1 from buffer 1 while tile t + 2 streams into buffer 0
    const bool has2 = t + 2 < ntile;
    if (has2) {
      issue(sb0, jb + (t + 2) * TS);
      vr = vload(jb + (t + 2) * TS);
    }
    compute(sb1, sv1);
    fold();   // TS = 256: one tile; TS = 128: the pair of tiles, 256 sources
    if (has2 && tid < TS) sv0[tid] = vr;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }

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

// Symmetric form for the square product u = K(X, X) v (one column), using K_ij = K_ji.  The index range is
// cut into super-tiles of E points; block b owns one pair (r, c), r <= c, of the upper triangle and
// evaluates the E x E tile once:
//   row sums  sum_{j in c} K_ij v_j  for i in r  -> part[c][i],
//   col sums  sum_{i in r} K_ij v_i  for j in c  -> part[r][j]   (off-diagonal pairs only).
// Every slot part[s][i] (s < NS) receives exactly one contribution, so the FP64 finishing pass sums NS
// partials per row in a fixed order.  Inside a block the pipelined LDS-staged tile loop of
// k_kmv_mixed_lds runs once per target tile of 64 NF points; each lane's column partial for one step (its
// source, over its 4 NF targets: FP32 over NF x 4 products) goes to LDS, and at the end of each source
// tile the 16 partials of a source (4 waves x 4 lane groups) are added pairwise in FP32 and the sum is
// added to the source's FP64 slot.  Row sums are folded from FP32 into FP64 every 512 sources.
// Items are laid out so that each XCD (blocks b = x mod 8) walks a contiguous run of the triangle in
// column order.
//
// CULL (points staged in spatial order): cmask[g * ngs + j] holds one bit per 16-source step of the
// 256-source group j for the target group g of 16 NF points (a wave's targets); a set bit means every kernel
// value of that step is exactly zero in FP32, so its exp/FMA work is skipped (the MFMA pipeline still runs).
// Adding exact zeros changes no sum, so the result is bit for bit that of the unculled kernel.  The skipped
// steps are counted (ccount[0]: diagonal super-tiles, ccount[1]: the others).
template <int NCH, int NF, bool CULL>
// (two resident blocks per CU: the register budget is held to 256 per lane; NF 8 spills a few values)
__global__ __launch_bounds__(256, 2) void k_kmv_mixed_sym(const uint4* __restrict__ A, const uint4* __restrict__ B,
                                                       const float* __restrict__ v, int Rp, int E, int NS,
                                                       int64_t npad, double* __restrict__ part, int Rout,
                                                       const uint16_t* __restrict__ cmask, int64_t ngs,
                                                       unsigned long long* __restrict__ ccount) {
  static_assert(NF >= 2, "the pipeline needs two fragments per step");
  constexpr int KV = NCH * 4;
  constexpr int RS = KV + 1;
  // sources per LDS tile (two tiles, the column partials and the weights fit twice per CU)
  constexpr int TS = NCH == 1 ? 256 : (NCH == 2 ? 128 : 64);
  constexpr int SPT = TS / 16;
  constexpr int TPF = 512 / TS;              // tiles per FP64 fold of the row sums (every 512 sources)
  constexpr int NI = (TS * RS + 63) / 64;
  constexpr int NQ = (NI + 3) / 4;           // staging loads per wave and tile (wave w issues i = w, w + 4, ...)
  constexpr int SBU = NI * 64 + 16 * RS;
  constexpr int TM = 64 * NF;                // targets per target tile (4 waves x 16 NF)
  constexpr int VPER = 8 / NCH;
  __shared__ uint4 sb0[SBU], sb1[SBU];
  __shared__ float sv0[TS + 16], sv1[TS + 16];
  __shared__ float cb0[16][TS], cb1[16][TS];   // column partials per (wave, lane group) and source

  // triangle item of this block (XCD-contiguous order), column-major: column c holds r = 0 .. c, so the
  // blocks that run together on one XCD mostly share their source super-tile (L2 reuse)
  const int64_t nitems = (int64_t)NS * (NS + 1) / 2;
  const int64_t per = (nitems + 7) / 8;
  const int64_t item = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (item >= nitems) return;
  int c = (int)((sqrt(8.0 * (double)item + 1.0) - 1.0) / 2);
  if (c < 0) c = 0;
  if (c > NS - 1) c = NS - 1;
  auto col_start = [&](int64_t cc) { return cc * (cc + 1) / 2; };
  while (c > 0 && col_start(c) > item) --c;
  while (c + 1 < NS && col_start(c + 1) <= item) ++c;
  const int r = (int)(item - col_start(c));
  const bool diag = r == c;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r16 = lane & 15;
  const int kq = lane >> 4;
  const int64_t t0 = (int64_t)r * E, t1 = t0 + E < npad ? t0 + E : npad;
  const int64_t s0 = (int64_t)c * E, s1 = s0 + E < npad ? s0 + E : npad;
  const int ntile = (int)((s1 - s0) / TS);
  constexpr float kZero = 0.0f;

  bf16x8 a[NF][NCH];
  float vt[NF][4];
  double acc[NF][4];
  float a32[NF][4];

  // LDS slot i * 64 + lane of a tile holds chunk u of source rr, slot = RS rr + u (rows padded to RS chunks;
  // the pad chunk loads chunk 0 of its row and the slots past the tile chunk 0 of the tile's first source,
  // neither of which is read).  Wave w stages slots tid + 256 q (i = w + 4 q), so (rr, u) advance by
  // (256 / RS, 256 % RS) per load instead of being divided out again.
  auto issue = [&](uint4* dst, int64_t j0) {
    const uint4* src = B + j0 * KV;
    int t = tid;
    asm volatile("" : "+v"(t));   // recomputed per tile rather than held in registers across the tile loop
    int rr = t / RS, u = t - rr * RS;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = wave + 4 * q;
      if (i < NI) {
        const int uu = u == KV ? 0 : u;
        __builtin_amdgcn_global_load_lds(src + (rr < TS ? rr * KV + uu : 0), dst + i * 64, 16, 0, 0);
      }
      rr += 256 / RS;
      u += 256 % RS;
      if (u >= RS) {
        u -= RS;
        ++rr;
      }
    }
  };
  auto vload = [&](int64_t j0) -> float { return tid < TS ? v[(j0 + tid) * Rp] : kZero; };

  // one LDS tile: row sums into a32; with COL, per-step column partials into cb[wave][step * 16 + r16];
  // SKIP: bit st of sk set means step st is culled (its exp/FMA work skipped); without SKIP the step loop has
  // no branches (tiles with nothing to skip run the same code as the unculled kernel)
  auto compute = [&](const uint4* sb, const float* sv, float (*cb)[TS], auto colflag, auto skipflag, unsigned sk) {
    constexpr bool COL = decltype(colflag)::value;
    constexpr bool SKIP = decltype(skipflag)::value;
    bf16x8 b[NCH], bn[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) b[ch] = __builtin_bit_cast(bf16x8, sb[r16 * RS + ch * 4 + kq]);
    float vj = sv[r16];
    f32x4 q0 = f32x4{0.f, 0.f, 0.f, 0.f}, q1 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) q0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][ch], b[ch], q0, 0, 0, 0);
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) q1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][ch], b[ch], q1, 0, 0, 0);
#pragma unroll 2
    for (int st = 0; st < SPT; ++st) {
      const int rn = (st + 1) * 16 + r16;
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) bn[ch] = __builtin_bit_cast(bf16x8, sb[rn * RS + ch * 4 + kq]);
      const float vn = sv[rn];
      float cs = 0.f;   // one chain over the NF x 4 targets (dependent FMAs issue back to back)
      const bool skip = SKIP && ((sk >> st) & 1u);
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        f32x4 q2 = f32x4{0.f, 0.f, 0.f, 0.f};
        if (f + 2 < NF) {
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch)
            q2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f + 2 < NF ? f + 2 : 0][ch], b[ch], q2, 0, 0, 0);
        } else {
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch)
            q2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f + 2 - NF >= 0 ? f + 2 - NF : 0][ch], bn[ch], q2, 0,
                                                         0, 0);
        }
        if (!skip) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float ex = __builtin_amdgcn_exp2f(q0[e]);
            a32[f][e] = __builtin_fmaf(ex, vj, a32[f][e]);
            if (COL) cs = __builtin_fmaf(ex, vt[f][e], cs);
          }
        }
        q0 = q1;
        q1 = q2;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x002, COL ? VPER + 4 / NCH : VPER, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      if (COL) cb[wave * 4 + kq][st * 16 + r16] = cs;
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) b[ch] = bn[ch];
      vj = vn;
    }
  };

  // (target tile, source tile) pairs in one sequence, so the first source tile of the next target tile is
  // staged while the last one of the current target tile is evaluated
  auto run = [&](auto colflag) {
    constexpr bool COL = decltype(colflag)::value;
    const int ntt = (int)((t1 - t0) / TM);
    const int total = ntt * ntile;
    issue(sb0, s0);
    {
      const float v0 = vload(s0);
      if (tid < TS) sv0[tid] = v0;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    int64_t row0 = 0;
    unsigned long long nskip = 0;
    for (int k = 0; k < total; ++k) {
      const int tt = k / ntile;
      const int t = k - tt * ntile;
      const bool odd = k & 1;
      const bool more = k + 1 < total;
      const int tn = t + 1 == ntile ? 0 : t + 1;
      if (t == 0) {
        row0 = t0 + (int64_t)tt * TM + (int64_t)wave * 16 * NF;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch)
            a[f][ch] = __builtin_bit_cast(bf16x8, A[(row0 + 16 * f + r16) * KV + ch * 4 + kq]);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            if (COL) vt[f][e] = v[(row0 + 16 * f + kq * 4 + e) * Rp];
            acc[f][e] = 0.0;
            a32[f][e] = 0.0f;
          }
        }
      }
      float vr = 0.0f;
      if (more) {
        issue(odd ? sb0 : sb1, s0 + (int64_t)tn * TS);
        vr = vload(s0 + (int64_t)tn * TS);
      }
      // column partial of the earlier target tiles for this source tile, fetched under the tile's work
      double* dst = part + (int64_t)r * npad + s0 + (int64_t)t * TS + (tid < TS ? tid : 0);   // dense partials
      double prev = 0.0;
      if (COL && tid < TS && tt > 0) prev = *dst;
      unsigned sk = 0;
      if (CULL) {   // this wave's skip bits for the tile's steps (one scalar value per wave)
        const int64_t j0 = s0 + (int64_t)t * TS;
        const unsigned m16 = cmask[(row0 / (16 * NF)) * ngs + j0 / 256];
        sk = __builtin_amdgcn_readfirstlane((m16 >> ((j0 % 256) / 16)) & ((1u << SPT) - 1u));
        nskip += (unsigned long long)__builtin_popcount(sk);
      }
      if (!CULL || sk == 0) {
        compute(odd ? sb1 : sb0, odd ? sv1 : sv0, odd ? cb1 : cb0, colflag, std::false_type{}, 0u);
      } else if (sk == (1u << SPT) - 1u) {   // the whole tile is culled: its column partials are zero
        if (COL) {
          float (*cb)[TS] = odd ? cb1 : cb0;
#pragma unroll
          for (int st = 0; st < SPT; ++st) cb[wave * 4 + kq][st * 16 + r16] = 0.0f;
        }
      } else {
        compute(odd ? sb1 : sb0, odd ? sv1 : sv0, odd ? cb1 : cb0, colflag, std::true_type{}, sk);
      }
      if (t % TPF == TPF - 1 || t == ntile - 1) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            acc[f][e] += (double)a32[f][e];
            a32[f][e] = 0.0f;
          }
      }
      if (more && tid < TS) (odd ? sv0 : sv1)[tid] = vr;
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (COL && tid < TS) {
        float (*cb)[TS] = odd ? cb1 : cb0;
        float h[8];
#pragma unroll
        for (int g = 0; g < 8; ++g) h[g] = cb[2 * g][tid] + cb[2 * g + 1][tid];
        const float cs = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7]));
        *dst = prev + (double)cs;
      }
      if (t == ntile - 1) {   // row sums of this target tile -> part[c][rows]
        double* prow = part + (int64_t)c * npad + row0 + kq * 4;
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            double x = acc[f][e];
            x += __shfl_xor(x, 8);
            x += __shfl_xor(x, 4);
            x += __shfl_xor(x, 2);
            x += __shfl_xor(x, 1);
            if (r16 == 0) prow[16 * f + e] = x;
          }
      }
    }
    if (CULL && lane == 0 && nskip) atomicAdd(ccount + (diag ? 0 : 1), nskip);
  };
  if (diag) run(std::false_type{});
  else run(std::true_type{});
}

}  // namespace krr
