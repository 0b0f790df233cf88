// Dense products of the preconditioner on the FP64 matrix cores (see gemm.h): the Nystrom core
// M = W^T W (Algorithm 3, last step), its inverse G = L^{-T} L^{-1} from the Cholesky factor
// (Eq. chol_factor), and the two skinny products of Algorithm 4 for several right-hand sides,
// T = W^T X and (X - W Z) diag(1/beta).
//
// Tiles: a block of four waves owns a 128 x BN tile of C; every wave a WR x WC sub-tile held as
// (WR/16) x (WC/16) accumulators of v_mfma_f64_16x16x4_f64.  The contraction dimension streams through
// LDS 16 at a time, double buffered: the next 16 are loaded into registers while the current ones are
// contracted.  MFMA operand layouts (gfx950): the A operand of lane l is element (row l % 16, k l / 16),
// the B operand element (k l / 16, column l % 16); result element e of lane l is (row 4 e + l / 16,
// column l % 16).
#include "gemm.h"

#include <algorithm>

namespace krr {

typedef double f64x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kBM = 128;   // tile rows (the A^T B form: columns of A)
constexpr int kTK = 16;    // contraction step staged in LDS
constexpr int kLdsStride = kBM + 1;   // LDS row stride in doubles (odd: staggered banks for the transposed stores)

template <int BN>
struct TileShape {
  static constexpr int WR = BN == 128 ? 64 : 32;    // wave tile rows
  static constexpr int WC = BN == 128 ? 64 : BN;    // wave tile columns
  static constexpr int WAVES_R = kBM / WR;          // waves along the rows
  static constexpr int TT = WR / 16, TU = WC / 16;  // MFMA tiles per wave
  static_assert((kBM / WR) * (BN / WC) == 4, "four waves per block");
};

template <typename T>
__device__ __forceinline__ double ld(const T* p) { return (double)*p; }

// Contract one LDS stage: As[kk][row], Bs[kk][col] (16 x 128 / 16 x BN).
template <int BN>
__device__ __forceinline__ void contract_stage(const double (*As)[kLdsStride], const double (*Bs)[kLdsStride],
                                               int wr, int wc, int r16, int kq,
                                               f64x4 (&acc)[TileShape<BN>::TT][TileShape<BN>::TU]) {
  using S = TileShape<BN>;
#pragma unroll
  for (int ks = 0; ks < kTK; ks += 4) {
    double a[S::TT], b[S::TU];
#pragma unroll
    for (int t = 0; t < S::TT; ++t) a[t] = As[ks + kq][wr * S::WR + t * 16 + r16];
#pragma unroll
    for (int u = 0; u < S::TU; ++u) b[u] = Bs[ks + kq][wc * S::WC + u * 16 + r16];
#pragma unroll
    for (int t = 0; t < S::TT; ++t)
#pragma unroll
      for (int u = 0; u < S::TU; ++u) acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[u], acc[t][u], 0, 0, 0);
  }
}

// part[s] (ka x kb) = sum over rows [s * chunk, (s + 1) * chunk) of A[i, a] B[i, b].
// SYM: B == A and only tiles ta <= tb are computed (blockIdx.x enumerates the upper block triangle).
template <typename TA, typename TB, int BN, bool SYM>
__global__ __launch_bounds__(256) void k_gemm_tn(const TA* __restrict__ A, int64_t lda, const TB* __restrict__ B,
                                                 int64_t ldb, int64_t rows, int ka, int kb, int64_t chunk, int ntb,
                                                 double* __restrict__ part) {
  using S = TileShape<BN>;
  __shared__ double As[2][kTK][kLdsStride];
  __shared__ double Bs[2][kTK][kLdsStride];
  int ta, tb;
  if (SYM) {
    const int id = blockIdx.x;
    int c = (int)((sqrt(8.0 * id + 1.0) - 1.0) / 2.0);
    while (c * (c + 1) / 2 > id) --c;
    while ((c + 1) * (c + 2) / 2 <= id) ++c;
    tb = c;
    ta = id - c * (c + 1) / 2;
  } else {
    ta = blockIdx.x / ntb;
    tb = blockIdx.x % ntb;
  }
  const int a0 = ta * kBM, b0 = tb * BN;
  const int64_t i_beg = (int64_t)blockIdx.y * chunk;
  const int64_t i_end = i_beg + chunk < rows ? i_beg + chunk : rows;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int wr = wave % S::WAVES_R, wc = wave / S::WAVES_R;
  f64x4 acc[S::TT][S::TU];
#pragma unroll
  for (int t = 0; t < S::TT; ++t)
#pragma unroll
    for (int u = 0; u < S::TU; ++u) acc[t][u] = f64x4{0.0, 0.0, 0.0, 0.0};
  constexpr int NA = kTK * kBM / 256, NB = kTK * BN / 256;
  double ra[NA], rb[NB];
  auto load = [&](int64_t i0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int e = tid + 256 * j, r = e / kBM, c = e % kBM;
      ra[j] = (i0 + r < i_end && a0 + c < ka) ? ld(A + (i0 + r) * lda + a0 + c) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int e = tid + 256 * j, r = e / BN, c = e % BN;
      rb[j] = (i0 + r < i_end && b0 + c < kb) ? ld(B + (i0 + r) * ldb + b0 + c) : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int e = tid + 256 * j;
      As[buf][e / kBM][e % kBM] = ra[j];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int e = tid + 256 * j;
      Bs[buf][e / BN][e % BN] = rb[j];
    }
  };
  const int nsteps = i_end > i_beg ? (int)((i_end - i_beg + kTK - 1) / kTK) : 0;
  if (nsteps > 0) {
    load(i_beg);
    store(0);
    __syncthreads();
    for (int st = 0; st < nsteps; ++st) {
      const int buf = st & 1;
      if (st + 1 < nsteps) load(i_beg + (int64_t)(st + 1) * kTK);
      contract_stage<BN>(As[buf], Bs[buf], wr, wc, r16, kq, acc);
      if (st + 1 < nsteps) store(buf ^ 1);
      __syncthreads();
    }
  }
  double* P = part + (int64_t)blockIdx.y * ka * kb;
#pragma unroll
  for (int t = 0; t < S::TT; ++t)
#pragma unroll
    for (int u = 0; u < S::TU; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int a = a0 + wr * S::WR + t * 16 + 4 * e + kq;
        const int b = b0 + wc * S::WC + u * 16 + r16;
        if (a < ka && b < kb) P[(int64_t)a * kb + b] = acc[t][u][e];
      }
}

// C[a, b] = sum_s part[s][a, b] in split order; sym: element (min, max) of the upper block triangle.
__global__ void k_sum_parts(const double* __restrict__ part, int S, int ka, int kb, bool sym,
                            double* __restrict__ C, int64_t ldc) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)ka * kb) return;
  int a = (int)(t / kb), b = (int)(t % kb);
  const int64_t off = sym ? (int64_t)std::min(a, b) * kb + std::max(a, b) : t;
  double s = 0.0;
  for (int p = 0; p < S; ++p) s += part[(int64_t)p * ka * kb + off];
  C[(int64_t)a * ldc + b] = s;
}

// C (m x nb) = A (m x k) B (k x nb); EPI: C = (X - A B) diag(scale).
template <typename TA, int BN, bool EPI>
__global__ __launch_bounds__(256) void k_gemm_nn(const TA* __restrict__ A, int64_t lda, const double* __restrict__ B,
                                                 int64_t ldb, int64_t m, int k, int nb, double* __restrict__ C,
                                                 int64_t ldc, const double* __restrict__ X, int64_t ldx,
                                                 const double* __restrict__ scale) {
  using S = TileShape<BN>;
  __shared__ double As[2][kTK][kLdsStride];   // transposed: As[kk][row]
  __shared__ double Bs[2][kTK][kLdsStride];
  const int64_t m0 = (int64_t)blockIdx.x * kBM;
  const int n0 = blockIdx.y * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int wr = wave % S::WAVES_R, wc = wave / S::WAVES_R;
  f64x4 acc[S::TT][S::TU];
#pragma unroll
  for (int t = 0; t < S::TT; ++t)
#pragma unroll
    for (int u = 0; u < S::TU; ++u) acc[t][u] = f64x4{0.0, 0.0, 0.0, 0.0};
  constexpr int NA = kTK * kBM / 256, NB = kTK * BN / 256;
  double ra[NA], rb[NB];
  auto load = [&](int k0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {   // 16 consecutive threads read 16 consecutive k of one row
      const int e = tid + 256 * j, r = e / kTK, kk = e % kTK;
      ra[j] = (m0 + r < m && k0 + kk < k) ? ld(A + (m0 + r) * lda + k0 + kk) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int e = tid + 256 * j, kk = e / BN, c = e % BN;
      rb[j] = (k0 + kk < k && n0 + c < nb) ? B[(int64_t)(k0 + kk) * ldb + n0 + c] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int e = tid + 256 * j;
      As[buf][e % kTK][e / kTK] = ra[j];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int e = tid + 256 * j;
      Bs[buf][e / BN][e % BN] = rb[j];
    }
  };
  const int nsteps = (k + kTK - 1) / kTK;
  load(0);
  store(0);
  __syncthreads();
  for (int st = 0; st < nsteps; ++st) {
    const int buf = st & 1;
    if (st + 1 < nsteps) load((st + 1) * kTK);
    contract_stage<BN>(As[buf], Bs[buf], wr, wc, r16, kq, acc);
    if (st + 1 < nsteps) store(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < S::TT; ++t)
#pragma unroll
    for (int u = 0; u < S::TU; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = m0 + wr * S::WR + t * 16 + 4 * e + kq;
        const int j = n0 + wc * S::WC + u * 16 + r16;
        if (i < m && j < nb) {
          const double v = acc[t][u][e];
          C[i * ldc + j] = EPI ? (X[i * ldx + j] - v) * scale[j] : v;
        }
      }
}

int pick_bn(int nb) { return nb <= 16 ? 16 : nb <= 32 ? 32 : nb <= 64 ? 64 : 128; }

// Row split of the A^T B forms: enough blocks to fill the part (about eight per CU), rows per split a
// multiple of the LDS step, the partial tiles kept under about 1 GB.
int64_t tn_splits(int64_t tiles, int64_t rows, int64_t ka, int64_t kb, int64_t& chunk) {
  int64_t S = std::max<int64_t>(1, ceil_div(2048, tiles));
  S = std::min<int64_t>(S, std::max<int64_t>(1, ceil_div(rows, 512)));
  S = std::min<int64_t>(S, std::max<int64_t>(1, ((int64_t)1 << 27) / std::max<int64_t>(1, ka * kb)));
  chunk = round_up(ceil_div(rows, S), kTK);
  return ceil_div(rows, chunk);
}

template <typename TA, typename TB, int BN, bool SYM>
void launch_tn(const TA* A, int64_t lda, const TB* B, int64_t ldb, int64_t rows, int ka, int kb, double* C,
               int64_t ldc, hipStream_t s, DevBuf<double>* ws) {
  const int nta = (int)ceil_div(ka, kBM), ntb = (int)ceil_div(kb, BN);
  const int64_t tiles = SYM ? (int64_t)nta * (nta + 1) / 2 : (int64_t)nta * ntb;
  int64_t chunk = 0;
  const int64_t S = tn_splits(tiles, rows, ka, kb, chunk);
  DevBuf<double> own;
  DevBuf<double>& part = ws ? *ws : own;
  if (part.n < (size_t)S * ka * kb) part.alloc((size_t)S * ka * kb, s);
  hipLaunchKernelGGL((k_gemm_tn<TA, TB, BN, SYM>), dim3((unsigned)tiles, (unsigned)S), dim3(256), 0, s, A, lda, B,
                     ldb, rows, ka, kb, chunk, ntb, part.p);
  KRR_LAUNCH_CHECK();
  const int64_t tot = (int64_t)ka * kb;
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, part.p, (int)S, ka, kb, SYM,
                     C, ldc);
  KRR_LAUNCH_CHECK();
}

template <typename TA, int BN>
void launch_nn(const TA* A, int64_t lda, const double* B, int64_t ldb, int64_t m, int k, int nb, double* C,
               int64_t ldc, const double* X, int64_t ldx, const double* scale, hipStream_t s) {
  const dim3 grid((unsigned)ceil_div(m, kBM), (unsigned)ceil_div(nb, BN));
  if (X)
    hipLaunchKernelGGL((k_gemm_nn<TA, BN, true>), grid, dim3(256), 0, s, A, lda, B, ldb, m, k, nb, C, ldc, X, ldx,
                       scale);
  else
    hipLaunchKernelGGL((k_gemm_nn<TA, BN, false>), grid, dim3(256), 0, s, A, lda, B, ldb, m, k, nb, C, ldc, X, ldx,
                       scale);
  KRR_LAUNCH_CHECK();
}

}  // namespace

template <typename TA, typename TB>
void gemm_tn(const TA* A, int64_t lda, const TB* B, int64_t ldb, int64_t rows, int ka, int kb, double* C,
             int64_t ldc, hipStream_t s, DevBuf<double>* ws) {
  KRR_REQUIRE(rows >= 1 && ka >= 1 && kb >= 1, "gemm_tn: empty operand");
  switch (pick_bn(kb)) {
    case 16: launch_tn<TA, TB, 16, false>(A, lda, B, ldb, rows, ka, kb, C, ldc, s, ws); break;
    case 32: launch_tn<TA, TB, 32, false>(A, lda, B, ldb, rows, ka, kb, C, ldc, s, ws); break;
    case 64: launch_tn<TA, TB, 64, false>(A, lda, B, ldb, rows, ka, kb, C, ldc, s, ws); break;
    default: launch_tn<TA, TB, 128, false>(A, lda, B, ldb, rows, ka, kb, C, ldc, s, ws); break;
  }
}

template <typename TA>
void syrk_tn(const TA* A, int64_t lda, int64_t rows, int k, double* C, int64_t ldc, hipStream_t s) {
  KRR_REQUIRE(rows >= 1 && k >= 1, "syrk_tn: empty operand");
  launch_tn<TA, TA, 128, true>(A, lda, A, lda, rows, k, k, C, ldc, s, nullptr);
}

template <typename TA>
void gemm_nn(const TA* A, int64_t lda, const double* B, int64_t ldb, int64_t m, int k, int nb, double* C,
             int64_t ldc, const double* X, int64_t ldx, const double* scale, hipStream_t s) {
  KRR_REQUIRE(m >= 1 && k >= 1 && nb >= 1, "gemm_nn: empty operand");
  KRR_REQUIRE((X == nullptr) == (scale == nullptr), "gemm_nn: X and scale go together");
  switch (pick_bn(nb)) {
    case 16: launch_nn<TA, 16>(A, lda, B, ldb, m, k, nb, C, ldc, X, ldx, scale, s); break;
    case 32: launch_nn<TA, 32>(A, lda, B, ldb, m, k, nb, C, ldc, X, ldx, scale, s); break;
    case 64: launch_nn<TA, 64>(A, lda, B, ldb, m, k, nb, C, ldc, X, ldx, scale, s); break;
    default: launch_nn<TA, 128>(A, lda, B, ldb, m, k, nb, C, ldc, X, ldx, scale, s); break;
  }
}

template void gemm_tn<double, double>(const double*, int64_t, const double*, int64_t, int64_t, int, int, double*,
                                      int64_t, hipStream_t, DevBuf<double>*);
template void gemm_tn<float, double>(const float*, int64_t, const double*, int64_t, int64_t, int, int, double*,
                                     int64_t, hipStream_t, DevBuf<double>*);
template void syrk_tn<double>(const double*, int64_t, int64_t, int, double*, int64_t, hipStream_t);
template void syrk_tn<float>(const float*, int64_t, int64_t, int, double*, int64_t, hipStream_t);
template void gemm_nn<double>(const double*, int64_t, const double*, int64_t, int64_t, int, int, double*, int64_t,
                              const double*, int64_t, const double*, hipStream_t);
template void gemm_nn<float>(const float*, int64_t, const double*, int64_t, int64_t, int, int, double*, int64_t,
                             const double*, int64_t, const double*, hipStream_t);

}  // namespace krr
