// FP64 direct-difference kernel instantiations.
#include "kmv_dispatch.h"
#include "kmv_kernels.h"

namespace krr {

template <int D, int TM, int RC, int DV, int TSX = 0>
static void go64(const KmvGrid& g, const double* xt, const double* xs, const double* v, double neg_c,
                 double* part, hipStream_t s) {
  if (g.occ) {
    KRR_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(g.occ, k_kmv_f64<D, TM, RC, DV, TSX>, 256, 0));
    return;
  }
  hipLaunchKernelGGL((k_kmv_f64<D, TM, RC, DV, TSX>), g.grid, dim3(256), 0, s, xt, xs, v, g.Rp, g.src_len,
                     g.n_src, neg_c, part, g.mpad, g.Rout);
}

#define KRR_DV(D, TM, RC)                                   \
  if (DV == 0) { go64<D, TM, RC, 0>(g, xt, xs, v, neg_c, part, s); return true; } \
  if (DV == 2) { go64<D, TM, RC, 2>(g, xt, xs, v, neg_c, part, s); return true; }
#define KRR_RC(D, TM) \
  if (RC == 1) { KRR_DV(D, TM, 1) } if (RC == 4) { KRR_DV(D, TM, 4) } if (RC == 8) { KRR_DV(D, TM, 8) }
// TM 1 also has wide column chunks (RC 16, 32; K only) for many right-hand sides
#define KRR_RCW(D) \
  KRR_RC(D, 1) \
  if (RC == 16 && DV == 0) { go64<D, 1, 16, 0>(g, xt, xs, v, neg_c, part, s); return true; } \
  if (RC == 32 && DV == 0) { go64<D, 1, 32, 0>(g, xt, xs, v, neg_c, part, s); return true; }
#define KRR_TM3(D) \
  if (TM == 1) { KRR_RCW(D) } if (TM == 2) { KRR_RC(D, 2) } if (TM == 4) { KRR_RC(D, 4) }
#define KRR_TM1(D) \
  if (TM == 1) { KRR_RC(D, 1) }

template <int D, int TM>
static void go64s(const KmvGrid& g, const double* x, const double* v, double neg_c, double* part, hipStream_t s) {
  if (g.occ) {
    KRR_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(g.occ, k_kmv_f64_sym<D, TM>, 256, 0));
    return;
  }
  hipLaunchKernelGGL((k_kmv_f64_sym<D, TM>), g.grid, dim3(256), 0, s, x, v, g.Rp, neg_c, g.E, g.NS, g.mpad, part,
                     g.Rout);
}

template <int D, int NRG>
static void go64m(const KmvGrid& g, const double* xt, const double* xs, const double* v, double neg_c,
                  double* part, hipStream_t s) {
  if (g.occ) {
    KRR_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(g.occ, k_kmv_f64_mfma_db<D, NRG>, 256, 0));
    return;
  }
  hipLaunchKernelGGL((k_kmv_f64_mfma_db<D, NRG>), g.grid, dim3(256), 0, s, xt, xs, v, g.Rp, g.src_len, g.n_src,
                     neg_c, part, g.mpad, g.Rout, g.m_store > 0 ? g.m_store : g.mpad,
                     g.n_store > 0 ? g.n_store : g.Rp);
}

bool launch_kmv_f64_mfma(int D, int NRG, const KmvGrid& g, const double* xt, const double* xs, const double* v,
                         double neg_c, double* part, hipStream_t s) {
#define KRR_M64(DD)                                                               \
  if (D == DD) {                                                                  \
    if (NRG == 1) { go64m<DD, 1>(g, xt, xs, v, neg_c, part, s); return true; }    \
    if (NRG == 2) { go64m<DD, 2>(g, xt, xs, v, neg_c, part, s); return true; }    \
    if (NRG == 4) { go64m<DD, 4>(g, xt, xs, v, neg_c, part, s); return true; }    \
    if (NRG == 6) { go64m<DD, 6>(g, xt, xs, v, neg_c, part, s); return true; }    \
    if (NRG == 8) { go64m<DD, 8>(g, xt, xs, v, neg_c, part, s); return true; }    \
  }
  KRR_M64(2) KRR_M64(3) KRR_M64(4) KRR_M64(6) KRR_M64(8) KRR_M64(16)
#undef KRR_M64
  return false;
}

template <int D, int NFR, bool CLAMP>
static void go64sm(const KmvGrid& g, const double* x, const double* v, double neg_c, double* part, hipStream_t s) {
  if (g.occ) {
    KRR_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(g.occ, k_kmv_f64_symm<D, NFR, CLAMP>, 256, 0));
    return;
  }
  hipLaunchKernelGGL((k_kmv_f64_symm<D, NFR, CLAMP>), g.grid, dim3(256), 0, s, x, v, g.Rp, neg_c, g.E, g.NS, g.mpad,
                     part, g.Rout);
}

bool launch_kmv_f64_symm(int D, int NFR, bool clamp, const KmvGrid& g, const double* x, const double* v,
                         double neg_c, double* part, hipStream_t s) {
#define KRR_SM64(DD)                                                                                 \
  if (D == DD) {                                                                                     \
    if (NFR == 2) { clamp ? go64sm<DD, 2, true>(g, x, v, neg_c, part, s)                             \
                          : go64sm<DD, 2, false>(g, x, v, neg_c, part, s); return true; }            \
    if (NFR == 4) { clamp ? go64sm<DD, 4, true>(g, x, v, neg_c, part, s)                             \
                          : go64sm<DD, 4, false>(g, x, v, neg_c, part, s); return true; }            \
  }
  KRR_SM64(2) KRR_SM64(4) KRR_SM64(6) KRR_SM64(8) KRR_SM64(16)
#undef KRR_SM64
  return false;
}

bool kmv_f64_has_sym(int D) { return D == 2 || D == 4 || D == 6 || D == 8 || D == 16; }

bool launch_kmv_f64_sym(int D, int TM, const KmvGrid& g, const double* x, const double* v, double neg_c,
                        double* part, hipStream_t s) {
#define KRR_S64(DD)                                                   \
  if (D == DD) {                                                      \
    if (TM == 2) { go64s<DD, 2>(g, x, v, neg_c, part, s); return true; } \
    if (TM == 4) { go64s<DD, 4>(g, x, v, neg_c, part, s); return true; } \
  }
  KRR_S64(2) KRR_S64(4) KRR_S64(6) KRR_S64(8) KRR_S64(16)
#undef KRR_S64
  return false;
}

bool launch_kmv_f64(int D, int TM, int RC, int DV, const KmvGrid& g, const double* xt, const double* xs,
                    const double* v, double neg_c, double* part, hipStream_t s) {
  if (g.src_len % 256 != 0) {   // short source splits: the 64-point tile form (one column, K only, D <= 16)
    if (TM != 1 || RC != 1 || DV != 0 || g.src_len % 64 != 0) return false;
    switch (D) {
      case 2: go64<2, 1, 1, 0, 64>(g, xt, xs, v, neg_c, part, s); return true;
      case 3: go64<3, 1, 1, 0, 64>(g, xt, xs, v, neg_c, part, s); return true;
      case 4: go64<4, 1, 1, 0, 64>(g, xt, xs, v, neg_c, part, s); return true;
      case 6: go64<6, 1, 1, 0, 64>(g, xt, xs, v, neg_c, part, s); return true;
      case 8: go64<8, 1, 1, 0, 64>(g, xt, xs, v, neg_c, part, s); return true;
      case 16: go64<16, 1, 1, 0, 64>(g, xt, xs, v, neg_c, part, s); return true;
    }
    return false;
  }
  switch (D) {
    case 2: KRR_TM3(2) break;
    case 3: KRR_TM3(3) break;
    case 4: KRR_TM3(4) break;
    case 6: KRR_TM3(6) break;
    case 8: KRR_TM3(8) break;
    case 16: KRR_TM3(16) break;
    case 32: KRR_TM1(32) break;
    case 64: KRR_TM1(64) break;
    case 128: KRR_TM1(128) break;
  }
  return false;
}

}  // namespace krr
