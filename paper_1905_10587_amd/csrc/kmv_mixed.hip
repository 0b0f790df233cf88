// Split-BF16 MFMA kernel instantiations.
#include "kmv_dispatch.h"
#include "kmv_kernels.h"

namespace krr {

int mixed_max_nf(int nch) { return nch <= 2 ? 8 : nch <= 4 ? 4 : nch <= 8 ? 2 : 1; }

template <int NCH, int NF, int DV>
static void gom(const KmvGrid& g, const uint16_t* A, const uint16_t* B, const float* v, int col, double* part,
                hipStream_t s) {
  if (g.occ) {
    KRR_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(g.occ, k_kmv_mixed<NCH, NF, DV>, 256, 0));
    return;
  }
  hipLaunchKernelGGL((k_kmv_mixed<NCH, NF, DV>), g.grid, dim3(256), 0, s, reinterpret_cast<const uint4*>(A),
                     reinterpret_cast<const uint4*>(B), v, g.Rp, col, g.src_len, g.n_src, part, g.mpad, g.Rout,
                     col);
}

template <int NCH, int NF, int DV>
static void gop(const KmvGrid& g, const uint16_t* A, const uint16_t* B, const float* v, int col, double* part,
                hipStream_t s) {
  if (g.occ) {
    KRR_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(g.occ, k_kmv_mixed_pp<NCH, NF, DV>, 256, 0));
    return;
  }
  hipLaunchKernelGGL((k_kmv_mixed_pp<NCH, NF, DV>), g.grid, dim3(256), 0, s, reinterpret_cast<const uint4*>(A),
                     reinterpret_cast<const uint4*>(B), v, g.Rp, col, g.src_len, g.n_src, part, g.mpad, g.Rout,
                     col);
}

template <int NCH, int NF, int DV>
static void gol(const KmvGrid& g, const uint16_t* A, const uint16_t* B, const float* v, int col, double* part,
                hipStream_t s) {
  if (g.occ) {
    KRR_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(g.occ, k_kmv_mixed_lds<NCH, NF, DV>, 256, 0));
    return;
  }
  hipLaunchKernelGGL((k_kmv_mixed_lds<NCH, NF, DV>), g.grid, dim3(256), 0, s, reinterpret_cast<const uint4*>(A),
                     reinterpret_cast<const uint4*>(B), v, g.Rp, col, g.src_len, g.n_src, part, g.mpad, g.Rout,
                     col);
}

#define KRR_MDV(NCH, NF)                                                        \
  if (DV == 0) { gom<NCH, NF, 0>(g, A, B, v, col, part, s); return true; }   \
  if (DV == 2) { gom<NCH, NF, 2>(g, A, B, v, col, part, s); return true; }
#define KRR_PDV(NCH, NF)                                                        \
  if (DV == 0) { gop<NCH, NF, 0>(g, A, B, v, col, part, s); return true; }   \
  if (DV == 2) { gop<NCH, NF, 2>(g, A, B, v, col, part, s); return true; }
#define KRR_LDV(NCH, NF)                                                        \
  if (DV == 0) { gol<NCH, NF, 0>(g, A, B, v, col, part, s); return true; }   \
  if (DV == 2) { gol<NCH, NF, 2>(g, A, B, v, col, part, s); return true; }
#define KRR_LNF8(NCH) \
  if (NF == 2) { KRR_LDV(NCH, 2) } if (NF == 4) { KRR_LDV(NCH, 4) } if (NF == 8) { KRR_LDV(NCH, 8) }
#define KRR_LNF4(NCH) \
  if (NF == 2) { KRR_LDV(NCH, 2) } if (NF == 4) { KRR_LDV(NCH, 4) }
#define KRR_NF8(NCH) \
  if (NF == 1) { KRR_MDV(NCH, 1) } if (NF == 2) { KRR_MDV(NCH, 2) } if (NF == 4) { KRR_MDV(NCH, 4) } if (NF == 8) { KRR_MDV(NCH, 8) }
#define KRR_NF4(NCH) \
  if (NF == 1) { KRR_MDV(NCH, 1) } if (NF == 2) { KRR_MDV(NCH, 2) } if (NF == 4) { KRR_MDV(NCH, 4) }
#define KRR_NF2(NCH) \
  if (NF == 1) { KRR_MDV(NCH, 1) } if (NF == 2) { KRR_MDV(NCH, 2) }
#define KRR_NF1(NCH) \
  if (NF == 1) { KRR_MDV(NCH, 1) }
#define KRR_PNF8(NCH) \
  if (NF == 2) { KRR_PDV(NCH, 2) } if (NF == 4) { KRR_PDV(NCH, 4) } if (NF == 8) { KRR_PDV(NCH, 8) }
#define KRR_PNF4(NCH) \
  if (NF == 2) { KRR_PDV(NCH, 2) } if (NF == 4) { KRR_PDV(NCH, 4) }

bool mixed_has_pp(int nch) { return nch <= 4; }

template <int NCH, int NF>
static void gos(const KmvGrid& g, const uint16_t* A, const uint16_t* B, const float* v, double* part,
                const uint16_t* cmask, hipStream_t s) {
  if (g.occ) {
    KRR_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(g.occ, k_kmv_mixed_sym<NCH, NF, false>, 256, 0));
    return;
  }
  const int64_t ngs = g.mpad / 256;
  if (cmask)
    hipLaunchKernelGGL((k_kmv_mixed_sym<NCH, NF, true>), g.grid, dim3(256), 0, s, reinterpret_cast<const uint4*>(A),
                       reinterpret_cast<const uint4*>(B), v, g.Rp, g.E, g.NS, g.mpad, part, g.Rout, cmask, ngs,
                       cull_counters());
  else
    hipLaunchKernelGGL((k_kmv_mixed_sym<NCH, NF, false>), g.grid, dim3(256), 0, s, reinterpret_cast<const uint4*>(A),
                       reinterpret_cast<const uint4*>(B), v, g.Rp, g.E, g.NS, g.mpad, part, g.Rout, nullptr, ngs,
                       nullptr);
}

bool launch_kmv_mixed_sym(int NCH, int NF, const KmvGrid& g, const uint16_t* A, const uint16_t* B,
                          const float* v, double* part, hipStream_t s, const uint16_t* cmask) {
  switch (NCH * 16 + NF) {
    case 1 * 16 + 4: gos<1, 4>(g, A, B, v, part, cmask, s); return true;
    case 1 * 16 + 8: gos<1, 8>(g, A, B, v, part, cmask, s); return true;
    case 2 * 16 + 4: gos<2, 4>(g, A, B, v, part, cmask, s); return true;
    case 2 * 16 + 8: gos<2, 8>(g, A, B, v, part, cmask, s); return true;
    case 3 * 16 + 4: gos<3, 4>(g, A, B, v, part, cmask, s); return true;
    case 4 * 16 + 4: gos<4, 4>(g, A, B, v, part, cmask, s); return true;
  }
  return false;
}

bool launch_kmv_mixed(int NCH, int NF, int DV, int form, const KmvGrid& g, const uint16_t* A,
                      const uint16_t* B, const float* v, int col, double* part, hipStream_t s) {
  if (form == 2) {
    switch (NCH) {
      case 1: KRR_LNF8(1) break;
      case 2: KRR_LNF8(2) break;
      case 3: KRR_LNF4(3) break;
      case 4: KRR_LNF4(4) break;
    }
    return false;
  }
  if (form == 1) {
    switch (NCH) {
      case 1: KRR_PNF8(1) break;
      case 2: KRR_PNF8(2) break;
      case 3: KRR_PNF4(3) break;
      case 4: KRR_PNF4(4) break;
    }
    return false;
  }
  switch (NCH) {
    case 1: KRR_NF8(1) break;
    case 2: KRR_NF8(2) break;
    case 3: KRR_NF4(3) break;
    case 4: KRR_NF4(4) break;
    case 6: KRR_NF2(6) break;
    case 8: KRR_NF2(8) break;
    case 13: KRR_NF1(13) break;
    case 25: KRR_NF1(25) break;
  }
  return false;
}

}  // namespace krr
