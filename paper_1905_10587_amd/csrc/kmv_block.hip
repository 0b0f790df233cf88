// Block-MVM (many right-hand sides) kernel instantiations.
#include "kmv_dispatch.h"
#include "kmv_block_kernels.h"

namespace krr {

template <int NCH, int NT, int NRC, int NS>
static void gob32(const KmvGrid& g, const uint16_t* A, const uint16_t* B, const uint16_t* Vh, const uint16_t* Vm,
                  const uint16_t* Vl, double* part, hipStream_t s) {
  if (g.occ) {
    KRR_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(g.occ, k_kmv_block32<NCH, NT, NRC, NS>, 256, 0));
    return;
  }
  hipLaunchKernelGGL((k_kmv_block32<NCH, NT, NRC, NS>), g.grid, dim3(256), 0, s, reinterpret_cast<const uint4*>(A),
                     reinterpret_cast<const uint4*>(B), reinterpret_cast<const uint2*>(Vh),
                     reinterpret_cast<const uint2*>(Vm), reinterpret_cast<const uint2*>(Vl), g.Rp, g.src_len, g.n_src,
                     part, g.mpad, g.Rout);
}

template <int NCH, int NT, int NRC, int NS>
static void gob(const KmvGrid& g, const uint16_t* A, const uint16_t* B, const uint16_t* Vh, const uint16_t* Vm,
                const uint16_t* Vl, double* part, hipStream_t s) {
  if (g.occ) {
    KRR_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(g.occ, k_kmv_block<NCH, NT, NRC, NS>, 256, 0));
    return;
  }
  hipLaunchKernelGGL((k_kmv_block<NCH, NT, NRC, NS>), g.grid, dim3(256), 0, s, reinterpret_cast<const uint4*>(A),
                     reinterpret_cast<const uint4*>(B), reinterpret_cast<const uint2*>(Vh),
                     reinterpret_cast<const uint2*>(Vm), reinterpret_cast<const uint2*>(Vl), g.Rp, g.src_len, g.n_src,
                     part, g.mpad, g.Rout);
}

#define KRR_BNS(NCH, NT, NRC) \
  if (NS == 3 && !k32) { gob<NCH, NT, NRC, 3>(g, A, B, Vh, Vm, Vl, part, s); return true; } \
  if (NS == 6 && !k32) { gob<NCH, NT, NRC, 6>(g, A, B, Vh, Vm, Vl, part, s); return true; } \
  if (NS == 3 && k32) { gob32<NCH, NT, NRC, 3>(g, A, B, Vh, Vm, Vl, part, s); return true; } \
  if (NS == 6 && k32) { gob32<NCH, NT, NRC, 6>(g, A, B, Vh, Vm, Vl, part, s); return true; }
#define KRR_BTR(NCH)                                                                    \
  if (NT == 1 && NRC == 1) { KRR_BNS(NCH, 1, 1) } if (NT == 1 && NRC == 2) { KRR_BNS(NCH, 1, 2) } \
  if (NT == 1 && NRC == 4) { KRR_BNS(NCH, 1, 4) } if (NT == 1 && NRC == 8) { KRR_BNS(NCH, 1, 8) } \
  if (NT == 2 && NRC == 1) { KRR_BNS(NCH, 2, 1) } if (NT == 2 && NRC == 2) { KRR_BNS(NCH, 2, 2) } \
  if (NT == 2 && NRC == 4) { KRR_BNS(NCH, 2, 4) } if (NT == 4 && NRC == 1) { KRR_BNS(NCH, 4, 1) } \
  if (NT == 4 && NRC == 2) { KRR_BNS(NCH, 4, 2) }

template <int NCH, int NS, int FW>
static void gobs(const KmvGrid& g, const uint16_t* A, const uint16_t* B, const uint16_t* Vh, const uint16_t* Vm,
                 const uint16_t* Vl, double* part, hipStream_t s) {
  if (g.occ) {
    KRR_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(g.occ, k_kmv_block32s<NCH, NS, FW>, 256, 0));
    return;
  }
  hipLaunchKernelGGL((k_kmv_block32s<NCH, NS, FW>), g.grid, dim3(256), 0, s, reinterpret_cast<const uint4*>(A),
                     reinterpret_cast<const uint4*>(B), reinterpret_cast<const uint2*>(Vh),
                     reinterpret_cast<const uint2*>(Vm), reinterpret_cast<const uint2*>(Vl), g.Rp, g.src_len, g.n_src,
                     part, g.mpad, g.Rout);
}

template <int NCH, int NS, int NCTF>
static void gobv_tiles(const KmvGrid& g, const uint16_t* A, const uint16_t* B, const uint16_t* VT, double* part,
                       hipStream_t s) {
  if (g.occ) {
    KRR_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(g.occ, k_kmv_block32v<NCH, NS, NCTF>, 256, 0));
    return;
  }
  hipLaunchKernelGGL((k_kmv_block32v<NCH, NS, NCTF>), g.grid, dim3(256), 0, s, reinterpret_cast<const uint4*>(A),
                     reinterpret_cast<const uint4*>(B), reinterpret_cast<const uint4*>(VT), g.Rp, g.src_len, g.n_src,
                     part, g.mpad, g.Rout);
}

template <int NCH, int NS>
static void gobv(const KmvGrid& g, const uint16_t* A, const uint16_t* B, const uint16_t* VT, double* part,
                 hipStream_t s) {
  // static column-tile count: every block holds 128 columns when the padded count is a multiple of 128; one
  // block of 3 to 7 tiles covers 48 to 112 columns; otherwise the last block's count is read at run time
  const int nctt = g.Rp / 16;
  switch (nctt % 8 == 0 ? 8 : nctt < 8 ? nctt : 0) {
    case 8: gobv_tiles<NCH, NS, 8>(g, A, B, VT, part, s); break;
    case 7: gobv_tiles<NCH, NS, 7>(g, A, B, VT, part, s); break;
    case 6: gobv_tiles<NCH, NS, 6>(g, A, B, VT, part, s); break;
    case 5: gobv_tiles<NCH, NS, 5>(g, A, B, VT, part, s); break;
    case 4: gobv_tiles<NCH, NS, 4>(g, A, B, VT, part, s); break;
    case 3: gobv_tiles<NCH, NS, 3>(g, A, B, VT, part, s); break;
    default: gobv_tiles<NCH, NS, 0>(g, A, B, VT, part, s);
  }
}

bool launch_kmv_block_vt(int NCH, int NS, const KmvGrid& g, const uint16_t* A, const uint16_t* B, const uint16_t* VT,
                         double* part, hipStream_t s) {
#define KRR_BV(C)                                                                  \
  if (NCH == C) {                                                                  \
    if (NS == 3) gobv<C, 3>(g, A, B, VT, part, s);                                 \
    else gobv<C, 6>(g, A, B, VT, part, s);                                         \
    return true;                                                                   \
  }
  if (NS != 3 && NS != 6) return false;
  KRR_BV(1) KRR_BV(2) KRR_BV(3) KRR_BV(4)
#undef KRR_BV
  return false;
}

bool launch_kmv_block_shared(int NCH, int NS, int FW, const KmvGrid& g, const uint16_t* A, const uint16_t* B,
                             const uint16_t* Vh, const uint16_t* Vm, const uint16_t* Vl, double* part, hipStream_t s) {
#define KRR_BSH(C)                                                                     \
  if (NCH == C) {                                                                      \
    if (NS == 3 && FW == 1) gobs<C, 3, 1>(g, A, B, Vh, Vm, Vl, part, s);               \
    else if (NS == 3) gobs<C, 3, 2>(g, A, B, Vh, Vm, Vl, part, s);                     \
    else if (FW == 1) gobs<C, 6, 1>(g, A, B, Vh, Vm, Vl, part, s);                     \
    else gobs<C, 6, 2>(g, A, B, Vh, Vm, Vl, part, s);                                  \
    return true;                                                                       \
  }
  if ((NS != 3 && NS != 6) || (FW != 1 && FW != 2)) return false;
  KRR_BSH(1) KRR_BSH(2) KRR_BSH(3) KRR_BSH(4)
#undef KRR_BSH
  return false;
}

bool launch_kmv_block(int NCH, int NT, int NRC, int NS, bool k32, const KmvGrid& g, const uint16_t* A,
                      const uint16_t* B, const uint16_t* Vh, const uint16_t* Vm, const uint16_t* Vl, double* part,
                      hipStream_t s) {
  switch (NCH) {
    case 1: KRR_BTR(1) break;
    case 2: KRR_BTR(2) break;
    case 3: KRR_BTR(3) break;
    case 4: KRR_BTR(4) break;
  }
  return false;
}

}  // namespace krr
