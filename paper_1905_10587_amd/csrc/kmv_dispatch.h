// Launch entry points of the per-precision kernel instantiations.
#pragma once

#include "kmv.h"

namespace krr {

struct KmvGrid {
  dim3 grid;
  int64_t src_len, n_src, mpad;
  int Rp, Rout;
  // When set, the launcher writes the kernel's resident blocks per CU here instead of launching.
  int* occ = nullptr;
  // symmetric form: super-tile edge and super-tiles per side (grid.x = 8 * ceil(NS (NS + 1) / 16))
  int E = 0, NS = 0;
  // FP64 matrix-core form writing a final result in place: rows >= m_store and columns >= n_store are not
  // stored (0: all padded rows, Rp columns)
  int64_t m_store = 0;
  int n_store = 0;
};

// FP64 / FP32 direct kernels: D in {2,3,4,6,8,16,32,64,128}, TM in {1,2,4} (D >= 32: TM 1),
// RC in {1,4,8}, DV in {0,2}; FP64 also RC in {16, 32} with TM 1, DV 0, D <= 16.  Return false if the
// combination is not instantiated.
bool launch_kmv_f64(int D, int TM, int RC, int DV, const KmvGrid& g, const double* xt, const double* xs,
                    const double* v, double neg_c, double* part, hipStream_t s);
// Symmetric FP64 square product of one column (D in {2, 4, 6, 8, 16}, TM in {2, 4}).
bool launch_kmv_f64_sym(int D, int TM, const KmvGrid& g, const double* x, const double* v, double neg_c,
                        double* part, hipStream_t s);
// The same with the cross term on the FP64 matrix cores (NFR in {2, 4}: 64 NFR targets per target tile);
// clamp false only when every pair's base-2 exponent is known to be >= -1020 (Staged::q_floor).
bool launch_kmv_f64_symm(int D, int NFR, bool clamp, const KmvGrid& g, const double* x, const double* v, double neg_c,
                         double* part, hipStream_t s);
bool kmv_f64_has_sym(int D);
// FP64 many-column product on the FP64 matrix cores: D <= 16 (instantiated D), NRG in {1, 2, 4, 8} groups
// of 16 columns per block (Rp a multiple of 16; the last block may be partly filled), K only.
bool launch_kmv_f64_mfma(int D, int NRG, const KmvGrid& g, const double* xt, const double* xs, const double* v,
                         double neg_c, double* part, hipStream_t s);
bool launch_kmv_f32(int D, int TM, int RC, int DV, const KmvGrid& g, const float* xt, const float* xs,
                    const float* v, double* part, hipStream_t s);
// MFMA kernel (one column per launch): NCH in {1,2,3,4,6,8,13,25}, NF in {1,2,4,8} (limited by NCH),
// DV in {0,2}.  form 0: plain; 1: software-pipelined; 2: pipelined with LDS-staged source tiles
// (forms 1 and 2: NCH <= 4, NF >= 2; all forms give identical results).
bool launch_kmv_mixed(int NCH, int NF, int DV, int form, const KmvGrid& g, const uint16_t* A,
                      const uint16_t* B, const float* v, int col, double* part, hipStream_t s);
int mixed_max_nf(int nch);
bool mixed_has_pp(int nch);
// Symmetric square product K(X, X) v, one column (NCH <= 4, NF in {4, 8}; NCH > 2: NF 4 only).
// cmask: skip masks of exact far-tile culling (points staged in spatial order), or nullptr.
bool launch_kmv_mixed_sym(int NCH, int NF, const KmvGrid& g, const uint16_t* A, const uint16_t* B,
                          const float* v, double* part, hipStream_t s, const uint16_t* cmask = nullptr);
// Block MVM (many right-hand sides): NCH in {1,2,3,4}, (NT, NRC) with NT * NRC <= 8, NS in {3, 6}.
// k32: the K.V contraction on v_mfma_f32_16x16x32_bf16 (32 sources per step) instead of 16x16x16.
bool launch_kmv_block(int NCH, int NT, int NRC, int NS, bool k32, const KmvGrid& g, const uint16_t* A,
                      const uint16_t* B, const uint16_t* Vh, const uint16_t* Vm, const uint16_t* Vl, double* part,
                      hipStream_t s);
// Shared-tile block MVM: 64 FW targets x 128 right-hand sides per block (V staged with a multiple of 32 columns),
// FW in {1, 2} fragments evaluated per wave.
// Staged-V block form (k_kmv_block32v): NCH in {1, 2, 3, 4}, NS in {3, 6}.
bool launch_kmv_block_vt(int NCH, int NS, const KmvGrid& g, const uint16_t* A, const uint16_t* B, const uint16_t* VT,
                         double* part, hipStream_t s);
bool launch_kmv_block_shared(int NCH, int NS, int FW, const KmvGrid& g, const uint16_t* A, const uint16_t* B,
                             const uint16_t* Vh, const uint16_t* Vm, const uint16_t* Vl, double* part, hipStream_t s);

}  // namespace krr
