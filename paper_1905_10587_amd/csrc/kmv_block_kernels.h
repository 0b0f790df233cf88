// Kernel templates of the block (many right-hand sides) Gaussian kernel MVM on the BF16 matrix cores,
// included by the block translation unit only.  See kmv.hip for the overview.
#pragma once

#include "kmv_kernels.h"

namespace krr {

// ------------------------------------------------------------------ block MVM (many right-hand sides)
// U[i, r] = sum_j P_ij V[j, r] with P_ij = exp2(q_ij) computed on the fly.  The cross term is issued with
// the sources as MFMA rows, so the 16 x 16 q tile lands in the lane layout of the A operand of
// v_mfma_f32_16x16x16_bf16 (lane l: target l%16, sources (l/16)*4 + e): the exp'd tile feeds the second
// contraction straight from registers.  P and V are split into BF16 parts (NS = 3: hi/lo with
// hi*hi + hi*lo + lo*hi; NS = 6: hi/mid/lo with the six products down to 2^-24).  Each wave owns NT
// target fragments of 16 and the block covers 16 * NRC right-hand sides (grid.z walks the rest).
// V is staged as BF16 parts in groups of four sources: V4[((j/4) * Rp + r) * 4 + j%4].
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));



template <int NCH, int NT, int NRC, int NS>
__global__ __launch_bounds__(256) void k_kmv_block(const uint4* __restrict__ A, const uint4* __restrict__ B,
                                                   const uint2* __restrict__ Vh, const uint2* __restrict__ Vm,
                                                   const uint2* __restrict__ Vl, int Rp, int64_t src_len,
                                                   int64_t n_src, double* __restrict__ part, int64_t mpad,
                                                   int Rout) {
  constexpr int KV = NCH * 4;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r16 = lane & 15;
  const int kq = lane >> 4;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * NT);
  const int rbase = blockIdx.z * 16 * NRC;
  const int64_t jb = (int64_t)blockIdx.y * src_len;
  const int64_t je = jb + src_len < n_src ? jb + src_len : n_src;

  bf16x8 tg[NT][NCH];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) tg[t][ch] = __builtin_bit_cast(bf16x8, A[(row0 + 16 * t + r16) * KV + ch * 4 + kq]);

  double acc[NT][NRC][4];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int c = 0; c < NRC; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[t][c][e] = 0.0;

  for (int64_t j0 = jb; j0 < je; j0 += 256) {
    f32x4 a32[NT][NRC];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int c = 0; c < NRC; ++c) a32[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t j = j0; j < j0 + 256; j += 16) {
      bf16x8 sf[NCH];
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) sf[ch] = __builtin_bit_cast(bf16x8, B[(j + r16) * KV + ch * 4 + kq]);
      // exp'd tiles, split into BF16 parts, in the A-operand layout of the 16x16x16 MFMA
      bf16x4 ph[NT], pm[NT], pl[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        f32x4 q = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) q = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sf[ch], tg[t][ch], q, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) {   // round-to-nearest-even splits (v_cvt_pk_bf16_f32, two per instruction)
          const float p = __builtin_amdgcn_exp2f(q[e]);
          ph[t][e] = (__bf16)p;
          const float r1 = p - (float)ph[t][e];
          pm[t][e] = (__bf16)r1;
          if (NS == 6) pl[t][e] = (__bf16)(r1 - (float)pm[t][e]);
        }
      }
      const int64_t vg = (j >> 2) + kq;   // group of four sources
#pragma unroll
      for (int c = 0; c < NRC; ++c) {
        const int64_t vi = vg * Rp + rbase + 16 * c + r16;
        const bf16x4 vh = __builtin_bit_cast(bf16x4, Vh[vi]);
        const bf16x4 vm = __builtin_bit_cast(bf16x4, Vm[vi]);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          a32[t][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ph[t], vh, a32[t][c], 0, 0, 0);
          a32[t][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ph[t], vm, a32[t][c], 0, 0, 0);
          a32[t][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pm[t], vh, a32[t][c], 0, 0, 0);
        }
        if (NS == 6) {
          const bf16x4 vl = __builtin_bit_cast(bf16x4, Vl[vi]);
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            a32[t][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ph[t], vl, a32[t][c], 0, 0, 0);
            a32[t][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pl[t], vh, a32[t][c], 0, 0, 0);
            a32[t][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pm[t], vm, a32[t][c], 0, 0, 0);
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int c = 0; c < NRC; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[t][c][e] += (double)a32[t][c][e];
  }
  // lane l holds targets (l/16)*4 + e of each fragment for right-hand side l%16 of each chunk
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = row0 + 16 * t + kq * 4 + e;
      double* prow = part + ((int64_t)blockIdx.y * mpad + i) * Rout;
#pragma unroll
      for (int c = 0; c < NRC; ++c) prow[rbase + 16 * c + r16] = acc[t][c][e];
    }
}

}  // namespace krr

namespace krr {


// Block MVM, K = 32 form: the K.V contraction uses v_mfma_f32_16x16x32_bf16 on 32 sources at a time.
// Two 16-source cross-term tiles give each lane 8 exp'd values (sources j+4g+e and j+16+4g+e,
// g = lane/16, e = 0..3); the K index of the second MFMA is relabelled so that lane l's eight A slots
// are exactly those sources, and its B slots read the same two groups of four sources from V4.
template <int NCH, int NT, int NRC, int NS>
__global__ __launch_bounds__(256) void k_kmv_block32(const uint4* __restrict__ A, const uint4* __restrict__ B,
                                                     const uint2* __restrict__ Vh, const uint2* __restrict__ Vm,
                                                     const uint2* __restrict__ Vl, int Rp, int64_t src_len,
                                                     int64_t n_src, double* __restrict__ part, int64_t mpad,
                                                     int Rout) {
  constexpr int KV = NCH * 4;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r16 = lane & 15;
  const int kq = lane >> 4;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * NT);
  const int rbase = blockIdx.z * 16 * NRC;
  const int64_t jb = (int64_t)blockIdx.y * src_len;
  const int64_t je = jb + src_len < n_src ? jb + src_len : n_src;

  bf16x8 tg[NT][NCH];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) tg[t][ch] = __builtin_bit_cast(bf16x8, A[(row0 + 16 * t + r16) * KV + ch * 4 + kq]);

  double acc[NT][NRC][4];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int c = 0; c < NRC; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[t][c][e] = 0.0;

  for (int64_t j0 = jb; j0 < je; j0 += 256) {
    f32x4 a32[NT][NRC];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int c = 0; c < NRC; ++c) a32[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t j = j0; j < j0 + 256; j += 32) {
      bf16x8 sa[NCH], sb[NCH];
      const uint4* bp = B + (j + r16) * KV + kq;   // one address per step, constant offsets after it
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        sa[ch] = __builtin_bit_cast(bf16x8, bp[ch * 4]);
        sb[ch] = __builtin_bit_cast(bf16x8, bp[16 * KV + ch * 4]);
      }
      bf16x8 ph[NT], pm[NT], pl[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        f32x4 qa = {0.f, 0.f, 0.f, 0.f}, qb = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          qa = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sa[ch], tg[t][ch], qa, 0, 0, 0);
          qb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sb[ch], tg[t][ch], qb, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 8; e += 2) {   // round-to-nearest-even splits, two values per v_cvt_pk_bf16_f32
          const f32x2 p = {__builtin_amdgcn_exp2f(e < 4 ? qa[e] : qb[e - 4]),
                           __builtin_amdgcn_exp2f(e < 4 ? qa[e + 1] : qb[e - 3])};
          const bf16x2 h = __builtin_convertvector(p, bf16x2);
          const f32x2 r1 = p - __builtin_convertvector(h, f32x2);
          const bf16x2 m = __builtin_convertvector(r1, bf16x2);
          ph[t][e] = h[0]; ph[t][e + 1] = h[1];
          pm[t][e] = m[0]; pm[t][e + 1] = m[1];
          if (NS == 6) {
            const bf16x2 lo = __builtin_convertvector(r1 - __builtin_convertvector(m, f32x2), bf16x2);
            pl[t][e] = lo[0]; pl[t][e + 1] = lo[1];
          }
        }
      }
      // the lane's two groups of four sources, (j/4 + kq) and four groups further
      const int64_t ga = (j >> 2) + kq;
      const uint2* vha = Vh + ga * Rp + rbase + r16;
      const uint2* vma = Vm + ga * Rp + rbase + r16;
      const int64_t g4 = 4 * (int64_t)Rp;
#pragma unroll
      for (int c = 0; c < NRC; ++c) {
        const uint2 h0 = vha[16 * c], h1 = vha[g4 + 16 * c];
        const uint2 m0 = vma[16 * c], m1 = vma[g4 + 16 * c];
        const bf16x8 vh = __builtin_bit_cast(bf16x8, uint4{h0.x, h0.y, h1.x, h1.y});
        const bf16x8 vm = __builtin_bit_cast(bf16x8, uint4{m0.x, m0.y, m1.x, m1.y});
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          a32[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ph[t], vh, a32[t][c], 0, 0, 0);
          a32[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ph[t], vm, a32[t][c], 0, 0, 0);
          a32[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pm[t], vh, a32[t][c], 0, 0, 0);
        }
        if (NS == 6) {
          const uint2* vla = Vl + ga * Rp + rbase + r16;
          const uint2 l0 = vla[16 * c], l1 = vla[g4 + 16 * c];
          const bf16x8 vl = __builtin_bit_cast(bf16x8, uint4{l0.x, l0.y, l1.x, l1.y});
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            a32[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ph[t], vl, a32[t][c], 0, 0, 0);
            a32[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pl[t], vh, a32[t][c], 0, 0, 0);
            a32[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pm[t], vm, a32[t][c], 0, 0, 0);
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int c = 0; c < NRC; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[t][c][e] += (double)a32[t][c][e];
  }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = row0 + 16 * t + kq * 4 + e;
      double* prow = part + ((int64_t)blockIdx.y * mpad + i) * Rout;
#pragma unroll
      for (int c = 0; c < NRC; ++c) prow[rbase + 16 * c + r16] = acc[t][c][e];
    }
}


// Block MVM, shared-tile form: a block covers 64 FW targets (4 FW fragments of 16) and 128 right-hand sides
// (grid.z walks the rest); wave w evaluates the cross term and exp2 of its FW fragments only, splits them into
// BF16 parts and stores them in LDS in the A-operand layout of the K.V MFMA, and after one barrier every wave
// contracts all 4 FW fragments with its own 32 right-hand sides.  Every V value a wave loads feeds 4 FW
// fragments, so FW = 2 halves the V traffic per pair of FW = 1.  The columns are padded to a multiple of
// 32 only: a wave whose 32 columns lie beyond the padded count still evaluates its fragment for the others
// but loads, contracts and stores nothing.  The exp/split work is done once per
// block instead of once per 32-column group.  Accumulation order per (fragment, column group) is that of
// k_kmv_block32<NCH, 4, 2, NS>.  With two-part splits, one fragment per wave and up to three K chunks the
// kernel fits three waves per SIMD (at most 168 registers, no spills; 170 and two waves without the hint):
// at d = 6, R = 128 a product then runs 1-9% faster than k_kmv_block32<2, 4, 2, 3> (two machines), where the
// two had tied.
template <int NCH, int NS, int FW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NS == 3 && FW == 1 && NCH <= 3 ? 3 : 1)))
void k_kmv_block32s(const uint4* __restrict__ A, const uint4* __restrict__ B, const uint2* __restrict__ Vh,
                    const uint2* __restrict__ Vm, const uint2* __restrict__ Vl, int Rp, int64_t src_len,
                    int64_t n_src, double* __restrict__ part, int64_t mpad, int Rout) {
  constexpr int KV = NCH * 4;
  constexpr int NT = 4 * FW, NRC = 2, NP = NS == 6 ? 3 : 2;
  __shared__ uint4 ps[2][NT][NP][64];   // exp'd fragments, double buffered: [step parity][fragment][part][lane]
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15;
  const int kq = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * (16 * NT);
  const int rbase = blockIdx.z * 128 + wave * 16 * NRC;
  const bool live = rbase < Rp;   // wave-uniform: Rp is a multiple of 32
  const int64_t jb = (int64_t)blockIdx.y * src_len;
  const int64_t je = jb + src_len < n_src ? jb + src_len : n_src;

  bf16x8 tg[FW][NCH];
#pragma unroll
  for (int f = 0; f < FW; ++f)
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
      tg[f][ch] = __builtin_bit_cast(bf16x8, A[(row0 + 16 * (wave * FW + f) + r16) * KV + ch * 4 + kq]);

  double acc[NT][NRC][4];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int c = 0; c < NRC; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[t][c][e] = 0.0;

  int buf = 0;
  for (int64_t j0 = jb; j0 < je; j0 += 256) {
    f32x4 a32[NT][NRC];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int c = 0; c < NRC; ++c) a32[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t j = j0; j < j0 + 256; j += 32) {
      // this wave's V values for the step, loaded first so that they arrive while the tile is computed
      const int64_t ga = (j >> 2) + kq;
      const int64_t g4 = 4 * (int64_t)Rp;
      bf16x8 vh[NRC], vm[NRC], vl[NRC];
      if (live) {
        const uint2* vha = Vh + ga * Rp + rbase + r16;
        const uint2* vma = Vm + ga * Rp + rbase + r16;
#pragma unroll
        for (int c = 0; c < NRC; ++c) {
          const uint2 h0 = vha[16 * c], h1 = vha[g4 + 16 * c];
          const uint2 m0 = vma[16 * c], m1 = vma[g4 + 16 * c];
          vh[c] = __builtin_bit_cast(bf16x8, uint4{h0.x, h0.y, h1.x, h1.y});
          vm[c] = __builtin_bit_cast(bf16x8, uint4{m0.x, m0.y, m1.x, m1.y});
          if (NS == 6) {
            const uint2* vla = Vl + ga * Rp + rbase + r16;
            const uint2 l0 = vla[16 * c], l1 = vla[g4 + 16 * c];
            vl[c] = __builtin_bit_cast(bf16x8, uint4{l0.x, l0.y, l1.x, l1.y});
          }
        }
      }
      const uint4* bp = B + (j + r16) * KV + kq;
#pragma unroll
      for (int f = 0; f < FW; ++f) {   // this wave's fragments: cross term, exp2, BF16 splits -> LDS
        f32x4 qa = {0.f, 0.f, 0.f, 0.f}, qb = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          qa = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, bp[ch * 4]), tg[f][ch], qa, 0, 0, 0);
          qb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, bp[16 * KV + ch * 4]), tg[f][ch],
                                                      qb, 0, 0, 0);
        }
        bf16x8 ph, pm, pl;
#pragma unroll
        for (int e = 0; e < 8; e += 2) {   // round-to-nearest-even splits, two values per v_cvt_pk_bf16_f32
          const f32x2 p = {__builtin_amdgcn_exp2f(e < 4 ? qa[e] : qb[e - 4]),
                           __builtin_amdgcn_exp2f(e < 4 ? qa[e + 1] : qb[e - 3])};
          const bf16x2 h = __builtin_convertvector(p, bf16x2);
          const f32x2 r1 = p - __builtin_convertvector(h, f32x2);
          const bf16x2 m = __builtin_convertvector(r1, bf16x2);
          ph[e] = h[0]; ph[e + 1] = h[1];
          pm[e] = m[0]; pm[e + 1] = m[1];
          if (NS == 6) {
            const bf16x2 lo = __builtin_convertvector(r1 - __builtin_convertvector(m, f32x2), bf16x2);
            pl[e] = lo[0]; pl[e + 1] = lo[1];
          }
        }
        ps[buf][wave * FW + f][0][lane] = __builtin_bit_cast(uint4, ph);
        ps[buf][wave * FW + f][1][lane] = __builtin_bit_cast(uint4, pm);
        if (NS == 6) ps[buf][wave * FW + f][2][lane] = __builtin_bit_cast(uint4, pl);
      }
      __syncthreads();   // the other buffer is rewritten only after the next barrier
      if (live) {
#pragma unroll
      for (int c = 0; c < NRC; ++c) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const bf16x8 ph = __builtin_bit_cast(bf16x8, ps[buf][t][0][lane]);
          const bf16x8 pm = __builtin_bit_cast(bf16x8, ps[buf][t][1][lane]);
          a32[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ph, vh[c], a32[t][c], 0, 0, 0);
          a32[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ph, vm[c], a32[t][c], 0, 0, 0);
          a32[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pm, vh[c], a32[t][c], 0, 0, 0);
        }
        if (NS == 6) {
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const bf16x8 ph = __builtin_bit_cast(bf16x8, ps[buf][t][0][lane]);
            const bf16x8 pm = __builtin_bit_cast(bf16x8, ps[buf][t][1][lane]);
            const bf16x8 pl = __builtin_bit_cast(bf16x8, ps[buf][t][2][lane]);
            a32[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ph, vl[c], a32[t][c], 0, 0, 0);
            a32[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pl, vh[c], a32[t][c], 0, 0, 0);
            a32[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pm, vm[c], a32[t][c], 0, 0, 0);
          }
        }
      }
      }
      buf ^= 1;
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int c = 0; c < NRC; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[t][c][e] += (double)a32[t][c][e];
  }
  if (!live) return;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = row0 + 16 * t + kq * 4 + e;
      double* prow = part + ((int64_t)blockIdx.y * mpad + i) * Rout;
#pragma unroll
      for (int c = 0; c < NRC; ++c) prow[rbase + 16 * c + r16] = acc[t][c][e];
    }
}


// Block MVM, staged-V form: a block covers 64 targets (wave w owns fragment w) and up to 128 right-hand sides
// (grid.z walks the rest).  Each wave evaluates the cross term, exp2 and BF16 split of its own fragment and
// contracts it with every column of the block, so no wave waits for another's exp'd tile; what the four waves
// share is the step's V tile (and the cross term's source fragments), which the block moves into LDS with
// direct global->LDS loads one 32-source step ahead (double buffered), one barrier per step.  V is staged in
// the B-operand lane layout of v_mfma_f32_16x16x32_bf16 (VT: per 32-source step, 16-column tile and part,
// 64 lanes x 8 BF16 values, lane r16 + 16 kq holding column r16 and sources {4kq + e, 16 + 4kq + e}), so a
// tile is a contiguous run of the staged array.  Accumulation order per (target, column) is that of
// k_kmv_block32s: the NS products of a step in the same order, FP32 over 256 sources, then FP64.
// NCTF > 0: every block holds NCTF column tiles (the padded column count a multiple of 128 with NCTF = 8, or
// NCTF tiles in all, fewer than eight), so the contraction and the V staging have static trip counts and the
// compiler can issue a step's V reads ahead of their products instead of branching per tile and waiting on
// each read.  NCTF = 0: the count is read at run time (a last block of fewer columns).
// Chunk swizzle of a staged source row of KV chunks in LDS: the 16 rows a lane group reads at one chunk land
// in distinct banks (rows 16 + r carry the swizzle of row r).  The staging lambda writes the same expression
// out: a lambda of a kernel that calls a device function leaves the kernel without its host launch stub.
template <int KV>
__device__ __forceinline__ int blk_sw(int row) {
  return KV == 8 ? (row >> 1) & 7 : KV == 16 ? row & 15 : (row >> 2) & 3;
}

template <int NCH, int NS, int NCTF>
__global__ __launch_bounds__(256) void k_kmv_block32v(const uint4* __restrict__ A, const uint4* __restrict__ B,
                                                      const uint4* __restrict__ VT, int Rb, int64_t src_len,
                                                      int64_t n_src, double* __restrict__ part, int64_t mpad,
                                                      int Rout) {
  constexpr int KV = NCH * 4;
  constexpr int NP = NS == 6 ? 3 : 2;     // BF16 parts of V and of the exp'd tile
  constexpr int NIS = 32 * KV / 64;       // 64-lane staging loads per step for the sources
  __shared__ uint4 vs0[8 * NP * 64], vs1[8 * NP * 64];   // V tiles, double buffered: [column tile x part][lane]
  __shared__ uint4 ss0[NIS * 64], ss1[NIS * 64];         // source rows: [row x KV + (chunk ^ blk_sw(row))]

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r16 = lane & 15;
  const int kq = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * 64 + wave * 16;
  const int nctt = Rb / 16;                           // column tiles of the staged V
  const int ct0 = blockIdx.z * 8;
  // this block's column tiles (block-uniform; a static trip count when NCTF > 0)
  const int nct = NCTF > 0 ? NCTF : nctt - ct0 < 8 ? nctt - ct0 : 8;
  const int nvi = nct * NP;                           // 64-lane staging loads of V per step
  const int64_t jb = (int64_t)blockIdx.y * src_len;
  const int64_t je = jb + src_len < n_src ? jb + src_len : n_src;
  const int nsteps = (int)((je - jb) / 32);

  bf16x8 tg[NCH];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) tg[ch] = __builtin_bit_cast(bf16x8, A[(row0 + r16) * KV + ch * 4 + kq]);
  double acc[8][4];
  f32x4 a32[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    a32[c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[c][e] = 0.0;
  }

  // staging of step st: V tiles (VT is contiguous per step and column tile) and the sources' split rows
  // (LDS slot row x KV + position holds chunk position ^ blk_sw(row))
  auto issue = [&](uint4* vdst, uint4* sdst, int st) {
    const uint4* vsrc = VT + ((int64_t)(jb / 32 + st) * nctt + ct0) * NP * 64;
    for (int i = wave; i < nvi; i += 4) __builtin_amdgcn_global_load_lds(vsrc + i * 64 + lane, vdst + i * 64, 16, 0, 0);
    const uint4* bsrc = B + (jb + 32 * (int64_t)st) * KV;
    for (int i = wave; i < NIS; i += 4) {
      const int slot = i * 64 + lane;
      const int rr = slot / KV, pos = slot - rr * KV;
      const int swr = KV == 8 ? (rr >> 1) & 7 : KV == 16 ? rr & 15 : (rr >> 2) & 3;   // blk_sw<KV>(rr)
      __builtin_amdgcn_global_load_lds(bsrc + rr * KV + (pos ^ swr), sdst + i * 64, 16, 0, 0);
    }
  };

  // residual of a split part: p - h[0] as the BF16 dot product p + (-1) h[0] + 0 h[1] (v_dot2_f32_bf16, one
  // instruction per value instead of a widening and a subtraction; exact, p - h[0] being an FP32 number).
  // The two weight pairs {-1, 0} and {0, -1} are held in registers: as an inline constant of the packed
  // operand the compiler's encoding of {-1, 0} does not reach the instruction as that pair.
  int nw0 = 0xBF80, nw1 = (int)0xBF800000u;
  asm volatile("" : "+v"(nw0), "+v"(nw1));
  const bf16x2 neg0 = __builtin_bit_cast(bf16x2, nw0), neg1 = __builtin_bit_cast(bf16x2, nw1);

  if (nsteps > 0) issue(vs0, ss0, 0);
  for (int st = 0; st < nsteps; ++st) {
    const int cur = st & 1;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();   // step st staged by every wave; step st - 1's buffer no longer read
    if (st + 1 < nsteps) {
      if (cur) issue(vs0, ss0, st + 1);
      else issue(vs1, ss1, st + 1);
    }
    const uint4* vsc = cur ? vs1 : vs0;
    const uint4* ssc = cur ? ss1 : ss0;
    // this wave's fragment: cross term (sources as MFMA rows), exp2, BF16 parts in the A-operand layout
    bf16x8 sa[NCH], sb[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const int pos = (ch * 4 + kq) ^ blk_sw<KV>(r16);
      sa[ch] = __builtin_bit_cast(bf16x8, ssc[r16 * KV + pos]);
      sb[ch] = __builtin_bit_cast(bf16x8, ssc[(16 + r16) * KV + pos]);
    }
    // NCTF > 0: the V operands of the first PF column tiles are read now, behind the cross term and the exp;
    // each later tile's are read PF tiles ahead of its products (a ring of PF + 1), so no product waits on
    // LDS.  PF = 1 where a second tile in flight would cost the third wave per SIMD (above 168 registers).
    constexpr int PF = NS == 3 && NCH == 4 ? 1 : 2;
    bf16x8 vr[PF + 1][NP];
    if (NCTF > 0) {
#pragma unroll
      for (int c = 0; c < PF && c < NCTF; ++c)
#pragma unroll
        for (int p = 0; p < NP; ++p) vr[c][p] = __builtin_bit_cast(bf16x8, vsc[(c * NP + p) * 64 + lane]);
      __builtin_amdgcn_sched_barrier(0);
    }
    f32x4 qa = {0.f, 0.f, 0.f, 0.f}, qb = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      qa = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sa[ch], tg[ch], qa, 0, 0, 0);
      qb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sb[ch], tg[ch], qb, 0, 0, 0);
    }
    bf16x8 ph, pm, pl;
#pragma unroll
    for (int e = 0; e < 8; e += 2) {   // round-to-nearest-even splits, two values per v_cvt_pk_bf16_f32
      const f32x2 p = {__builtin_amdgcn_exp2f(e < 4 ? qa[e] : qb[e - 4]),
                       __builtin_amdgcn_exp2f(e < 4 ? qa[e + 1] : qb[e - 3])};
      const bf16x2 h = __builtin_convertvector(p, bf16x2);
      const f32x2 r1 = {__builtin_amdgcn_fdot2_f32_bf16(h, neg0, p[0], false),
                        __builtin_amdgcn_fdot2_f32_bf16(h, neg1, p[1], false)};
      const bf16x2 m = __builtin_convertvector(r1, bf16x2);
      ph[e] = h[0]; ph[e + 1] = h[1];
      pm[e] = m[0]; pm[e + 1] = m[1];
      if (NS == 6) {
        const f32x2 r2 = {__builtin_amdgcn_fdot2_f32_bf16(m, neg0, r1[0], false),
                          __builtin_amdgcn_fdot2_f32_bf16(m, neg1, r1[1], false)};
        const bf16x2 lo = __builtin_convertvector(r2, bf16x2);
        pl[e] = lo[0]; pl[e + 1] = lo[1];
      }
    }
    // contraction with the block's column tiles
    if (NCTF > 0) {
#pragma unroll
      for (int c = 0; c < NCTF; ++c) {
        if (c + PF < NCTF) {
#pragma unroll
          for (int p = 0; p < NP; ++p)
            vr[(c + PF) % (PF + 1)][p] = __builtin_bit_cast(bf16x8, vsc[((c + PF) * NP + p) * 64 + lane]);
        }
        __builtin_amdgcn_sched_barrier(0);
        const bf16x8* v = vr[c % (PF + 1)];
        a32[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ph, v[0], a32[c], 0, 0, 0);
        a32[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ph, v[1], a32[c], 0, 0, 0);
        a32[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pm, v[0], a32[c], 0, 0, 0);
        if (NS == 6) {
          a32[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ph, v[NP - 1], a32[c], 0, 0, 0);
          a32[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pl, v[0], a32[c], 0, 0, 0);
          a32[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pm, v[1], a32[c], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (c < nct) {
        const bf16x8 vh = __builtin_bit_cast(bf16x8, vsc[(c * NP + 0) * 64 + lane]);
        const bf16x8 vm = __builtin_bit_cast(bf16x8, vsc[(c * NP + 1) * 64 + lane]);
        a32[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ph, vh, a32[c], 0, 0, 0);
        a32[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ph, vm, a32[c], 0, 0, 0);
        a32[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pm, vh, a32[c], 0, 0, 0);
        if (NS == 6) {
          const bf16x8 vl = __builtin_bit_cast(bf16x8, vsc[(c * NP + 2) * 64 + lane]);
          a32[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ph, vl, a32[c], 0, 0, 0);
          a32[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pl, vh, a32[c], 0, 0, 0);
          a32[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pm, vm, a32[c], 0, 0, 0);
        }
      }
    }
    }
    if ((st & 7) == 7 || st + 1 == nsteps) {   // FP64 fold every 256 sources
#pragma unroll
      for (int c = 0; c < (NCTF > 0 ? NCTF : 8); ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          acc[c][e] += (double)a32[c][e];
          a32[c][e] = 0.0f;
        }
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t i = row0 + kq * 4 + e;
    double* prow = part + ((int64_t)blockIdx.y * mpad + i) * Rout + ct0 * 16 + r16;
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (c < nct) prow[16 * c] = acc[c][e];
  }
}

}  // namespace krr
