// Exact Gaussian kernel MVM kernels for gfx950.
//
//   U[i, c] = sum_j exp(-||t_i - s_j||^2 / eps) V[j, c]          (Sec. 1 Eq. 1; Sec. 2.4 Eq. dscrt_gt with eps = h^2)
//   K'  :    sum_j (D2_ij/eps) exp(-D2_ij/eps) V[j, c]             (eps dK/deps, for the gradient path)
//
// Three arithmetic forms:
//   FP64  direct differences; 2^q split as 2^rint(q) * 2^f, 2^f by a degree-10 near-minimax polynomial.
//   FP32  direct differences on coordinates pre-scaled by sqrt(log2 e / eps), hardware exp2.
//   MIXED the exp2 argument q_ij = -log2(e) ||t_i - s_j||^2 / eps comes straight out of one
//         v_mfma_f32_16x16x32_bf16 per 32-wide K chunk: both operands are 3-way BF16 splits of
//         the centred coordinates (hi/mid/lo, six cross products) plus the split row norms, so the
//         MFMA's FP32 accumulation yields q without any VALU work; the VALU then does only
//         exp2 and one FMA with v per pair.
// Many right-hand sides: the exp'd tile is itself an MFMA operand.  MIXED and FP32 split it into BF16
// parts and contract with split-BF16 V on v_mfma_f32_16x16x32_bf16 (block kernels); FP64 contracts it on
// v_mfma_f64_16x16x4_f64 (k_kmv_f64_mfma_db).  Square one-column products have symmetric forms (MIXED and
// FP64) that evaluate each pair once for both of its rows.
// Sources are split across the grid's y dimension; every block writes FP64 partial sums which a
// finishing kernel adds in a fixed order (deterministic), together with the ridge term.
#include "anchors.h"
#include "kmv.h"
#include "kmv_dispatch.h"

#include <algorithm>
#include <cctype>
#include <map>
#include <mutex>
#include <sstream>

namespace krr {

// ------------------------------------------------------------------ dims / variants
int padded_dim(int d) {
  static const int widths[] = {2, 3, 4, 6, 8, 16, 32, 64, 128};   // instantiated kernel widths
  for (int w : widths)
    if (d <= w) return w;
  return -1;
}
int mixed_chunks(int d) {
  static const int chunks[] = {1, 2, 3, 4, 6, 8, 13, 25};            // instantiated chunk counts
  const int need = (int)ceil_div(6 * d + 6, 32);
  for (int c : chunks)
    if (need <= c) return c;
  return -1;
}

// ------------------------------------------------------------------ staging kernels
__global__ void k_point_sum(const double* __restrict__ X, int64_t n, int d, double* __restrict__ out) {
  // one block per dimension, fixed-order tree reduction
  __shared__ double red[256];
  const int k = blockIdx.x;
  double s = 0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += X[i * d + k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = red[0] / (double)n;
}

__global__ void k_zero_tail(double* p, int from, int to) {
  int i = from + threadIdx.x;
  if (i < to) p[i] = 0.0;
}

void point_mean(const double* X, int64_t n, int d, int dpad, double* center, hipStream_t s) {
  hipLaunchKernelGGL(k_point_sum, dim3(d), dim3(256), 0, s, X, n, d, center);
  KRR_LAUNCH_CHECK();
  if (dpad > d) {
    hipLaunchKernelGGL(k_zero_tail, dim3(1), dim3(128), 0, s, center, d, dpad);
    KRR_LAUNCH_CHECK();
  }
}

// FP64 copy, translated by center when given (the kernel is translation invariant; centred coordinates keep
// the norms, and so the cancellation of the matrix-core form, small)
__global__ void k_stage_f64(const double* __restrict__ X, int64_t n, int d, int64_t npad, int dpad,
                            const double* __restrict__ center, double* __restrict__ out) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= npad * dpad) return;
  int64_t i = idx / dpad;
  int k = (int)(idx % dpad);
  out[idx] = (i < n && k < d) ? X[i * d + k] - (center ? center[k] : 0.0) : 0.0;
}

__global__ void k_stage_f32(const double* __restrict__ X, int64_t n, int d, int64_t npad, int dpad,
                            const double* __restrict__ center, double scale, float* __restrict__ out) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= npad * dpad) return;
  int64_t i = idx / dpad;
  int k = (int)(idx % dpad);
  out[idx] = (i < n && k < d) ? (float)((X[i * d + k] - center[k]) * scale) : 0.0f;
}

__device__ __forceinline__ uint16_t bf16_rn(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}
__device__ __forceinline__ double bf16_to_double(uint16_t h) {
  return (double)__uint_as_float(((uint32_t)h) << 16);
}
// x = h + m + l with each part a BF16 number; the residual of each step is exact in FP64.
__device__ __forceinline__ void split3(double x, uint16_t& h, uint16_t& m, uint16_t& l) {
  h = bf16_rn((float)x);
  double r = x - bf16_to_double(h);
  m = bf16_rn((float)r);
  r -= bf16_to_double(m);
  l = bf16_rn((float)r);
}

// Split vectors for the MFMA cross term.  z = x - center, c = log2(e)/eps.
//   target side a: [2c z]h [2c z]h [2c z]m [2c z]h [2c z]l [2c z]m | nh nm nl 1 1 1 | 0...
//   source side b: [z]h    [z]m    [z]h    [z]l    [z]h    [z]m    | 1 1 1 nh nm nl | 0...
// with n = -c ||z||^2 split into three parts.  sum_k a_k b_k = -c ||z_t - z_s||^2 up to the
// dropped m*l, l*m, l*l products (relative size below 2^-24).
__global__ void k_stage_split(const double* __restrict__ X, int64_t n, int d, int64_t npad, int ka,
                              const double* __restrict__ center, double c, int side,
                              const int64_t* __restrict__ perm, uint16_t* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  uint16_t* o = out + i * ka;
  for (int k = 0; k < ka; ++k) o[k] = 0;
  if (i >= n) return;
  const int64_t src = perm ? perm[i] : i;   // staged point i is the caller's point src
  const uint16_t one = 0x3F80;   // 1.0 in BF16
  double nz = 0;
  for (int k = 0; k < d; ++k) {
    double z = X[src * d + k] - center[k];
    nz += z * z;
    double zz = side == 0 ? 2.0 * c * z : z;
    uint16_t h, m, l;
    split3(zz, h, m, l);
    if (side == 0) {
      o[0 * d + k] = h; o[1 * d + k] = h; o[2 * d + k] = m;
      o[3 * d + k] = h; o[4 * d + k] = l; o[5 * d + k] = m;
    } else {
      o[0 * d + k] = h; o[1 * d + k] = m; o[2 * d + k] = h;
      o[3 * d + k] = l; o[4 * d + k] = h; o[5 * d + k] = m;
    }
  }
  uint16_t h, m, l;
  split3(-c * nz, h, m, l);
  const int base = 6 * d;
  if (side == 0) {
    o[base + 0] = h; o[base + 1] = m; o[base + 2] = l;
    o[base + 3] = one; o[base + 4] = one; o[base + 5] = one;
  } else {
    o[base + 0] = one; o[base + 1] = one; o[base + 2] = one;
    o[base + 3] = h; o[base + 4] = m; o[base + 5] = l;
  }
}

void spatial_order(Staged& st, const double* X, const double* center, hipStream_t s);

void stage_points(Staged& st, const double* X, int64_t n, int d, double eps, int prec,
                  const double* center, bool as_target, bool as_source, hipStream_t s, bool sort) {
  st.n = n;
  st.d = d;
  st.npad = round_up(n, kRowPad);
  st.dpad = padded_dim(d);
  st.prec = prec;
  st.eps = eps;
  KRR_REQUIRE(st.dpad > 0, "d exceeds KRR_MAX_D");
  const int64_t tot = st.npad * st.dpad;
  const int blk = 256;
  if (prec == KRR_FP64) {
    st.x64.alloc(tot, s);
    hipLaunchKernelGGL(k_stage_f64, dim3(ceil_div(tot, blk)), dim3(blk), 0, s, X, n, d, st.npad, st.dpad, center,
                       st.x64.p);
    KRR_LAUNCH_CHECK();
    // the box of the points bounds every squared distance by diag2 and the staged squared norms by max2
    std::vector<double> lo(d), hi(d), ctr(d, 0.0);
    if (center) KRR_CHECK_HIP(hipMemcpyAsync(ctr.data(), center, sizeof(double) * d, hipMemcpyDeviceToHost, s));
    bounding_box(X, n, d, lo.data(), hi.data(), s);   // synchronises the stream
    double diag2 = 0.0, max2 = 0.0;
    for (int k = 0; k < d; ++k) {
      diag2 += (hi[k] - lo[k]) * (hi[k] - lo[k]);
      const double a = lo[k] - ctr[k], b = hi[k] - ctr[k];
      max2 += std::max(a * a, b * b);
    }
    const double c = kLog2e / eps;
    st.q_floor = c * diag2 <= 1000.0 && c * max2 <= 1e10;
  } else {
    if (prec == KRR_FP32) {
      st.x32.alloc(tot, s);
      const double scale = std::sqrt(kLog2e / eps);
      hipLaunchKernelGGL(k_stage_f32, dim3(ceil_div(tot, blk)), dim3(blk), 0, s, X, n, d, st.npad, st.dpad,
                         center, scale, st.x32.p);
      KRR_LAUNCH_CHECK();
    }
    // split vectors: the MFMA kernels (single column for MIXED, block for MIXED and FP32)
    st.ka = 32 * mixed_chunks(d);
    const double c = kLog2e / eps;
    if (sort) {
      KRR_REQUIRE(prec == KRR_MIXED && as_target && as_source, "spatial order is for square mixed operators");
      spatial_order(st, X, center, s);
    }
    if (as_target) {
      st.sa.alloc(st.npad * st.ka, s);
      hipLaunchKernelGGL(k_stage_split, dim3(ceil_div(st.npad, blk)), dim3(blk), 0, s, X, n, d, st.npad,
                         st.ka, center, c, 0, (const int64_t*)st.perm.p, st.sa.p);
      KRR_LAUNCH_CHECK();
    }
    if (as_source) {
      st.sb.alloc((st.npad + kPrefetchRows) * st.ka, s);   // padding rows: read by the last prefetch only
      hipLaunchKernelGGL(k_stage_split, dim3(ceil_div(st.npad, blk)), dim3(blk), 0, s, X, n, d, st.npad,
                         st.ka, center, c, 1, (const int64_t*)st.perm.p, st.sb.p);
      KRR_LAUNCH_CHECK();
    }
  }
}

__global__ void k_stage_vec(const double* __restrict__ V, int64_t n, int R, int64_t npad, int Rp,
                            const int64_t* __restrict__ perm, const int* __restrict__ cols, int ldv,
                            double* __restrict__ o64, float* __restrict__ o32) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= npad * Rp) return;
  int64_t i = idx / Rp;
  int c = (int)(idx % Rp);
  double v = (i < n && c < R) ? V[(perm ? perm[i] : i) * ldv + (cols ? cols[c] : c)] : 0.0;
  if (o64) o64[idx] = v;
  if (o32) o32[idx] = (float)v;
}

void stage_vectors(StagedVec& sv, const double* V, int64_t n, int64_t npad, int R, int prec,
                   hipStream_t s, const int64_t* perm, const int* cols, int ldv) {
  KRR_REQUIRE(!cols || (ldv >= R && !perm), "internal: a column subset needs its row stride and the caller's order");
  sv.npad = npad;
  sv.Rreal = R;
  sv.cols = cols;
  sv.ldv = cols ? ldv : R;
  // column chunks are at most 8 wide; FP64 with more than 8 columns pads to 16 for the matrix-core kernel
  sv.R = (int)round_up(R, prec == KRR_FP64 && R > 8 ? 16 : 8);
  const int64_t tot = npad * sv.R;
  const size_t cap = (size_t)(npad + kPrefetchRows) * sv.R;   // padding rows: read by the last prefetch only
  // grow only: a solve whose active columns shrink reuses the buffer, so products captured into a graph after
  // the first one allocate nothing
  if (prec == KRR_FP64) {
    if (sv.v64.n < cap) sv.v64.alloc(cap, s);
  } else {
    if (sv.v32.n < cap) sv.v32.alloc(cap, s);
  }
  hipLaunchKernelGGL(k_stage_vec, dim3(ceil_div(tot, 256)), dim3(256), 0, s, V, n, R, npad, sv.R, perm, cols,
                     sv.ldv, sv.v64.p, sv.v32.p);
  KRR_LAUNCH_CHECK();
}

__global__ void k_stage_v4(const double* __restrict__ V, int64_t n, int R, int64_t npad, int Rb, int nsplit,
                           const int* __restrict__ cols, int ldv, uint16_t* __restrict__ vh,
                           uint16_t* __restrict__ vm, uint16_t* __restrict__ vl) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= npad * Rb) return;
  const int64_t j = t / Rb;
  const int r = (int)(t % Rb);
  const double x = (j < n && r < R) ? V[j * ldv + (cols ? cols[r] : r)] : 0.0;
  const int64_t o = ((j >> 2) * Rb + r) * 4 + (j & 3);
  uint16_t h, m, l;
  split3(x, h, m, l);
  if (nsplit == 2) {   // two parts: lo takes the whole remainder x - hi
    m = bf16_rn((float)(x - bf16_to_double(h)));
  }
  vh[o] = h;
  vm[o] = m;
  if (vl) vl[o] = l;
}

// Block-MVM operands in the B-operand lane layout of the staged-V form (k_kmv_block32v): per 32-source step
// st, 16-column tile ct and part p, 64 lanes x 8 BF16 values; lane kq * 16 + r16 holds column 16 ct + r16 and
// the sources 4 kq + e (values 0..3) and 16 + 4 kq + e (values 4..7) of the step.
__global__ void k_stage_vt(const double* __restrict__ V, int64_t n, int R, int64_t npad, int Rb, int nsplit,
                           const int* __restrict__ cols, int ldv, uint16_t* __restrict__ vt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= npad * Rb) return;
  const int64_t j = t / Rb;
  const int r = (int)(t % Rb);
  const double x = (j < n && r < R) ? V[j * ldv + (cols ? cols[r] : r)] : 0.0;
  uint16_t h, m, l;
  split3(x, h, m, l);
  if (nsplit == 2) m = bf16_rn((float)(x - bf16_to_double(h)));   // two parts: the remainder x - hi
  const int np = nsplit == 2 ? 2 : 3;
  const int jj = (int)(j & 31);
  const int lanev = ((jj & 15) >> 2) * 16 + (r & 15);
  const int pos = (jj & 3) + 4 * (jj >> 4);
  const int64_t base = (((j >> 5) * (Rb / 16) + r / 16) * np) * 64 + lanev;
  vt[(base + 0 * 64) * 8 + pos] = h;
  vt[(base + 1 * 64) * 8 + pos] = m;
  if (np == 3) vt[(base + 2 * 64) * 8 + pos] = l;
}

void stage_vectors_vt(StagedVec& sv, const double* V, int64_t n, int64_t npad, int R, int nsplit, hipStream_t s) {
  sv.npad = npad;
  sv.Rreal = R;
  sv.Rb = (int)round_up(R, 16);
  const size_t tot = (size_t)npad * sv.Rb * (nsplit == 2 ? 2 : 3);
  if (sv.vt.n < tot) sv.vt.alloc(tot, s);   // grow only, as in stage_vectors
  hipLaunchKernelGGL(k_stage_vt, dim3((unsigned)ceil_div(npad * (int64_t)sv.Rb, 256)), dim3(256), 0, s, V, n, R, npad,
                     sv.Rb, nsplit, sv.cols, sv.cols ? sv.ldv : R, sv.vt.p);
  KRR_LAUNCH_CHECK();
}

void stage_vectors_block(StagedVec& sv, const double* V, int64_t n, int64_t npad, int R, int rpad, int nsplit,
                         hipStream_t s) {
  sv.npad = npad;
  sv.Rreal = R;
  sv.Rb = (int)round_up(R, rpad);
  const size_t tot = (size_t)npad * sv.Rb;
  if (sv.vh.n < tot) sv.vh.alloc(tot, s);   // grow only, as in stage_vectors
  if (sv.vm.n < tot) sv.vm.alloc(tot, s);
  if (nsplit == 3 && sv.vl.n < tot) sv.vl.alloc(tot, s);
  hipLaunchKernelGGL(k_stage_v4, dim3((unsigned)ceil_div((int64_t)tot, 256)), dim3(256), 0, s, V, n, R, npad, sv.Rb,
                     nsplit, sv.cols, sv.cols ? sv.ldv : R, sv.vh.p, sv.vm.p, nsplit == 3 ? sv.vl.p : nullptr);
  KRR_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ finishing kernel
// U[i, oc] = sum_s part[s, i, pc] (+ shift[oc] * Vraw[i, oc] on K columns), where the part row holds
// the K columns at [0, Rp) and the K' columns at [Rp, 2 Rp).
struct ShiftArg {
  double v[256];
};

__global__ void k_kmv_finish(const double* __restrict__ part, int S, int64_t mpad, int Rp, int Rout,
                             int deriv, int64_t m, int R, int has_shift, ShiftArg sh,
                             const double* __restrict__ Vraw, const int64_t* __restrict__ perm,
                             const int* __restrict__ cols, int ldv, double* __restrict__ U, int64_t ldu) {
  const int Rcols = deriv == 2 ? 2 * R : R;
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * Rcols) return;
  const int64_t i = idx / Rcols;
  const int oc = (int)(idx % Rcols);
  int pc;
  bool kcol;
  if (deriv == 0) { pc = oc; kcol = true; }
  else if (deriv == 1) { pc = Rp + oc; kcol = false; }
  else { kcol = oc < R; pc = kcol ? oc : Rp + (oc - R); }
  double acc = 0;
  // unrolled so that sixteen loads are in flight at once; the additions keep their order
#pragma unroll 16
  for (int p = 0; p < S; ++p) acc += part[((int64_t)p * mpad + i) * Rout + pc];
  const int64_t oi = perm ? perm[i] : i;   // staged row i is the caller's row oi
  const int col = cols ? cols[oc] : oc;     // (a column subset: one product without the derivative kernel)
  if (has_shift && kcol) acc += sh.v[oc] * Vraw[oi * ldv + col];
  U[oi * ldu + col] = acc;
}

// ------------------------------------------------------------------ variants and launcher
namespace {
std::mutex g_mu;
// Launch table: key "prec:d:rclass:nbucket:square" -> (variant, split).  nbucket = floor(log2 n) of the
// source count, or "*" for an entry that applies at every n (krr_set_variant); square 1 for K(X, X) v
// products, 0 for cross-set products, "*" for both.  split: sources per block of the direct forms (the
// source split over the grid) or the super-tile edge of the symmetric forms; 0 keeps the launcher's own
// choice.  Exact entries win over
// wildcard ones.  The table records the GPU architecture it was tuned on.
std::map<std::string, KmvChoice> g_table;
// shape classes of the variant table: 1 = one column, 2 = several columns (direct kernels),
// 3 = block MVM (many columns on MFMA)
int rclass(int prec, int R) {
  if (R == 1) return 1;
  if (prec == KRR_MIXED || (prec == KRR_FP32 && R > 8)) return 3;
  return 2;
}
std::string vprefix(int d, int R, int prec) {
  std::ostringstream o;
  o << prec << ":" << d << ":" << rclass(prec, R) << ":";
  return o.str();
}
std::string vkey(int d, int R, int prec) { return vprefix(d, R, prec) + "*:*"; }
int n_bucket(int64_t n) {
  int b = 0;
  while (n > 1) { n >>= 1; ++b; }
  return b;
}
std::string exact_key(int d, int R, int prec, int64_t n, bool square) {
  return vprefix(d, R, prec) + std::to_string(n_bucket(n)) + ":" + (square ? "1" : "0");
}
thread_local KmvLaunchInfo t_last;
const int kTM[3] = {1, 2, 4};
const int kNF[4] = {1, 2, 4, 8};
// block variants 0..5 contract with 16x16x16 MFMAs, 6..11 with 16x16x32 (same tile shapes)
const int kBlockNT[6] = {2, 4, 1, 2, 4, 1};
const int kBlockNRC[6] = {4, 2, 8, 2, 1, 4};
}  // namespace

std::string device_arch() {
  int dev = 0;
  KRR_CHECK_HIP(hipGetDevice(&dev));
  static std::map<int, std::string> cache;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  hipDeviceProp_t prop;
  KRR_CHECK_HIP(hipGetDeviceProperties(&prop, dev));
  std::string a(prop.gcnArchName);
  a = a.substr(0, a.find(':'));
  return cache[dev] = a;
}

KmvLaunchInfo kmv_last_launch() { return t_last; }

// The shared-tile block forms (variants 12, 13) cover 128 columns per block in 32-column waves; with fewer
// than 7/8 of those waves holding columns the idle ones cost more than the shared exp/split saves.
static bool shared_block_fits(int R) {
  const int rb = (int)round_up(R, 32);
  return R >= 128 && 8 * rb >= 7 * 128 * (int)ceil_div(rb, 128);
}

KmvChoice kmv_lookup(int prec, int d, int R, int64_t n, bool square) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (n > 0) {
    auto it = g_table.find(exact_key(d, R, prec, n, square));
    if (it != g_table.end()) {
      // a tuned entry covers every column count of its shape class: a shared-tile block form tuned at a
      // full count gives way to the per-wave form (variant 7) where its waves would idle, e.g. when a
      // block solve's active columns shrink (forced variants are taken as they are)
      if (rclass(prec, R) == 3 && (it->second.variant == 12 || it->second.variant == 13) && !shared_block_fits(R))
        return KmvChoice{7, 0};
      // the staged-V form likewise gives way to variant 7 at 32 columns or fewer (its exp per pair then
      // serves too few contractions)
      if (rclass(prec, R) == 3 && it->second.variant == 14 && R <= 32) return KmvChoice{7, 0};
      return it->second;
    }
  }
  auto it = g_table.find(vkey(d, R, prec));
  return it == g_table.end() ? KmvChoice{} : it->second;
}

void kmv_set_tuned(int prec, int d, int R, int64_t n, bool square, KmvChoice c) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[exact_key(d, R, prec, n, square)] = c;
}

int kmv_num_variants(int prec, int R) {
  // block: 0..5 K = 16, 6..11 K = 32 tile shapes, 12 shared tile (64 targets), 13 shared tile (128 targets),
  // 14 staged V (64 targets, each wave all of the block's columns)
  if (rclass(prec, R) == 3) return 15;
  // mixed: 0..3 plain (NF 1, 2, 4, 8), 4..6 pipelined (NF 2, 4, 8), 7..9 pipelined + LDS tiles (NF 2, 4, 8),
  // 10..11 symmetric square product (NF 4, 8; other shapes run variant 8 / 9);
  // FP64 one column: 0..2 direct (TM 1, 2, 4), 3..4 symmetric square product (TM 2, 4; else variant 1 / 2),
  // 5..6 symmetric with the cross term on the FP64 matrix cores (4, 2 target fragments per wave; else variant 2)
  // FP64 several columns: 0..2 direct (TM 1, 2, 4; R >= 16: TM 1 with 16 / 32-column chunks), 3 the FP64
  // matrix-core form (d <= 16, K only; else variant 1)
  if (prec == KRR_MIXED) return 12;
  if (prec == KRR_FP64) return rclass(prec, R) == 1 ? 7 : 4;
  return 3;
}

bool kmv_f64_uses_mfma(int prec, int d, int R, int deriv, int variant) {
  return prec == KRR_FP64 && R > 1 && deriv == 0 && variant == 3 && padded_dim(d) >= 1 && padded_dim(d) <= 16;
}

bool kmv_uses_block(int prec, int d, int R, int deriv) {
  return deriv == 0 && rclass(prec, R) == 3 && mixed_chunks(d) <= 4;
}

int kmv_default_variant(int prec, int d, int R, int64_t m, int64_t, bool square) {
  // block MVM (measured at n = 5e5, d = 6): the shared-tile form (variant 12, each pair's exp/split once per
  // 128 columns) against K = 32 contractions over 4 target fragments x 2 column groups (variant 7): with two
  // parts (MIXED, three waves per SIMD) 316 against 348 ms at R = 128 on one machine, 321 against 324 ms
  // (four products at n = 2.5e5) on another; with three parts (FP32) 1.26x faster;
  // variant 12 when at least 7/8 of its waves hold columns (below, its idle waves cost more: 2.9x / 1.6x
  // slower at R = 32 / 64), else variant 7 (1.36x faster than variant 0).
  // The staged-V form (variant 14: each wave contracts its own exp'd fragment with all of the block's
  // columns, V staged through LDS one step ahead) beats both from R = 64 on (n = 2e5, d = 6, MIXED: R = 64
  // 24.1 against 26.5 ms for variant 7, R = 128 34.1 against 51.5 for variant 12, R = 256 67.2 against 102.4;
  // n = 5e5, R = 128: 205.8 against 317.6, FP32 364 against 466), not at R = 32 (20.4 against 13.9 for
  // variant 7).
  if (rclass(prec, R) == 3) return R > 32 ? 14 : 7;
  if (prec == KRR_MIXED) {
    // one K chunk: the exp/FMA stream bounds the kernel and the plain NF 8 form is fastest; two to four
    // chunks: the MFMA stream grows and the LDS-staged pipelined form wins (measured on MI355X, d = 4 / 8)
    const int nch = mixed_chunks(d);
    if (kmv_is_symmetric(prec, d, R, 0, square, 11)) return 11;   // symmetric square product (NF 8; 4 above 2 chunks)
    if (nch == 1) return 3;
    if (nch == 2) return 9;
    if (nch <= 4) return 8;
    return mixed_max_nf(nch) >= 2 ? 1 : 0;
  }
  // FP64 symmetric square product with the exponent's cross term on the matrix cores, 4 target fragments per
  // wave (n = 1e6, d = 4: 331 ms against 392 ms for the direct symmetric form; n = 5e5, d = 6: 90.5 ms against
  // 116 ms; n = 2e5, d = 16: 21 ms against 32 ms; 2 fragments per wave within 4% of it)
  if (kmv_is_symmetric(prec, d, R, 0, square, 5)) return 5;
  if (padded_dim(d) >= 32) return 0;
  // FP64, more than 8 columns: the matrix-core kernel evaluates each pair once for up to 128 columns
  // (n = 2e5, d = 6: 2.05x faster than the 32-column chunks at R = 128, 1.14x at R = 16)
  if (prec == KRR_FP64 && R > 8) return 3;
  return m >= 65536 ? 1 : 0;
}

bool kmv_is_symmetric(int prec, int d, int R, int deriv, bool square, int v) {
  if (R != 1 || deriv != 0 || !square) return false;
  if (prec == KRR_MIXED) return v >= 10 && mixed_chunks(d) <= 4;
  if (prec == KRR_FP64) return v >= 3 && kmv_f64_has_sym(padded_dim(d));
  return false;
}

void kmv_set_override(int d, int R, int prec, int variant) {
  // a forced variant applies at every n: it replaces the tuned entries of its (prec, d, shape class)
  std::lock_guard<std::mutex> lk(g_mu);
  const std::string pre = vprefix(d, R, prec);
  for (auto it = g_table.begin(); it != g_table.end();)
    it = it->first.compare(0, pre.size(), pre) == 0 ? g_table.erase(it) : std::next(it);
  if (variant >= 0) g_table[vkey(d, R, prec)] = KmvChoice{variant, 0};
}

int kmv_get_override(int d, int R, int prec) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_table.find(vkey(d, R, prec));
  return it == g_table.end() ? -1 : it->second.variant;
}

std::string kmv_table_json() {
  std::string arch;
  try { arch = device_arch(); } catch (...) { arch = ""; }
  std::lock_guard<std::mutex> lk(g_mu);
  std::ostringstream o;
  o << "{\"arch\": \"" << arch << "\", \"entries\": {";
  bool first = true;
  for (auto& kv : g_table) {
    o << (first ? "" : ", ") << "\"" << kv.first << "\": [" << kv.second.variant << ", " << kv.second.split << "]";
    first = false;
  }
  o << "}}\n";
  return o.str();
}

// Entries are "prec:d:rclass:nbucket:square": [variant, split] pairs inside the "entries" object.  A table
// tuned on another architecture is rejected.
void kmv_table_from_json(const std::string& s) {
  size_t pa = s.find("\"arch\"");
  if (pa != std::string::npos) {
    const size_t q1 = s.find('"', s.find(':', pa) + 1);
    const size_t q2 = q1 == std::string::npos ? q1 : s.find('"', q1 + 1);
    KRR_REQUIRE(q2 != std::string::npos, "autotune table: malformed arch");
    const std::string arch = s.substr(q1 + 1, q2 - q1 - 1);
    std::string here;
    try { here = device_arch(); } catch (...) { here = arch; }
    KRR_REQUIRE(arch.empty() || arch == here, "autotune table was tuned on " + arch + ", this GPU is " + here);
  }
  size_t pos = s.find("\"entries\"");
  KRR_REQUIRE(pos != std::string::npos, "autotune table: no entries object");
  pos = s.find('{', pos);
  KRR_REQUIRE(pos != std::string::npos, "autotune table: malformed entries object");
  std::map<std::string, KmvChoice> parsed;
  size_t i = pos + 1;
  auto read_int = [&](size_t& j) {
    while (j < s.size() && (s[j] == ' ' || s[j] == ',' || s[j] == '[' || s[j] == ':')) ++j;
    size_t e = j;
    while (e < s.size() && (std::isdigit((unsigned char)s[e]) || s[e] == '-')) ++e;
    KRR_REQUIRE(e > j, "autotune table: missing number");
    const int v = std::atoi(s.substr(j, e - j).c_str());
    j = e;
    return v;
  };
  while (i < s.size() && s[i] != '}') {
    if (s[i] != '"') { ++i; continue; }
    const size_t q2 = s.find('"', i + 1);
    KRR_REQUIRE(q2 != std::string::npos, "autotune table: unterminated key");
    const std::string key = s.substr(i + 1, q2 - i - 1);
    KRR_REQUIRE(std::count(key.begin(), key.end(), ':') == 4, "autotune table: bad key " + key);
    size_t j = q2 + 1;
    KmvChoice c;
    c.variant = read_int(j);
    c.split = read_int(j);
    const size_t close = s.find(']', j);
    KRR_REQUIRE(close != std::string::npos, "autotune table: unterminated entry " + key);
    parsed[key] = c;
    i = close + 1;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : parsed) g_table[kv.first] = kv.second;
}

// Compute units of the current device (cached per device).
static int64_t device_cus() {
  int dev = 0;
  KRR_CHECK_HIP(hipGetDevice(&dev));
  static std::map<int, int64_t> cache;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int cus = 0;
  KRR_CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  return cache[dev] = std::max(cus, 1);
}

// Resident blocks of a kernel configuration on the current device (blocks per CU x CUs), cached by key.
template <typename Query>
static int64_t resident_blocks(Query query, const std::string& key) {
  int dev = 0;
  KRR_CHECK_HIP(hipGetDevice(&dev));
  const std::string k = std::to_string(dev) + "/" + key;
  static std::map<std::string, int64_t> cache;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = cache.find(k);
    if (it != cache.end()) return it->second;
  }
  int per_cu = 0, cus = 0;
  query(&per_cu);
  KRR_CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t cap = std::max<int64_t>(1, (int64_t)std::max(per_cu, 1) * std::max(cus, 1));
  std::lock_guard<std::mutex> lk(g_mu);
  cache[k] = cap;
  return cap;
}

// V (k x ncol, stride ldt) -> rows x Rp zero-padded copy (the FP64 matrix-core kernel's operand layout)
__global__ void k_pad_matrix(const double* __restrict__ T, int64_t k, int64_t ldt, int ncol, int64_t rows, int Rp,
                             double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * Rp) return;
  const int64_t j = t / Rp;
  const int c = (int)(t % Rp);
  out[t] = (j < k && c < ncol) ? T[j * ldt + c] : 0.0;
}

bool kernel_times_matrix_f64(const double* Xt, int64_t m, const double* Xs, int64_t k, int d, double eps,
                             const double* T, int64_t ldt, int ncol, double* W, int64_t ldw, hipStream_t s) {
  const int D = padded_dim(d);
  if (D < 1 || D > 16) return false;
  Staged St, Ss;
  stage_points(St, Xt, m, d, eps, KRR_FP64, nullptr, true, false, s);
  stage_points(Ss, Xs, k, d, eps, KRR_FP64, nullptr, false, true, s);
  const int Rp = (int)round_up(ncol, 16);
  DevBuf<double> V((size_t)Ss.npad * Rp, s);
  hipLaunchKernelGGL(k_pad_matrix, dim3((unsigned)ceil_div(Ss.npad * Rp, 256)), dim3(256), 0, s, T, k, ldt, ncol,
                     Ss.npad, Rp, V.p);
  KRR_LAUNCH_CHECK();
  // block width 16 NRG: per 4-source step NRG MFMAs (64 cycles each) plus the pair's distance and exp
  // (about 112 VALU cycles), over ceil(Rp / 16 NRG) column blocks
  int NRG = 8;
  double best = 1e300;
  for (int nr : {8, 6, 4, 2, 1}) {
    const double cost = (double)ceil_div(Rp, 16 * nr) * (64.0 * nr + 112.0);
    if (cost < best * (1 - 1e-9)) { best = cost; NRG = nr; }
  }
  KmvGrid g{dim3((unsigned)(St.npad / 64), 1u, (unsigned)ceil_div(Rp, 16 * NRG)), Ss.npad, Ss.npad, St.npad, Rp,
            (int)ldw};
  g.m_store = m;
  g.n_store = ncol;
  KRR_REQUIRE(launch_kmv_f64_mfma(D, NRG, g, St.x64.p, Ss.x64.p, V.p, -kLog2e / eps, W, s),
              "FP64 matrix-core kernel not instantiated for this width");
  KRR_LAUNCH_CHECK();
  return true;
}

void kmv_launch(const Staged& T, const Staged& S, StagedVec& V, int deriv, const double* shift_host,
                const double* Vraw, int prec, double* U, int64_t ldu, hipStream_t s, int variant,
                DevBuf<double>* ws, const hipEvent_t* kev, int split_req) {
  KRR_REQUIRE(T.prec == prec && S.prec == prec, "staged precision mismatch");
  KRR_REQUIRE(!V.cols || (deriv == 0 && ldu >= V.ldv), "internal: a column subset is for one K product into U");
  const int R = V.Rreal, Rp = V.R;
  KRR_REQUIRE(R >= 1 && R <= 256, "R must be in [1, 256]");
  const int DV = deriv == 0 ? 0 : 2;
  const int Rout = (DV == 2 ? 2 : 1) * Rp;
  if (variant < 0) {
    const KmvChoice ch = kmv_lookup(prec, T.d, R, S.n, &T == &S && deriv == 0);
    variant = ch.variant;
    if (split_req <= 0 && variant >= 0) split_req = ch.split;
  }
  if (variant < 0) variant = kmv_default_variant(prec, T.d, R, T.n, S.n, &T == &S && deriv == 0);
  KRR_REQUIRE(variant < kmv_num_variants(prec, R), "unknown kernel variant");
  int64_t rows;
  int gz, TM = 1, NF = 1, RC = R == 1 ? 1 : R <= 4 ? 4 : 8;
  int form = 0;   // mixed single-column kernel form
  bool sym = false;   // symmetric square product (mixed, one column)
  bool f64sm = false; // FP64 symmetric form with the cross term on the matrix cores
  const int D = T.dpad;
  // FP64 many-column product on the FP64 matrix cores (variant 3 of FP64 with R > 1)
  const bool f64m = kmv_f64_uses_mfma(prec, T.d, R, deriv, variant) && Rp % 16 == 0;
  int NRG = 8;
  const bool block = kmv_uses_block(prec, T.d, R, deriv);
  int NT = 1, NRC = 1, Rpart = Rp;
  bool k32 = false, shared = false, vtile = false;
  int shared_fw = 1;   // fragments per wave of the shared-tile form
  if (block && variant == 14) {   // staged-V form: 64 targets and up to 128 columns per block
    vtile = true;
    stage_vectors_vt(V, Vraw, S.n, S.npad, R, prec == KRR_MIXED ? 2 : 3, s);
    Rpart = V.Rb;
    rows = 64;
    gz = (int)ceil_div(V.Rb, 128);
  } else if (block) {
    shared = variant >= 12;
    shared_fw = variant == 13 ? 2 : 1;
    const int vb = shared ? 1 : variant % 6;
    k32 = variant >= 6;
    int nrc_max = 1;
    while (nrc_max * 2 <= ceil_div(R, 16)) nrc_max *= 2;
    NT = kBlockNT[vb];
    NRC = std::min(kBlockNRC[vb], nrc_max);
    stage_vectors_block(V, Vraw, S.n, S.npad, R, shared ? 32 : 16 * NRC, prec == KRR_MIXED ? 2 : 3, s);
    Rpart = V.Rb;
    rows = shared ? 64 * shared_fw : 64 * NT;
    gz = shared ? (int)ceil_div(V.Rb, 128) : V.Rb / (16 * NRC);   // shared form: 128 columns per block
  } else if (prec == KRR_MIXED) {
    const int nch = T.ka / 32;
    int var = variant;
    if (var >= 10) {
      // the symmetric form needs the square product of one column without the derivative kernel
      sym = kmv_is_symmetric(prec, T.d, R, deriv, &T == &S, var);
      if (!sym) var -= 2;
    }
    if (sym) {
      NF = nch <= 2 && var == 11 ? 8 : 4;
    } else {
      form = var >= 7 ? 2 : var >= 4 ? 1 : 0;
      NF = std::min(var >= 7 ? kNF[var - 6] : var >= 4 ? kNF[var - 3] : kNF[var], mixed_max_nf(nch));
      if (!mixed_has_pp(nch) || NF < 2) form = 0;   // no pipelined form: the plain kernel, same NF
    }
    rows = 64 * NF;
    gz = 1;
  } else if (f64m) {
    // block width 16 * NRG: per 4-source step a block costs NRG MFMAs (64 cycles each) plus the pair's
    // distance and exp (about 112 VALU cycles); dead groups of a partly filled last block are contracted too
    double best = 1e300;
    for (int nr : {8, 6, 4, 2, 1}) {
      const double cost = (double)ceil_div(Rp, 16 * nr) * (64.0 * nr + 112.0);
      if (cost < best * (1 - 1e-9)) { best = cost; NRG = nr; }
    }
    rows = 64;
    gz = (int)ceil_div(Rp, 16 * NRG);   // the last block may hold fewer than 16 * NRG columns
  } else {
    int var = variant;
    if (prec == KRR_FP64 && var >= 3) {
      sym = kmv_is_symmetric(prec, T.d, R, deriv, &T == &S, var);
      f64sm = sym && var >= 5;
      if (f64sm) NF = var == 5 ? 4 : 2;   // target fragments per wave of the matrix-core form
      if (!sym) var = var >= 5 ? 2 : var - 2;
    }
    TM = f64sm ? 1 : sym ? (var == 3 ? 2 : 4) : D >= 32 ? 1 : kTM[var];
    // many right-hand sides in FP64: wide column chunks (the exp of a pair is shared by RC columns)
    // (a chunk must not run past the padded column count Rp: RC divides Rp)
    if (prec == KRR_FP64 && !sym && DV == 0 && D <= 16 && R >= 16 && Rp % 16 == 0) {
      RC = R >= 32 && Rp % 32 == 0 ? 32 : 16;
      TM = 1;
    }
    rows = f64sm ? 64 * NF : 256 * TM;
    gz = (int)ceil_div(R, RC);   // real columns only (Rp is padded to 8)
    KRR_REQUIRE(Rp % RC == 0, "internal: column chunk does not divide the padded column count");
  }
  KRR_REQUIRE(!block || (!T.perm.p && !S.perm.p), "internal: spatially ordered operators take one column");
  // exact far-tile culling: only the symmetric form of an operator staged in spatial order skips work
  // (cull_masks returns nullptr when automatic mode finds too little to skip)
  const uint16_t* cmask = (sym && T.perm.p && T.box16.p && cull_mode() != 2) ? cull_masks(T, NF, s) : nullptr;
  const int64_t gx = T.npad / rows;
  const int64_t nsrc = S.npad;
  const int RpK = block ? Rpart : Rp;                  // row width of the K part in `part`
  // one column without the derivative kernel: partials are stored densely (one value per row and split)
  const int RoutK = !block && DV == 0 && R == 1 ? 1 : (DV == 2 ? 2 : 1) * RpK;
  DevBuf<double> own;
  DevBuf<double>& part = ws ? *ws : own;
  auto run = [&](const KmvGrid& g) -> bool {
    if (vtile) return launch_kmv_block_vt(T.ka / 32, prec == KRR_MIXED ? 3 : 6, g, T.sa.p, S.sb.p, V.vt.p, part.p, s);
    if (block && shared)
      return launch_kmv_block_shared(T.ka / 32, prec == KRR_MIXED ? 3 : 6, shared_fw, g, T.sa.p, S.sb.p, V.vh.p, V.vm.p,
                                     prec == KRR_MIXED ? nullptr : V.vl.p, part.p, s);
    if (block)
      return launch_kmv_block(T.ka / 32, NT, NRC, prec == KRR_MIXED ? 3 : 6, k32, g, T.sa.p, S.sb.p, V.vh.p,
                              V.vm.p, prec == KRR_MIXED ? nullptr : V.vl.p, part.p, s);
    if (f64sm) return launch_kmv_f64_symm(D, NF, !T.q_floor, g, T.x64.p, V.v64.p, -kLog2e / T.eps, part.p, s);
    if (prec == KRR_FP64 && sym) return launch_kmv_f64_sym(D, TM, g, T.x64.p, V.v64.p, -kLog2e / T.eps, part.p, s);
    if (f64m) return launch_kmv_f64_mfma(D, NRG, g, T.x64.p, S.x64.p, V.v64.p, -kLog2e / T.eps, part.p, s);
    if (prec == KRR_FP64) return launch_kmv_f64(D, TM, RC, DV, g, T.x64.p, S.x64.p, V.v64.p, -kLog2e / T.eps, part.p, s);
    if (prec == KRR_FP32) return launch_kmv_f32(D, TM, RC, DV, g, T.x32.p, S.x32.p, V.v32.p, part.p, s);
    if (sym) return launch_kmv_mixed_sym(T.ka / 32, NF, g, T.sa.p, S.sb.p, V.v32.p, part.p, s, g.occ ? nullptr : cmask);
    bool ok = true;
    for (int c = 0; c < R && ok; ++c) {
      ok = launch_kmv_mixed(T.ka / 32, NF, DV, form, g, T.sa.p, S.sb.p, V.v32.p, c, part.p, s);
      if (g.occ) break;
      KRR_LAUNCH_CHECK();
    }
    return ok;
  };
  // Source split: the grid runs in rounds of `cap` resident blocks; choose the split that minimises
  // rounds x (per-block source count + a fixed per-block cost), so the last round is not mostly idle.
  // The block path caps its FP64 partial buffer near 2 GB.
  KmvGrid q{dim3(1, 1, 1), 0, nsrc, T.npad, RpK, RoutK};
  const int64_t cap = resident_blocks(
      [&](int* occ) {
        q.occ = occ;
        KRR_REQUIRE(run(q), "kernel variant not instantiated for this shape");
      },
      vkey(T.d, R, prec) + ":" + std::to_string(variant) + ":" + std::to_string(DV));
  int64_t smax = std::max<int64_t>(1, nsrc / 256);
  if (block) smax = std::min<int64_t>(smax, std::max<int64_t>(1, ((int64_t)1 << 28) / (T.npad * (int64_t)RoutK)));
  const int64_t per_split = gx * gz;
  int64_t split = 1;
  double best = 1e300;
  // (source chunks of at most 64K points keep each block's run short against the kernel's total)
  for (int64_t sp = std::min(smax, ceil_div(nsrc, 65536)); sp <= smax; ++sp) {
    const int64_t len = round_up(ceil_div(nsrc, sp), 256);
    const int64_t spl = ceil_div(nsrc, len);
    if (spl != sp) continue;   // the same source length as a smaller split
    const double rounds = (double)ceil_div(per_split * spl, cap);
    const double cost = rounds * (double)(len + 512);
    if (cost < best * (1 - 1e-9)) { best = cost; split = spl; }
  }
  int64_t src_len = round_up(ceil_div(nsrc, split), 256);
  if (split_req > 0 && !sym) {   // a requested source length per block (at most smax splits)
    src_len = std::max<int64_t>(round_up(split_req, 256), round_up(ceil_div(nsrc, smax), 256));
    split = ceil_div(nsrc, src_len);
  }
  // Small one-column FP64 products: when splits of 256 sources leave CUs idle, the sources are split in
  // multiples of 64 (the direct kernel's 64-point tile form) for about two blocks per CU.
  if (prec == KRR_FP64 && !sym && !f64m && !block && R == 1 && DV == 0 && TM == 1 && split_req <= 0 &&
      D <= 16 && per_split * split < device_cus()) {
    const int64_t sp = std::min<int64_t>(std::max<int64_t>(1, nsrc / 64), ceil_div(2 * device_cus(), per_split));
    src_len = round_up(ceil_div(nsrc, sp), 64);
    split = ceil_div(nsrc, src_len);
  }
  KmvGrid g{dim3((unsigned)gx, (unsigned)split, (unsigned)gz), src_len, nsrc, T.npad, RpK, RoutK};
  if (sym) {
    KRR_REQUIRE(RoutK == 1, "internal: the symmetric kernels write dense one-column partials");
    // super-tile edge E: the per-CU work ceil(items / CUs) x E^2 (at least two blocks per CU to hide
    // latency) is minimised, with the partial buffer (NS x npad doubles) kept near 2 GB
    const int64_t cus = device_cus();
    int64_t bestE = 0;
    double bestc = 1e300;
    for (int64_t E : {1024, 2048, 3072, 4096, 6144, 8192, 12288, 16384}) {
      if (E % rows) continue;
      const int64_t ns = ceil_div(T.npad, E);
      if ((double)ns * T.npad * 8.0 > 2.2e9 && E != 16384) continue;
      const int64_t items = ns * (ns + 1) / 2;
      const double cost = (double)std::max<int64_t>(ceil_div(items, cus), 2) * (double)E * (double)E;
      if (cost < bestc * (1 - 1e-9)) { bestc = cost; bestE = E; }
    }
    // a requested edge: one of the candidates, a multiple of the target tile, partials near 2 GB at most
    if (split_req > 0 && split_req % rows == 0 && split_req >= 1024 && split_req <= 16384 &&
        (double)ceil_div(T.npad, split_req) * T.npad * 8.0 <= 2.2e9)
      bestE = split_req;
    const int64_t ns = ceil_div(T.npad, bestE);
    const int64_t items = ns * (ns + 1) / 2;
    split = ns;
    src_len = bestE;
    g = KmvGrid{dim3((unsigned)(8 * ceil_div(items, 8))), src_len, nsrc, T.npad, RpK, RoutK};
    g.E = (int)bestE;
    g.NS = (int)ns;
  }
  const size_t need = (size_t)split * T.npad * RoutK;
  if (part.n < need) part.alloc(need, s);
  t_last = KmvLaunchInfo{variant, (int)(sym ? g.E : src_len), sym ? 1 : 0, cmask ? 1 : 0, T.npad, NF};
  if (cmask) cull_reset_counters(s);
  if (kev) KRR_CHECK_HIP(hipEventRecord(kev[0], s));
  const bool ok = run(g);
  if (kev) KRR_CHECK_HIP(hipEventRecord(kev[1], s));
  KRR_REQUIRE(ok, "kernel variant not instantiated for this shape");
  KRR_LAUNCH_CHECK();
  ShiftArg sh{};
  const int has_shift = shift_host != nullptr;
  if (has_shift)
    for (int c = 0; c < R; ++c) sh.v[c] = shift_host[c];
  const int Rcols = deriv == 2 ? 2 * R : R;
  const int64_t tot = T.n * Rcols;
  hipLaunchKernelGGL(k_kmv_finish, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, s, part.p, (int)split,
                     T.npad, RpK, RoutK, deriv, T.n, R, has_shift, sh, Vraw, (const int64_t*)T.perm.p, V.cols,
                     V.cols ? V.ldv : R, U, ldu);
  KRR_LAUNCH_CHECK();
}

}  // namespace krr
