// Exact far-tile culling for the symmetric mixed kernel MVM (the fast-MVM slot the paper leaves open,
// Sec. 2.4, without an approximation): the points of a square operator are staged in Morton order of their
// grid cells, so that consecutive groups of points are spatially compact, and a 16-source step of a wave's
// targets is skipped when the boxes of the two groups are so far apart that every kernel value between them
// is exactly zero in FP32.
//
// Exactness: the symmetric kernel's exp2 argument is q = -||z'_i - z'_j||^2 with z' = (x - center) sqrt(c),
// c = log2(e) / eps, computed by the split-BF16 MFMA chain with FP32 accumulation; its rounding error is at
// most 2^-18 (|z'_i|^2 + |z'_j|^2) (about thirty exact BF16 products summed in FP32).  exp2 of anything below
// -150 is 0 in FP32 (the smallest subnormal is 2^-149).  A step is culled when the boxes' minimum scaled
// squared distance exceeds 161 + 2^-18 (R_t^2 + R_s^2), R^2 the largest |z'|^2 over a box, so every skipped
// value is exactly 0 and the sums are bit for bit those of the unculled kernel.
#include <atomic>
#include <map>
#include <mutex>

#include "anchors.h"
#include "kmv.h"
#include "radix_sort.h"


namespace krr {

namespace {
std::atomic<int> g_cull_mode{-1};
constexpr double kCullQ = 161.0;   // exp2(-q) underflows to exactly 0 in FP32 for q > 150
constexpr double kCullMin = 0.10;  // least share of skippable steps for automatic culling

__device__ unsigned long long cull_count[2];   // skipped 16-source steps: diagonal / off-diagonal super-tiles
std::mutex g_cnt_mu;
std::map<int, unsigned long long*> g_cnt_ptr;  // device ordinal -> address of that device's cull_count

// Morton code of the grid cell of point i (b bits per coordinate over the bounding box).
__global__ void k_morton(const double* __restrict__ X, int64_t n, int d, const double* __restrict__ lo,
                         const double* __restrict__ inv_w, int b, uint64_t* __restrict__ code,
                         int64_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t q[32];
  const double top = (double)((1u << b) - 1u);
  for (int k = 0; k < d && k < 32; ++k) {
    double t = (X[i * d + k] - lo[k]) * inv_w[k] * top;
    t = t < 0.0 ? 0.0 : (t > top ? top : t);
    q[k] = (uint32_t)t;
  }
  uint64_t c = 0;
  for (int j = b - 1; j >= 0; --j)
    for (int k = 0; k < d && k < 32; ++k) c = (c << 1) | ((q[k] >> j) & 1u);
  code[i] = c;
  idx[i] = i;
}

// Box of each group of 16 staged points in the scaled coordinates z' = (x - center) sqrt(c): lo[dpad] hi[dpad].
// A group without real points gets an empty box (lo = +inf, hi = -inf).
__global__ void k_box16(const double* __restrict__ X, int64_t n, int d, int dpad, const int64_t* __restrict__ perm,
                        const double* __restrict__ center, double sc, int64_t ngroups, double* __restrict__ box) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngroups) return;
  double* b = box + g * 2 * dpad;
  for (int k = 0; k < dpad; ++k) {
    double lo = k < d ? INFINITY : 0.0, hi = k < d ? -INFINITY : 0.0;
    if (k < d)
      for (int64_t i = g * 16; i < g * 16 + 16 && i < n; ++i) {
        const double z = (X[perm[i] * d + k] - center[k]) * sc;
        lo = fmin(lo, z);
        hi = fmax(hi, z);
      }
    b[k] = lo;
    b[dpad + k] = hi;
  }
}

__device__ __forceinline__ bool box_empty(const double* b, int dpad) { return !(b[0] <= b[dpad]); }

// mask[tg * ngs + sg]: bit s set when the 16-source group 16 sg + s and the target group tg (16 NF points)
// have no pair whose kernel value can be non-zero in FP32 (see the file comment).
__global__ void k_cull_masks(const double* __restrict__ box, int dpad, int nf, int64_t ntg, int64_t ngs,
                             uint16_t* __restrict__ mask, unsigned long long* __restrict__ count) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntg * ngs) return;
  const int64_t tg = t / ngs, sg = t % ngs;
  double tlo[32], thi[32];
  bool tempty = true;
  for (int k = 0; k < dpad; ++k) {
    tlo[k] = INFINITY;
    thi[k] = -INFINITY;
  }
  for (int f = 0; f < nf; ++f) {
    const double* b = box + (tg * nf + f) * 2 * dpad;
    if (box_empty(b, dpad)) continue;
    tempty = false;
    for (int k = 0; k < dpad; ++k) {
      tlo[k] = fmin(tlo[k], b[k]);
      thi[k] = fmax(thi[k], b[dpad + k]);
    }
  }
  double rt = 0.0;
  if (!tempty)
    for (int k = 0; k < dpad; ++k) rt += fmax(tlo[k] * tlo[k], thi[k] * thi[k]);
  unsigned m = 0;
  for (int s = 0; s < 16; ++s) {
    const double* b = box + (sg * 16 + s) * 2 * dpad;
    if (tempty || box_empty(b, dpad)) {
      m |= 1u << s;
      continue;
    }
    double dist = 0.0, rs = 0.0;
    for (int k = 0; k < dpad; ++k) {
      const double gap = fmax(0.0, fmax(b[k] - thi[k], tlo[k] - b[dpad + k]));
      dist += gap * gap;
      rs += fmax(b[k] * b[k], b[dpad + k] * b[dpad + k]);
    }
    if (dist > kCullQ + 0x1p-18 * (rt + rs)) m |= 1u << s;
  }
  mask[t] = (uint16_t)m;
  const unsigned c = __popc(m);
  if (c) atomicAdd(count, (unsigned long long)c);
}

__global__ void k_cull_zero(unsigned long long* c) {
  if (threadIdx.x < 2) c[threadIdx.x] = 0ull;
}
}  // namespace

int cull_mode() { return g_cull_mode.load(); }
void set_cull_mode(int mode) { g_cull_mode.store(mode < 0 ? -1 : (mode > 2 ? 2 : mode)); }

bool cull_wanted(const double* X, int64_t n, int d, double eps, hipStream_t s) {
  const int mode = cull_mode();
  if (mode == 0 || mixed_chunks(d) > 4 || n < 2048) return false;   // the symmetric form needs d <= 20
  if (mode >= 1) return true;
  // automatic: only when the data's extent reaches well past the threshold (twice its scaled distance)
  std::vector<double> lo(d), hi(d);
  bounding_box(X, n, d, lo.data(), hi.data(), s);
  double diag2 = 0.0;
  for (int k = 0; k < d; ++k) diag2 += (hi[k] - lo[k]) * (hi[k] - lo[k]);
  return diag2 * kLog2e / eps > 2.0 * kCullQ;
}

void spatial_order(Staged& st, const double* X, const double* center, hipStream_t s) {
  const int64_t n = st.n;
  const int d = st.d, dpad = st.dpad;
  std::vector<double> lo(d), hi(d), inv(d);
  bounding_box(X, n, d, lo.data(), hi.data(), s);
  for (int k = 0; k < d; ++k) inv[k] = hi[k] > lo[k] ? 1.0 / (hi[k] - lo[k]) : 0.0;
  const int b = std::max(1, std::min(20, 63 / d));
  DevBuf<double> lod(d, s), invd(d, s);
  KRR_CHECK_HIP(hipMemcpyAsync(lod.p, lo.data(), sizeof(double) * d, hipMemcpyHostToDevice, s));
  KRR_CHECK_HIP(hipMemcpyAsync(invd.p, inv.data(), sizeof(double) * d, hipMemcpyHostToDevice, s));
  DevBuf<uint64_t> code(n, s), scode(n, s);
  DevBuf<int64_t> idx(n, s);
  st.perm.alloc(st.npad, s);
  hipLaunchKernelGGL(k_morton, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, X, n, d, lod.p, invd.p, b, code.p,
                     idx.p);
  KRR_LAUNCH_CHECK();
  RadixSortWork rsw;
  radix_sort_pairs(code.p, scode.p, idx.p, st.perm.p, n, b * d, rsw, s);
  const int64_t ng = st.npad / 16;
  st.box16.alloc((size_t)ng * 2 * dpad, s);
  hipLaunchKernelGGL(k_box16, dim3((unsigned)ceil_div(ng, 256)), dim3(256), 0, s, X, n, d, dpad,
                     (const int64_t*)st.perm.p, center, std::sqrt(kLog2e / st.eps), ng, st.box16.p);
  KRR_LAUNCH_CHECK();
}

const uint16_t* cull_masks(const Staged& S, int NF, hipStream_t s) {
  KRR_REQUIRE(S.box16.p && S.dpad <= 32, "internal: culling boxes missing");
  if (S.cull_nf == NF) return S.cull_mask.p;   // built (or found not worth it) for this NF
  const int64_t ntg = S.npad / (16 * NF), ngs = S.npad / 256;
  S.cull_mask.alloc((size_t)ntg * ngs, s);
  DevBuf<unsigned long long> cnt(1, s);
  KRR_CHECK_HIP(hipMemsetAsync(cnt.p, 0, sizeof(unsigned long long), s));
  hipLaunchKernelGGL(k_cull_masks, dim3((unsigned)ceil_div(ntg * ngs, 256)), dim3(256), 0, s,
                     (const double*)S.box16.p, S.dpad, NF, ntg, ngs, S.cull_mask.p, cnt.p);
  KRR_LAUNCH_CHECK();
  S.cull_nf = NF;
  // automatic mode: culling a small share does not pay for the skip logic (about 5% of the kernel's time
  // measured at a 2% share), so below kCullMin of the steps the operator keeps its spatial order only
  if (cull_mode() < 0) {
    unsigned long long h = 0;
    KRR_CHECK_HIP(hipMemcpyAsync(&h, cnt.p, sizeof(h), hipMemcpyDeviceToHost, s));
    KRR_CHECK_HIP(hipStreamSynchronize(s));
    if ((double)h < kCullMin * 16.0 * (double)ntg * (double)ngs) S.cull_mask.release();
  }
  return S.cull_mask.p;
}

unsigned long long* cull_counters() {
  int dev = 0;
  KRR_CHECK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_cnt_mu);
  auto it = g_cnt_ptr.find(dev);
  if (it != g_cnt_ptr.end()) return it->second;
  void* p = nullptr;
  KRR_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(cull_count)));
  KRR_REQUIRE(p != nullptr, "hipGetSymbolAddress returned no address for the culling counters");
  g_cnt_ptr[dev] = static_cast<unsigned long long*>(p);
  return g_cnt_ptr[dev];
}

void cull_reset_counters(hipStream_t s) {
  hipLaunchKernelGGL(k_cull_zero, dim3(1), dim3(64), 0, s, cull_counters());
  KRR_LAUNCH_CHECK();
}

}  // namespace krr

extern "C" int krr_set_cull(int32_t mode) {
  return krr::guarded([&] {
    KRR_REQUIRE(mode >= -1 && mode <= 2, "mode must be -1 (automatic), 0 (off), 1 (on) or 2 (spatial order only)");
    krr::set_cull_mode(mode);
    return (int)KRR_OK;
  });
}

extern "C" int krr_cull_stats(int64_t* pairs_total, int64_t* pairs_skipped, void* stream) {
  return krr::guarded([&] {
    KRR_REQUIRE(pairs_total && pairs_skipped, "null output pointer");
    const krr::KmvLaunchInfo li = krr::kmv_last_launch();
    *pairs_total = li.npad * li.npad;
    *pairs_skipped = 0;
    if (!li.culled) return (int)KRR_OK;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long c[2] = {0, 0};
    KRR_CHECK_HIP(hipMemcpyAsync(c, krr::cull_counters(), sizeof(c), hipMemcpyDeviceToHost, s));
    KRR_CHECK_HIP(hipStreamSynchronize(s));
    // a skipped step of a diagonal super-tile covers 16 NF x 16 pairs of the product; off the diagonal the
    // evaluated pair serves the pair and its mirror
    const int64_t unit = 16LL * li.nf * 16;
    *pairs_skipped = (int64_t)(c[0] + 2 * c[1]) * unit;
    return (int)KRR_OK;
  });
}
