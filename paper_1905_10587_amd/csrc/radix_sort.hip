// Stable LSD radix sort of (uint64 key, int64 value) pairs, 8-bit digits.
//
// One pass per digit, three kernels each: per-block digit counts of a contiguous chunk of the input, a scan
// of each digit's counts over the blocks (with the digit totals scanned again by every block of the next
// kernel, each block knows where each of its digits starts), and a scatter in which each block walks its chunk in index order, 256 pairs at a time: a pair's place among
// the equal digits of its wave comes from eight ballots (one per digit bit), its place among the earlier
// waves of the same 256 from per-wave counts in LDS, and the running per-digit bases carry over to the next
// 256.  Equal digits therefore keep their input order within a block and, through the scan, across blocks:
// the sort is stable and deterministic.
#include "radix_sort.h"

namespace krr {

namespace {
constexpr int kRsThreads = 256;    // threads per block: one pair each per sub-tile
constexpr int kRsMaxBlocks = 512;  // blocks per pass (each takes a contiguous chunk)
}  // namespace

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                        uint32_t dmask, int64_t chunk, int nblk,
                                                        uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t start = (int64_t)blockIdx.x * chunk;
  const int64_t end = start + chunk < n ? start + chunk : n;
  for (int64_t i = start + tid; i < end; i += kRsThreads) atomicAdd(&h[(keys[i] >> shift) & dmask], 1u);
  __syncthreads();
  hist[(int64_t)tid * nblk + blockIdx.x] = h[tid];
}

// Exclusive scan of each digit's counts over the blocks, in place (block d takes digit d's row of nblk <=
// kRsMaxBlocks counts); the row's total goes to totals[d].
__global__ __launch_bounds__(kRsMaxBlocks) void k_rs_rowscan(uint32_t* __restrict__ hist, int nblk,
                                                             uint32_t* __restrict__ totals) {
  __shared__ uint32_t sm[kRsMaxBlocks];
  const int t = threadIdx.x;
  uint32_t* row = hist + (int64_t)blockIdx.x * nblk;
  const uint32_t v = t < nblk ? row[t] : 0u;
  sm[t] = v;
  __syncthreads();
  for (int o = 1; o < kRsMaxBlocks; o <<= 1) {
    const uint32_t add = t >= o ? sm[t - o] : 0u;
    __syncthreads();
    sm[t] += add;
    __syncthreads();
  }
  if (t < nblk) row[t] = sm[t] - v;
  if (t == kRsMaxBlocks - 1) totals[blockIdx.x] = sm[t];
}

__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                           const int64_t* __restrict__ vin,
                                                           uint64_t* __restrict__ kout, int64_t* __restrict__ vout,
                                                           int64_t n, int shift, uint32_t dmask, int64_t chunk,
                                                           int nblk, const uint32_t* __restrict__ offs,
                                                           const uint32_t* __restrict__ totals) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[4][256];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const uint64_t below = (1ull << lane) - 1ull;   // lanes before this one
  // where digit tid starts: the counts of the smaller digits (a scan of the 256 totals) plus this digit's
  // counts in the earlier blocks
  const uint32_t tot = totals[tid];
  base[tid] = tot;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const uint32_t add = tid >= o ? base[tid - o] : 0u;
    __syncthreads();
    base[tid] += add;
    __syncthreads();
  }
  base[tid] += offs[(int64_t)tid * nblk + blockIdx.x] - tot;
  const int64_t start = (int64_t)blockIdx.x * chunk;
  const int64_t end = start + chunk < n ? start + chunk : n;
  for (int64_t t0 = start; t0 < end; t0 += kRsThreads) {   // block-uniform trip count
#pragma unroll
    for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0u;
    const int64_t i = t0 + tid;
    const bool valid = i < end;
    const uint64_t key = valid ? kin[i] : 0ull;
    const uint32_t d = (uint32_t)(key >> shift) & dmask;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool set = (d >> bit) & 1u;
      const uint64_t m = __ballot(set);
      peers &= set ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & below);
    __syncthreads();   // counts cleared (and the previous sub-tile's bases updated)
    if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t off = base[d] + rank;
      for (int w = 0; w < wave; ++w) off += wcnt[w][d];
      kout[off] = key;
      vout[off] = vin[i];
    }
    __syncthreads();   // every thread has read base and wcnt
    base[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
  }
}

void RadixSortWork::reserve(int64_t n, hipStream_t s) {
  if ((int64_t)tkey.n < n) tkey.alloc((size_t)n, s);
  if ((int64_t)tval.n < n) tval.alloc((size_t)n, s);
  if (hist.n < (size_t)257 * kRsMaxBlocks) hist.alloc((size_t)257 * kRsMaxBlocks, s);   // counts, then totals
}

void radix_sort_pairs(const uint64_t* keys_in, uint64_t* keys_out, const int64_t* vals_in, int64_t* vals_out,
                      int64_t n, int end_bit, RadixSortWork& w, hipStream_t s) {
  KRR_REQUIRE(n >= 0 && n < ((int64_t)1 << 31), "radix sort: n out of range");
  KRR_REQUIRE(end_bit >= 1 && end_bit <= 64, "radix sort: end_bit out of range");
  if (n == 0) return;
  w.reserve(n, s);
  const int passes = (end_bit + 7) / 8;
  const int nblk = (int)std::min<int64_t>(kRsMaxBlocks, std::max<int64_t>(1, ceil_div(n, 2048)));
  const int64_t chunk = round_up(ceil_div(n, nblk), kRsThreads);
  const uint64_t* kin = keys_in;
  const int64_t* vin = vals_in;
  for (int p = 0; p < passes; ++p) {
    // alternate between the output and the work buffers so that the last pass lands in the output
    const bool to_out = (passes - 1 - p) % 2 == 0;
    uint64_t* kout = to_out ? keys_out : w.tkey.p;
    int64_t* vout = to_out ? vals_out : w.tval.p;
    const int shift = 8 * p;
    const uint32_t dmask = end_bit - shift >= 8 ? 255u : (1u << (end_bit - shift)) - 1u;   // bits below end_bit
    hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(kRsThreads), 0, s, kin, n, shift, dmask, chunk, nblk, w.hist.p);
    uint32_t* totals = w.hist.p + (size_t)256 * kRsMaxBlocks;
    hipLaunchKernelGGL(k_rs_rowscan, dim3(256), dim3(kRsMaxBlocks), 0, s, w.hist.p, nblk, totals);
    hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(kRsThreads), 0, s, kin, vin, kout, vout, n, shift, dmask,
                       chunk, nblk, (const uint32_t*)w.hist.p, (const uint32_t*)totals);
    KRR_LAUNCH_CHECK();
    kin = kout;
    vin = vout;
  }
}

}  // namespace krr

extern "C" int krr_radix_sort_pairs(const uint64_t* keys_in, uint64_t* keys_out, const int64_t* vals_in,
                                    int64_t* vals_out, int64_t n, int32_t end_bit, void* stream) {
  return krr::guarded([&] {
    KRR_REQUIRE(n == 0 || (keys_in && keys_out && vals_in && vals_out), "null pointer argument");
    KRR_REQUIRE(n == 0 || (keys_in != keys_out && vals_in != vals_out), "the sort does not work in place");
    krr::RadixSortWork w;
    krr::radix_sort_pairs(keys_in, keys_out, vals_in, vals_out, n, end_bit, w, (hipStream_t)stream);
    return (int)KRR_OK;
  });
}
