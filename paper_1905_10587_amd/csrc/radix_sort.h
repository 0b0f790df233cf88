// Stable least-significant-digit radix sort of (uint64 key, int64 value) pairs on the device: the order of
// the pivoted QR's candidate set (column norms) and of the spatial (Morton) staging of culled operators.
#pragma once

#include "krr_internal.h"

namespace krr {

// Work buffers of one sort size (reused across calls of the same or a smaller n).
struct RadixSortWork {
  DevBuf<uint64_t> tkey;
  DevBuf<int64_t> tval;
  DevBuf<uint32_t> hist;
  void reserve(int64_t n, hipStream_t s);
};

// keys_out / vals_out = the pairs ordered by key bits [0, end_bit), ascending; pairs with equal bits keep
// their input order.  keys_in / vals_in are not modified.  n >= 0, 1 <= end_bit <= 64; the four arrays
// are device memory of n entries and must not overlap.  Deterministic.
void radix_sort_pairs(const uint64_t* keys_in, uint64_t* keys_out, const int64_t* vals_in, int64_t* vals_out,
                      int64_t n, int end_bit, RadixSortWork& w, hipStream_t s);

}  // namespace krr
