// Runtime support: thread-local error messages, the device allocator hook, input validation.
#include <hip/hip_runtime.h>

#include <mutex>

#include "krr_internal.h"

namespace krr {

namespace {
thread_local std::string t_error;
std::mutex g_alloc_mu;
void* (*g_alloc)(size_t, void*, void*) = nullptr;
void (*g_free)(void*, void*) = nullptr;
void* g_ctx = nullptr;
}  // namespace

void set_error(const std::string& msg) { t_error = msg; }
const char* get_error() { return t_error.c_str(); }

void* dev_alloc(size_t bytes, hipStream_t stream) {
  void* (*a)(size_t, void*, void*);
  void* ctx;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    a = g_alloc;
    ctx = g_ctx;
  }
  void* p = nullptr;
  if (a) {
    p = a(bytes, (void*)stream, ctx);
    if (!p) throw Error{KRR_ENOMEM, "allocator callback returned NULL for " + std::to_string(bytes) + " bytes"};
    return p;
  }
  hipError_t e = hipMallocAsync(&p, bytes, stream);
  if (e != hipSuccess || !p)
    throw Error{KRR_ENOMEM, "hipMallocAsync(" + std::to_string(bytes) + "): " + hipGetErrorString(e)};
  return p;
}

void dev_free(void* p, hipStream_t stream) {
  if (!p) return;
  void (*f)(void*, void*);
  void* ctx;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    f = g_alloc ? g_free : nullptr;
    ctx = g_ctx;
  }
  if (f) f(p, ctx);
  else (void)hipFreeAsync(p, stream);   // errors on release are not recoverable; ignore
}

// ------------------------------------------------------------------ non-finite input check
__global__ void k_count_nonfinite(const double* __restrict__ p, int64_t n, unsigned int* __restrict__ bad) {
  unsigned int local = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    local |= !isfinite(p[i]);
  if (local) atomicOr(bad, 1u);
}

void check_finite_device(const double* p, int64_t count, const char* what, hipStream_t s) {
  if (count <= 0) return;
  DevBuf<unsigned int> flag(1, s);
  KRR_CHECK_HIP(hipMemsetAsync(flag.p, 0, sizeof(unsigned int), s));
  const int64_t blocks = std::min<int64_t>(ceil_div(count, 256), 4096);
  hipLaunchKernelGGL(k_count_nonfinite, dim3((unsigned)blocks), dim3(256), 0, s, p, count, flag.p);
  KRR_LAUNCH_CHECK();
  unsigned int h = 0;
  KRR_CHECK_HIP(hipMemcpyAsync(&h, flag.p, sizeof(h), hipMemcpyDeviceToHost, s));
  KRR_CHECK_HIP(hipStreamSynchronize(s));
  if (h) throw Error{KRR_EINVAL, std::string(what) + " contains NaN or Inf"};
}

}  // namespace krr

extern "C" {

int krr_version(void) { return 10000; }

const char* krr_last_error(void) { return krr::get_error(); }

int krr_set_allocator(void* (*alloc)(size_t, void*, void*), void (*free_)(void*, void*), void* ctx) {
  return krr::guarded([&] {
    KRR_REQUIRE((alloc == nullptr) == (free_ == nullptr), "alloc and free must both be set or both be NULL");
    std::lock_guard<std::mutex> lk(krr::g_alloc_mu);
    krr::g_alloc = alloc;
    krr::g_free = free_;
    krr::g_ctx = ctx;
    return (int)KRR_OK;
  });
}

}  // extern "C"
