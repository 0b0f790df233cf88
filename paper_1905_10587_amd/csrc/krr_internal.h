// Internal helpers shared by the library's translation units: status/error reporting,
// device memory from the registered allocator, launch checks, small device utilities.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/krr.h"

namespace krr {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
const char* get_error();

struct Error {
  int code;
  std::string msg;
};

#define KRR_CHECK_HIP(expr)                                                                  \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      throw ::krr::Error{KRR_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)};       \
  } while (0)

#define KRR_REQUIRE(cond, msg)                                                               \
  do {                                                                                       \
    if (!(cond)) throw ::krr::Error{KRR_EINVAL, std::string(msg)};                           \
  } while (0)

#define KRR_LAUNCH_CHECK() KRR_CHECK_HIP(hipGetLastError())

// Runs body, converting exceptions into a status code and the thread-local message.
template <typename F>
int guarded(F&& body) {
  try {
    set_error("");
    return body();
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(std::string("internal error: ") + e.what());
    return KRR_EHIP;
  }
}

// ------------------------------------------------------------------ memory
void* dev_alloc(size_t bytes, hipStream_t stream);
void dev_free(void* p, hipStream_t stream);

// Owning device buffer released (stream-ordered) at scope exit.
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  hipStream_t s = nullptr;
  DevBuf() = default;
  DevBuf(size_t count, hipStream_t stream) { alloc(count, stream); }
  void alloc(size_t count, hipStream_t stream) {
    release();
    s = stream;
    n = count;
    if (count) p = static_cast<T*>(dev_alloc(count * sizeof(T), stream));
  }
  void release() {
    if (p) dev_free(p, s);
    p = nullptr;
    n = 0;
  }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), s(o.s) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; s = o.s; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  size_t bytes() const { return n * sizeof(T); }
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// ------------------------------------------------------------------ validation
void check_finite_device(const double* p, int64_t count, const char* what, hipStream_t s);

// ------------------------------------------------------------------ constants
constexpr double kLog2e = 1.4426950408889634073599246810018921;   // log2(e)
constexpr double kLn2 = 0.6931471805599453094172321214581765680755; // ln(2)

}  // namespace krr
