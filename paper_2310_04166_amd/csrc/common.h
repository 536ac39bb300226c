// Shared plumbing of the library: status handling, HIP checks, small device
// helpers.  Nothing here knows about the method.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

#include "../../include/nqs.h"

namespace nqs {

// An error carrying its C-ABI status; thrown inside the library, turned into
// a return code at the boundary.
struct Error : std::runtime_error {
  int status;
  Error(int s, const std::string &msg) : std::runtime_error(msg), status(s) {}
};

void set_last_error(const std::string &msg);

#define NQS_REQUIRE(cond, status, msg)                                        \
  do {                                                                        \
    if (!(cond)) throw ::nqs::Error((status), std::string(msg));              \
  } while (0)

#define HIP_OK(expr)                                                          \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess)                                                     \
      throw ::nqs::Error(e_ == hipErrorOutOfMemory ? NQS_ENOMEM : NQS_EHIP,   \
                         std::string(#expr " failed: ") + hipGetErrorString(e_)); \
  } while (0)

#define HIP_LAUNCH_OK()                                                       \
  do {                                                                        \
    hipError_t e_ = hipGetLastError();                                        \
    if (e_ != hipSuccess)                                                     \
      throw ::nqs::Error(NQS_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

// Run f, translating exceptions into a status code.
template <class F>
int guarded(F &&f) {
  try {
    f();
    return NQS_OK;
  } catch (const Error &e) {
    set_last_error(e.what());
    return e.status;
  } catch (const std::bad_alloc &) {
    set_last_error("host allocation failed");
    return NQS_ENOMEM;
  } catch (const std::exception &e) {
    set_last_error(e.what());
    return NQS_EINVAL;
  } catch (...) {
    set_last_error("unknown error");
    return NQS_EINVAL;
  }
}

// A growable device buffer owned by the library.
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  // Grow to at least n bytes (contents are not kept).
  void *reserve(size_t n) {
    if (n <= bytes && ptr) return ptr;
    release();
    size_t want = n < 256 ? 256 : n;
    HIP_OK(hipMalloc(&ptr, want));
    bytes = want;
    return ptr;
  }
  template <class T>
  T *as() const { return static_cast<T *>(ptr); }
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline hipStream_t as_stream(nqs_stream s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace nqs
