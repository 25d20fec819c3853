// Host-side helpers shared by the solver entry points: a scope-bound set of
// device work buffers and the status-propagation macros.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "internal.hpp"

namespace mkpw {

// Device buffers from the context's (budgeted, stream-ordered) allocator,
// freed together when the object goes out of scope.
struct DevBufs {
  pw_ctx* c;
  std::vector<void*> ptrs;
  explicit DevBufs(pw_ctx* cc) : c(cc) {}
  DevBufs(const DevBufs&) = delete;
  DevBufs& operator=(const DevBufs&) = delete;
  ~DevBufs() {
    for (void* p : ptrs) dev_free(c, p);
  }
  template <class T>
  pw_status get(size_t n, T** out) {
    void* p = nullptr;
    pw_status s = dev_alloc(c, n * sizeof(T), &p);
    if (s != PW_OK) return s;
    ptrs.push_back(p);
    *out = (T*)p;
    return PW_OK;
  }
};

}  // namespace mkpw

// return the status of x unless it is PW_OK
#define MKPW_TRY(x)                 \
  do {                              \
    pw_status s_ = (x);             \
    if (s_ != PW_OK) return s_;     \
  } while (0)

// return PW_EDEVICE with the HIP error text if the HIP call fails
#define MKPW_HIP(c, call)                                                                      \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      (void)hipGetLastError();                                                                 \
      return mkpw::set_err((c), PW_EDEVICE, std::string(#call " failed: ") + hipGetErrorString(e_)); \
    }                                                                                          \
  } while (0)
