// Host-side helpers shared by the solver entry points: the status-propagation
// macros, a scope-bound set of device work buffers and page-locked staging for
// small copies.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"

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

// Page-locked staging for a solver's small host<->device copies.  A copy from
// pageable memory is staged by the runtime while the device waits (tens of
// microseconds each); from page-locked memory it is one asynchronous transfer.
// Uploads take consecutive slices of the upload area, untouched until sync(),
// so the host may change its arrays as soon as an upload is queued (an upload
// that does not fit synchronises first).  The read-back area follows it; the
// caller addresses it with back().
class HostStage {
 public:
  HostStage(pw_ctx* c, hipStream_t st) : c_(c), st_(st) {}
  pw_status init(size_t up_bytes, size_t back_bytes) {
    up_cap_ = align(up_bytes);
    void* p = nullptr;
    MKPW_TRY(host_pinned(c_, up_cap_ + align(back_bytes), &p));
    base_ = (char*)p;
    used_ = 0;
    return PW_OK;
  }
  template <class T>
  hipError_t up(T* d, const T* h, size_t n) {
    const size_t bytes = n * sizeof(T);
    if (used_ + align(bytes) > up_cap_) {
      hipError_t e = sync();
      if (e != hipSuccess) return e;
      if (align(bytes) > up_cap_) {  // larger than the whole area: copied and waited for
        e = hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st_);
        return e != hipSuccess ? e : sync();
      }
    }
    char* p = base_ + used_;
    std::memcpy(p, h, bytes);
    used_ += align(bytes);
    return hipMemcpyAsync(d, p, bytes, hipMemcpyHostToDevice, st_);
  }
  template <class T>
  T* back(size_t offset_bytes) const {
    return reinterpret_cast<T*>(base_ + up_cap_ + offset_bytes);
  }
  hipError_t sync() {
    hipError_t e = hipStreamSynchronize(st_);
    used_ = 0;
    return e;
  }

 private:
  static size_t align(size_t b) { return (b + 255) & ~(size_t)255; }
  pw_ctx* c_;
  hipStream_t st_;
  char* base_ = nullptr;
  size_t up_cap_ = 0, used_ = 0;
};

}  // namespace mkpw
