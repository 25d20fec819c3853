// Entry of the batched H|psi> (Sec. 3, Algorithm new_gpu): mesh dispatch to the
// fused kernel instantiated for each supported mesh (hpsi_kernel.hpp,
// hpsi_n<N>.hip) and the process-wide autotuning table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hpsi_kernel.hpp"

namespace mkpw {

std::mutex g_hpsi_tune_mu;
std::map<std::vector<long>, HpsiShape> g_hpsi_tuned;

MKPW_HPSI_EXTERN(15)
MKPW_HPSI_EXTERN(18)
MKPW_HPSI_EXTERN(20)
MKPW_HPSI_EXTERN(24)
MKPW_HPSI_EXTERN(30)
MKPW_HPSI_EXTERN(32)
MKPW_HPSI_EXTERN(36)

namespace {

constexpr int kMeshes[] = {15, 18, 20, 24, 30, 32, 36};

template <class T>
pw_status launch_t(pw_ctx* c, const VecSel& sel, const void* psi, void* hpsi, hipStream_t st, void* vscratch) {
  switch (c->fft[0]) {
    case 15: return launch_n<T, 15>(c, sel, psi, hpsi, st, vscratch);
    case 18: return launch_n<T, 18>(c, sel, psi, hpsi, st, vscratch);
    case 20: return launch_n<T, 20>(c, sel, psi, hpsi, st, vscratch);
    case 24: return launch_n<T, 24>(c, sel, psi, hpsi, st, vscratch);
    case 30: return launch_n<T, 30>(c, sel, psi, hpsi, st, vscratch);
    case 32: return launch_n<T, 32>(c, sel, psi, hpsi, st, vscratch);
    case 36: return launch_n<T, 36>(c, sel, psi, hpsi, st, vscratch);
    default: break;
  }
  return set_err(c, PW_EINVAL, "unsupported FFT mesh");
}

// Staging of pw_h_psi_noalloc: the potential permuted for the kernel's slab
// width (N^3 values of the launch's precision) or the x-line convolution taps
// (N^2 lines x at most N + 3 complex taps), for every supported mesh (the
// largest is 36^3 in FP64: 36^2 x 39 complex doubles).  One copy per GPU,
// held until the process ends.
constexpr size_t kNoallocScratchBytes = 36u * 36u * 39u * 2u * sizeof(double);
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

// Its device address per GPU (the array's name is a host-side stand-in, not a
// device address), looked up once per device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

}  // namespace

// Looks up this device's copy of the no-allocation staging array; called by
// pw_create with the context's device current.
pw_status hpsi_scratch_init(pw_ctx* c) {
  if (c->device < 0 || c->device >= kMaxDevices) return PW_OK;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_done[c->device]) return PW_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return set_err(c, PW_EDEVICE, std::string("hipGetSymbolAddress of the H|psi> staging array failed: ") +
                                      hipGetErrorString(e));
  }
  g_scratch_ptr[c->device] = ptr;
  g_scratch_done[c->device] = true;
  return PW_OK;
}

bool hpsi_supported(int n1, int n2, int n3) {
  if (n1 != n2 || n1 != n3) return false;
  for (int n : kMeshes)
    if (n == n1) return true;
  return false;
}

pw_status launch_hpsi(pw_ctx* c, pw_prec prec, const VecSel& sel, const void* psi, void* hpsi, hipStream_t st,
                      void* vscratch) {
  if (!hpsi_supported(c->fft[0], c->fft[1], c->fft[2]))
    return set_err(c, PW_EINVAL,
                   "unsupported FFT mesh " + std::to_string(c->fft[0]) + "x" + std::to_string(c->fft[1]) + "x" +
                       std::to_string(c->fft[2]) + " (cubic 15, 18, 20, 24, 30, 32, 36)");
  if (prec == PW_FP64) return launch_t<double>(c, sel, psi, hpsi, st, vscratch);
  return launch_t<float>(c, sel, psi, hpsi, st, vscratch);
}

}  // namespace mkpw

extern "C" pw_status pw_h_psi_noalloc(pw_ctx* c, pw_prec prec, int nbnd, const void* psi, void* hpsi) {
  using namespace mkpw;
  if (!c) return PW_EINVAL;
  if (c->host_only) return set_err(c, PW_ESTATE, "host-only context runs no device work");
  if (!c->have_k || !c->have_v) return set_err(c, PW_ESTATE, "set k-points and potential before h_psi");
  if (prec != PW_FP64 && prec != PW_MIXED) return set_err(c, PW_EINVAL, "unknown precision");
  if (nbnd <= 0 || nbnd > 65535) return set_err(c, PW_EINVAL, "nbnd must be in [1, 65535]");
  if (!psi || !hpsi) return set_err(c, PW_EINVAL, "null psi or hpsi");
  const size_t real = prec == PW_FP64 ? sizeof(double) : sizeof(float);
  const size_t n = (size_t)c->fft[0];
  const size_t need = std::max(n * n * n * real, n * n * (n + 3) * 2 * real);
  if (need > kNoallocScratchBytes)
    return set_err(c, PW_EINVAL, "pw_h_psi_noalloc: the mesh needs " + std::to_string(need) +
                                     " bytes of staging, more than its " + std::to_string(kNoallocScratchBytes));
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (c->device >= 0 && c->device < kMaxDevices) ptr = g_scratch_ptr[c->device];
  }
  if (!ptr) return set_err(c, PW_EDEVICE, "pw_h_psi_noalloc: no staging array on this device");
  (void)hipSetDevice(c->device);
  VecSel sel;
  sel.nvec = nbnd;
  sel.kstride = (long)nbnd * c->npwx;
  return launch_hpsi(c, prec, sel, psi, hpsi, c->stream, ptr);
}
