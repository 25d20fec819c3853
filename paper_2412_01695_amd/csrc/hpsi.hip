// Entry of the batched H|psi> (Sec. 3, Algorithm new_gpu): mesh dispatch to the
// fused kernel instantiated for each supported mesh (hpsi_kernel.hpp,
// hpsi_n<N>.hip) and the process-wide autotuning table.
#include <hip/hip_runtime.h>

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
pw_status launch_t(pw_ctx* c, const VecSel& sel, const void* psi, void* hpsi, hipStream_t st) {
  switch (c->fft[0]) {
    case 15: return launch_n<T, 15>(c, sel, psi, hpsi, st);
    case 18: return launch_n<T, 18>(c, sel, psi, hpsi, st);
    case 20: return launch_n<T, 20>(c, sel, psi, hpsi, st);
    case 24: return launch_n<T, 24>(c, sel, psi, hpsi, st);
    case 30: return launch_n<T, 30>(c, sel, psi, hpsi, st);
    case 32: return launch_n<T, 32>(c, sel, psi, hpsi, st);
    case 36: return launch_n<T, 36>(c, sel, psi, hpsi, st);
    default: break;
  }
  return set_err(c, PW_EINVAL, "unsupported FFT mesh");
}

}  // namespace

bool hpsi_supported(int n1, int n2, int n3) {
  if (n1 != n2 || n1 != n3) return false;
  for (int n : kMeshes)
    if (n == n1) return true;
  return false;
}

pw_status launch_hpsi(pw_ctx* c, pw_prec prec, const VecSel& sel, const void* psi, void* hpsi, hipStream_t st) {
  if (!hpsi_supported(c->fft[0], c->fft[1], c->fft[2]))
    return set_err(c, PW_EINVAL,
                   "unsupported FFT mesh " + std::to_string(c->fft[0]) + "x" + std::to_string(c->fft[1]) + "x" +
                       std::to_string(c->fft[2]) + " (cubic 15, 18, 20, 24, 30, 32, 36)");
  if (prec == PW_FP64) return launch_t<double>(c, sel, psi, hpsi, st);
  return launch_t<float>(c, sel, psi, hpsi, st);
}

}  // namespace mkpw
