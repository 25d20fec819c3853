// H|psi> kernels and launcher for the 24^3 FFT mesh, both precisions.
#include "hpsi_kernel.hpp"

namespace mkpw {
MKPW_HPSI_INSTANTIATE(24)
}  // namespace mkpw
