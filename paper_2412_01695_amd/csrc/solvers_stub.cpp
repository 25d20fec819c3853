// Temporary: solver entry points until the batched Davidson and CG land.
#include "internal.hpp"

extern "C" {
pw_status pw_davidson(pw_ctx* c, pw_prec, int, void*, double*, double, int, int32_t*, int32_t*) {
  return mkpw::set_err(c, PW_ESTATE, "pw_davidson: not built yet");
}
pw_status pw_dfpt_cg(pw_ctx* c, pw_prec, int, const void*, const double*, const double*, int, const void*, void*,
                     double, int, int32_t*) {
  return mkpw::set_err(c, PW_ESTATE, "pw_dfpt_cg: not built yet");
}
}
