// Learned correction of the preconditioner inside flexible GMRES.
#include <hip/hip_runtime.h>

#include "engine.h"

namespace pfft {

bool learned_apply(pfft_ctx *c, int R, const double2 *v, double2 *z, hipStream_t st) {
  (void)c; (void)R; (void)v; (void)z; (void)st;
  return false;
}

}  // namespace pfft

void learned_free(pfft_ctx *c) { (void)c; }

extern "C" pfft_status pfft_precond_load(pfft_ctx *c, const void *w, int64_t nbytes) {
  (void)c; (void)w; (void)nbytes;
  pfft::set_error("pfft_precond_load: no learned correction in this build");
  return PFFT_EINVAL;
}
