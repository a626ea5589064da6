// Preconditioner (Eq. Precond), flexible GMRES and port solves (Sec. IV-A, V).
#include <hip/hip_runtime.h>

#include "engine.h"

using namespace pfft;

void pfft_ctx_free(pfft_ctx *c) {
  for (void *p : c->ws_allocs) hipFree(p);
  for (void *p : c->allocs) hipFree(p);
  delete c;
}

pfft_status pfft_internal_precond_matvec(pfft_ctx *c, int R, const double *omega, int flags, const double2 *x,
                                         double2 *y, hipStream_t st) {
  (void)c; (void)R; (void)omega; (void)flags; (void)x; (void)y; (void)st;
  set_error("pfft_matvec: preconditioner not available");
  return PFFT_EINVAL;
}

extern "C" {

pfft_status solve_ports(pfft_ctx *c, int32_t nfreq, const double *freq_hz, double tol, int32_t maxit,
                        int32_t restart, int32_t precond, void *Y_out, int32_t *iters_out, double *relres_out,
                        void *hip_stream) {
  (void)c; (void)nfreq; (void)freq_hz; (void)tol; (void)maxit; (void)restart; (void)precond;
  (void)Y_out; (void)iters_out; (void)relres_out; (void)hip_stream;
  set_error("solve_ports: not available");
  return PFFT_EINVAL;
}

pfft_status pfft_precond_load(pfft_ctx *c, const void *w, int64_t nbytes) {
  (void)c; (void)w; (void)nbytes;
  set_error("pfft_precond_load: not available");
  return PFFT_EINVAL;
}

}  // extern "C"
