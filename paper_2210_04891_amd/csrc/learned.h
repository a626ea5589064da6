// Internal interface between the FGMRES driver and the learned correction.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <vector>

struct pfft_ctx;

namespace pfft {

// z = P^-1 v + learned correction (per right-hand side; a right-hand side
// whose correction is not finite or too large keeps P^-1 v).  Returns false,
// touching nothing, when the context has no network.
// enable (host [R], may be NULL = all): right-hand sides that get the
// correction; false when none does.
bool learned_apply(pfft_ctx *c, int R, const double *omega, const double2 *v, double2 *z, const uint8_t *enable,
                   hipStream_t st);
// Per-step residual reduction factor of the plain preconditioner measured
// when the training pairs were collected (times a 1.1 margin); 0 when unknown.
double learned_judge_factor(pfft_ctx *c);
void learned_judged_off(pfft_ctx *c, int n);
// Sets the convergence judge's per-step factor (0 disables switching).
void learned_set_judge(pfft_ctx *c, double factor);
void learned_free(pfft_ctx *c);

// One-cycle port solve with the plain preconditioner (restart = maxit,
// x0 = 0) that exposes its Krylov data: V [R][m+1][l] (v_0 = b/|b|),
// Z [R][m][l] with z_k = P^-1 v_k, the unrotated Hessenberg Hraw [R][m+1][m]
// (Z_l z_k = sum_i Hraw[i][k] v_i), the final iterate x [R][l] (device), and
// per RHS the Krylov length k, the residual estimates after each step,
// |b| and the final true relative residual (host).
struct KrylovView {
  int R, l, m;
  const double2 *V, *Z, *Hraw, *x;
  const double *omega;
  std::vector<int> k;
  std::vector<std::vector<double>> res;
  std::vector<double> bnorm, relres;
};
using KrylovFn = std::function<void(const KrylovView &)>;
void solve_ports_krylov(pfft_ctx *c, int nfreq, const double *freq_hz, double tol, int maxit, const KrylovFn &done,
                        hipStream_t st);

}  // namespace pfft
