// Context of the C ABI: host model, device arrays, workspaces.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/pfft.h"
#include "kernels.h"
#include "model.h"

namespace pfft {

struct DeviceError {
  int code;
  std::string msg;
};

void set_error(const std::string &msg);
void hip_ok(hipError_t e, const char *what);

// Per-stage HIP-event timing of the hot path (enabled with pfft_profile).
enum Stage {
  ST_LOOP_TO_BRANCH = 0, ST_TRI_CURRENT, ST_PROJECT, ST_FFT_X, ST_FFT_Y, ST_FFT_Z_CONV, ST_IFFT_Y,
  ST_IFFT_X, ST_INTERP, ST_COMBINE, ST_BRANCH_TO_LOOP, ST_PRECOND, ST_COUNT
};

struct StageTimer {
  bool on = false;
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  double ms[ST_COUNT] = {0};
  long long calls[ST_COUNT] = {0};
  int open_stage = -1;
  hipEvent_t open_ev = nullptr;
  void begin(int s, hipStream_t st);
  void end(hipStream_t st);
  void collect();   // waits for recorded events, folds them into ms/calls
};

struct Precond;   // nodal-route preconditioner factors (one per frequency)
struct Learned;   // learned correction network

}  // namespace pfft

struct pfft_ctx {
  pfft::HostModel m;
  int grid_fp64 = 0;
  double sigma = 5.8e7, mu_r = 1.0;
  int max_chunk = 0;
  int device = 0;
  std::vector<void *> allocs;
  size_t dev_bytes = 0;
  pfft::LoopMaps lm{};
  pfft::GridMaps gm{};
  pfft::CombineMaps cm{};
  // per-matvec workspace, sized for ws_R right-hand sides
  int ws_R = 0;
  std::vector<void *> ws_allocs;
  double2 *ws_alpha = nullptr, *ws_scan = nullptr, *ws_part = nullptr, *ws_U = nullptr,
          *ws_yb = nullptr, *ws_coef = nullptr;
  void *ws_J = nullptr, *ws_Q = nullptr, *ws_T1 = nullptr, *ws_T2 = nullptr;
  std::vector<double2> host_coef;
  std::vector<double2> coef_on_device;   // what ws_coef holds (single-chunk calls), empty if unknown
  // plan options (pfft_set_option, pfft_autotune)
  struct Plans {
    int fft = 0;      // 0 register-resident FFT passes where the shape allows, 1 LDS Stockham
    int ldl = 0;      // 0 register-window band solve when the band fits a wave, 1 LDS window
    int proj = 0;     // 0 tiled projection, 1 node-major gather
    int graphs = 1;   // 1 FGMRES replays the product and P^-1 as HIP graphs
  } plans;
  pfft::StageTimer timer;
  // solver state
  pfft::Precond *pre = nullptr;
  pfft::Learned *learned = nullptr;

  void *dalloc(size_t bytes);
  size_t per_rhs_bytes() const;
  int chunk_for(int R) const;
  void ensure_workspace(int R);
  // y = op(x) for R right-hand sides already resident on the device
  void matvec(int R, const double *omega, int space, int flags, const double2 *x, double2 *y,
              hipStream_t st);
};

// P^-1 (Z_l x) or P^-1 x in loop space (defined with the solver)
pfft_status pfft_internal_precond_matvec(pfft_ctx *c, int R, const double *omega, int flags,
                                         const double2 *x, double2 *y, hipStream_t st);
void pfft_ctx_free(pfft_ctx *c);
