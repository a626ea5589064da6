// Context of the C ABI: host model, device arrays, workspaces.
#pragma once
#include <algorithm>
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

// Per-product workspace for up to R right-hand sides (one per stream lane).
struct Workspace {
  int R = 0;
  bool fixed = false;   // carved from caller-independent scratch: never (re)allocated
  std::vector<void *> allocs;
  double2 *alpha = nullptr, *scan = nullptr, *part = nullptr, *U = nullptr, *yb = nullptr, *coef = nullptr;
  void *J = nullptr, *Q = nullptr, *T1 = nullptr, *T2 = nullptr;
  std::vector<double2> host_coef;
  std::vector<double2> coef_on_device;   // what coef holds (single-chunk ranges), empty if unknown
};

}  // namespace pfft

struct pfft_ctx {
  pfft::HostModel m;
  int grid_fp64 = 0;
  double sigma = 5.8e7, mu_r = 1.0;
  int max_chunk = 0;
  size_t ws_budget = (size_t)24 << 30;   // product workspace bytes (chunk size)
  int device = 0;
  void *scratch = nullptr;   // this device's no-allocation scratch (address of the static array)
  pfft::Workspace ws_fixed;  // carved from scratch by pfft_matvec_noalloc
  std::vector<void *> allocs;
  size_t dev_bytes = 0;
  pfft::LoopMaps lm{};
  pfft::GridMaps gm{};
  pfft::CombineMaps cm{};
  // per-product workspaces and the two stream lanes the right-hand sides
  // are split over (fork/join by events on the caller's stream)
  static constexpr int kLanes = 2;   // stream lanes of the split product (four measured slower)
  pfft::Workspace ws[kLanes];
  hipStream_t lane[kLanes] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kLanes] = {};
  // plan options (pfft_set_option, pfft_autotune)
  struct Plans {
    int fft = 0;      // 0 register-resident FFT passes where the shape allows, 1 LDS Stockham
    int ldl = 0;      // 0 register-window band solve when the band fits a wave, 1 LDS window
    int proj = 0;     // 0 tiled projection, 1 node-major gather
    int proj_rhs = 0; // tiled projection (FP32): 0 16 right-hand sides per workgroup, 1 eight
    int graphs = 1;   // 1 FGMRES replays the product and P^-1 as HIP graphs
    int stream_split = 0;  // 1: the right-hand sides of a product are split over kLanes streams
    int factor = 0;   // 0 preconditioner factored on the device, 1 on the host
    int comb = 0;     // 0 LDS-tiled near-field product when the tiles fit, 1 gather
    int prune = 1;    // 1 register FFT passes skip grid columns and nodes no stencil touches
    int near_dense = 1;  // 1 near field on FP64 matrix cores over dense row tiles (when built)
    int nd = 0;       // preconditioner ordering: 0 nested dissection for wide bands only, 1 always
  } plans;
  pfft::StageTimer timer;
  // solver state
  pfft::Precond *pre = nullptr;
  pfft::Learned *learned = nullptr;

  void *dalloc(size_t bytes);
  size_t per_rhs_bytes() const;
  int chunk_for(int R) const;
  void ensure_workspace(pfft::Workspace &w, int R);
  // frees the product workspaces (not the fixed one); the next product
  // allocates them again for its own chunk and plans
  void release_workspaces();
  // y = op(x) for R right-hand sides already resident on the device
  void matvec(int R, const double *omega, int space, int flags, const double2 *x, double2 *y,
              hipStream_t st);
  // op for right-hand sides [0, R) of x/y/omega on stream st with workspace w
  // post (loop space only, optional): also writes the post-processing
  // outputs of x taken as loop currents (rows offset by the chunk)
  void matvec_range(pfft::Workspace &w, int R, const double *omega, int space, int flags, const double2 *x,
                    double2 *y, hipStream_t st, const pfft::PostOut *post = nullptr);
  // device maps of the post-processing (built on first use)
  int *d_tri_pos = nullptr, *d_tri_ref = nullptr, *d_port_loop = nullptr;
  // Runs fn(r0, rn, stream, workspace) for the right-hand sides [0, R),
  // split over the kLanes stream lanes when enabled (not while profiling).
  template <typename Fn> void run_split(int R, hipStream_t st, Fn &&fn);
  bool split_ok(int R) const { return plans.stream_split == 1 && !timer.on && R >= 8; }
};

template <typename Fn>
void pfft_ctx::run_split(int R, hipStream_t st, Fn &&fn) {
  if (!split_ok(R)) {
    fn(0, R, st, ws[0]);
    return;
  }
  for (int i = 0; i < kLanes; ++i)
    if (!lane[i]) {
      pfft::hip_ok(hipStreamCreateWithFlags(&lane[i], hipStreamNonBlocking), "lane stream");
      pfft::hip_ok(hipEventCreateWithFlags(&ev_join[i], hipEventDisableTiming), "lane event");
    }
  if (!ev_fork) pfft::hip_ok(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming), "fork event");
  pfft::hip_ok(hipEventRecord(ev_fork, st), "fork");
  const int q = (R + kLanes - 1) / kLanes;
  for (int i = 0; i < kLanes; ++i) {
    const int r0 = i * q, rn = std::min(R, r0 + q) - r0;
    if (rn <= 0) break;
    pfft::hip_ok(hipStreamWaitEvent(lane[i], ev_fork, 0), "fork wait");
    fn(r0, rn, lane[i], ws[i]);
    pfft::hip_ok(hipEventRecord(ev_join[i], lane[i]), "join");
    pfft::hip_ok(hipStreamWaitEvent(st, ev_join[i], 0), "join wait");
  }
}

// 1 / 0 when the context's preconditioner uses nested dissection or the
// band, -1 before it is built (defined with the solver)
int precond_uses_nd(const pfft_ctx *c);
// P^-1 (Z_l x) or P^-1 x in loop space (defined with the solver)
pfft_status pfft_internal_precond_matvec(pfft_ctx *c, int R, const double *omega, int flags,
                                         const double2 *x, double2 *y, hipStream_t st);
void pfft_ctx_free(pfft_ctx *c);
