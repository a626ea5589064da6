// Preconditioner P = A diag(Z_b) A^T (Eq. Precond) applied through the node
// space.  For e = E_L y (loop EMFs placed on the links) and D = diag(Z_b):
//     P^-1 y = E_L^T [ D^-1 e - D^-1 N^T (N D^-1 N^T)^-1 N D^-1 e ]
// (the loop-space and node-space projectors are complementary), so one solve
// with the nodal matrix L_w = N D^-1 N^T replaces the factorization of P.  A
// port's zero-impedance source branch ties its sink node to its source node
// (supernode with a known potential offset); one node per conductor is
// grounded.  L_w is ordered on the host (reverse Cuthill-McKee per
// conductor, supernodes last), factored per frequency (LDL^T without
// pivoting: Re L_w is positive definite) on the device, or on the host, and
// solved on the device.
#pragma once
#include <hip/hip_runtime.h>

#include <complex>
#include <map>
#include <vector>

#include "model.h"

namespace pfft {

struct PrecondStruct {
  int nu = 0;                     // unknowns (merged, grounded nodes removed)
  int ncomp = 0;
  int W = 0;                      // max envelope width of the band rows
  std::vector<int> comp_off;      // [ncomp+1] unknown ranges
  std::vector<int> comp_mid;      // [ncomp] first dense (supernode) row of each conductor:
                                  // rows [comp_off, comp_mid) form a narrow band,
                                  // rows [comp_mid, comp_off+1) are supernodes ordered last
  std::vector<int> first;         // [nu] first column of each row's envelope
  std::vector<int64_t> env_off;   // [nu+1]
  // column profile of L: column j spans rows j+1 .. clast[j] (zeros where a
  // row's envelope starts later)
  int Wc = 0;
  std::vector<int> clast;         // [nu]
  // pitches of the padded row / column layouts: 64 (zero beyond the band)
  // when both band widths are at most 63, else max(W, 1) / max(Wc, 1)
  int pr = 1, pc = 1;
  std::vector<int64_t> col_off;   // [nu+1]
  // branch data (mesh edges)
  std::vector<int> br_ru, br_rv;  // unknown of merged end nodes (-1: ground)
  std::vector<int> br_link;       // link index or -1
  std::vector<int> br_offu, br_offv;  // port whose EMF offsets the end node (-1: none)
  // unknown -> incident branches (sign +1 leaving, -1 entering)
  std::vector<int> inc_off, inc_br;
  std::vector<int8_t> inc_sg;
  // source node of each port -> incident mesh branches (unmerged)
  std::vector<int> src_off, src_br;
  std::vector<int8_t> src_sg;
  // per link: branch id (mesh) or -(port+1)
  std::vector<int> link_kind;
  std::vector<int> port_loop;
  // ---- nested-dissection ordering (nd = true): a conductor's unknowns are
  // ordered by recursive geometric bisection with vertex separators (each
  // separator after the two halves it splits, a conductor's port
  // supernodes after everything else), and L_w is factored by supernodes:
  // supernode s holds the contiguous unknowns [sn_start[s], sn_start[s+1])
  // and, below them, the rows st_ids[st_off[s] .. st_off[s+1]) (its
  // "structure": ascending unknowns of ancestor supernodes).  The band
  // fields above (first, env_off, clast, col_off, W, Wc) are unused then.
  bool nd = false;
  int nsn = 0;
  std::vector<int> sn_start;        // [nsn + 1]
  std::vector<int> sn_parent;       // [nsn] (-1: root of a conductor)
  std::vector<int> sn_height;       // [nsn] 0 for supernodes without children
  std::vector<int64_t> st_off;      // [nsn + 1]
  std::vector<int> st_ids;          // structure rows
  std::vector<int> st_pos;          // position of each structure row in the parent's front
  std::vector<int> ch_off, ch_ids;  // children of each supernode
  std::vector<int> lvl_off, lvl_sn; // supernodes grouped by height
  std::vector<int> lvl_front;       // largest ns + nst of each level
  std::vector<int64_t> l11_off;     // [nsn + 1] ns^2 values each
  std::vector<int64_t> l21_off;     // [nsn + 1] ns * nst values each
  int max_front = 0;                // largest ns + nst
};

// nd_mode: 0 nested dissection only for conductors whose reverse
// Cuthill-McKee band would be wider than the band solvers take (then for all
// of them), 1 nested dissection always.
void build_precond_struct(const HostModel &m, PrecondStruct &ps, int nd_mode = 0);
// Supernodal (multifrontal) LDL^T of L_w on a nested-dissection structure for
// one frequency: l11 [ps.l11_off[nsn]] unit-lower pivot blocks stored by
// columns (entry (i, k) of supernode s at l11_off[s] + k ns + i), l11t the
// same blocks stored by rows, l21 [ps.l21_off[nsn]] the rows below them by
// columns (entry (t, k) at l21_off[s] + k nst + t), diag [nu], yinv [b].
// Returns false on a zero pivot.
bool factor_precond_nd(const HostModel &m, const PrecondStruct &ps, double omega, double sigma, double mu_r,
                       std::vector<std::complex<double>> &l11, std::vector<std::complex<double>> &l11t,
                       std::vector<std::complex<double>> &l21, std::vector<std::complex<double>> &diag,
                       std::vector<std::complex<double>> &yinv);

// Factor for one angular frequency: envelope values (unit lower L), diagonal
// and the branch admittances 1/D_e.  Returns false on a zero pivot.
// The solve kernel reads L in two padded layouts (no per-row offsets):
//   rowpad[i][t] = L(i, i-1-t) for t < pr  (zero outside row i's envelope)
//   colpad[j][t] = L(j+1+t, j) for t < pc  (zero outside column j's profile)
bool factor_precond(const HostModel &m, const PrecondStruct &ps, double omega, double sigma, double mu_r,
                    std::vector<std::complex<double>> &rowpad, std::vector<std::complex<double>> &diag,
                    std::vector<std::complex<double>> &yinv, std::vector<std::complex<double>> &colpad,
                    std::vector<std::complex<double>> &full);

// Device factorization: the same factor, in the same layouts, as
// factor_precond, for nf frequencies at once (one workgroup per conductor and
// frequency, right-looking over the band with the active (W+1) x (W+1)
// window in LDS).  The branch
// admittances 1/D_e are formed on the device from the Gram and kernel
// diagonals.  FACT_NS bounds the supernode rows of a conductor.
constexpr int FACT_NS = 4;
struct FactorArgs {
  int nu, b, W, Wc, ncomp, nf;       // W, Wc: max(W, 1), max(Wc, 1)
  int pr, pc;                        // layout pitches
  const int *comp_off, *comp_mid, *first, *inc_off, *inc_br, *br_ru, *br_rv;
  const int64_t *env_off;
  int64_t nnz_full;
  const double *gdiag, *kdiag;       // [b] Gram and kernel diagonals
  const double *omega;               // [nf] rad/s (device)
  double sigma, mu_r;
  double2 *env, *colenv, *full, *diag, *yinv;
  int *status;                       // [nf * ncomp + nf]: nonzero on a zero pivot / impedance
};
// Whether the device factorization applies: every conductor carries at most
// FACT_NS supernode rows and the band window fits in LDS (W up to about 85).
bool factor_device_ok(const PrecondStruct &ps);
void factor_precond_device(const FactorArgs &a, hipStream_t st);

struct PrecondDev {
  int nu, ncomp, W, Wc, b, l, p, nf;
  int pr, pc;            // pitches of the padded row / column layouts
  const int *comp_off, *comp_mid, *first, *clast;
  int64_t nnz_full;
  const double2 *full;   // [nf][env_off[nu]] row envelopes (used for supernode rows)
  const int64_t *env_off, *col_off;
  int64_t nnz_col;       // nu * Wc
  const double2 *colenv; // [nf][nu][pc] padded columns
  const double2 *env;    // [nf][nu][pr] padded rows
  const double2 *diag;   // [nf][nu]
  const double2 *yinv;   // [nf][b]
  const int *br_ru, *br_rv, *br_link, *br_offu, *br_offv;
  const int *inc_off, *inc_br;
  const int8_t *inc_sg;
  const int *src_off, *src_br;
  const int8_t *src_sg;
  const int *link_kind, *port_loop;
  int64_t nnz_env;
  int ldl_plan;          // 0 register window when W, Wc <= 63; 1 LDS window
  // nested-dissection solve (nd = 1): supernode structure as in
  // PrecondStruct, factors per frequency ([nf][nl11], [nf][nl21]), and the
  // forward sweep's update vectors [R][st_off[nsn]]
  int nd, nsn, nlvl, max_front;
  const int *sn_start, *st_ids, *st_pos, *ch_off, *ch_ids, *lvl_off, *lvl_sn;
  const int64_t *st_off, *l11_off, *l21_off;
  int64_t nl11, nl21, nst_tot;
  const double2 *l11, *l11t, *l21;
  double2 *uvec;
  const int *lvl_off_host;     // lvl_off in host memory (the launch loop)
  const int *lvl_front_host;   // largest front of each level, host
};

// z = P^-1 y for R right-hand sides; fidx[r] selects the factor of RHS r
// (device array).  work: [R][nu] complex128 scratch.
void precond_apply(const PrecondDev &d, const int *fidx, const double2 *y, double2 *z, double2 *work, int R,
                   hipStream_t st);

// Preconditioner state of a context: structure (built once), factors of the
// distinct frequencies of the current batch, per-RHS factor index.
struct Precond {
  PrecondStruct ps;
  bool built = false;
  PrecondDev dev{};
  std::vector<void *> allocs;
  std::vector<double> omegas;            // factored frequencies (rad/s)
  std::vector<int> fidx_host;            // factor index per RHS, as on the device
  int cap_f = 0, cap_R = 0;
  double2 *d_env = nullptr, *d_diag = nullptr, *d_yinv = nullptr, *d_work = nullptr, *d_tmp = nullptr,
          *d_colenv = nullptr, *d_full = nullptr;
  int *d_fidx = nullptr;
  // device factorization inputs and scratch
  double *d_gdiag = nullptr, *d_kdiag = nullptr, *d_om = nullptr;
  int *d_status = nullptr;
  int factor_plan = -1;                  // plan the current factors were made with
  int nd_mode = 0;                       // nd_mode the structure was built with
  // nested-dissection factors and the forward sweep's update vectors
  double2 *d_l11 = nullptr, *d_l11t = nullptr, *d_l21 = nullptr, *d_uvec = nullptr;
};

}  // namespace pfft

struct pfft_ctx;

namespace pfft {
// Builds the structure once, factors every distinct frequency of omega[0..R)
// (host, rad/s) and uploads the per-RHS factor index; returns the context's
// preconditioner.
Precond *precond_prepare(pfft_ctx *c, int R, const double *omega, hipStream_t st);

}  // namespace pfft

