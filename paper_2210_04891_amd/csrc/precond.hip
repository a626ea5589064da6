// Preconditioner of Eq. Precond through the node space (see precond.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <deque>
#include <numeric>
#include <string>

#include "precond.h"
#include "xcd.h"

namespace pfft {

void hip_ok(hipError_t e, const char *what);   // throws DeviceError

typedef std::complex<double> cd;
static constexpr double MU0 = 4e-7 * M_PI;

// ---------------------------------------------------------------------------
// structure: supernodes, grounds, reverse Cuthill-McKee order, envelope
// ---------------------------------------------------------------------------
void nd_order_conductor(const std::vector<std::vector<int>> &adj, const std::vector<double> &xyz,
                        const std::vector<int> &mem, const std::vector<int> &dmem, std::vector<int> &stamp,
                        int &next, std::vector<int> &unk, PrecondStruct &ps);
void nd_symbolic(const std::vector<std::vector<int>> &uadj, PrecondStruct &ps);

// widest band row above which a conductor is ordered by nested dissection
static constexpr int ND_BAND_MAX = 256;

void build_precond_struct(const HostModel &m, PrecondStruct &ps, int nd_mode) {
  const int nn = m.nn, b = m.b, p = m.p;
  // ports: sink node merged into source node, phi_K = phi_S - s_k
  std::vector<int> rep(nn), off_port(nn, -1), role(nn, 0);
  std::iota(rep.begin(), rep.end(), 0);
  for (int k = 0; k < p; ++k) {
    int K = m.bu[b + k], S = m.bv[b + k];
    if (++role[K] > 1 || ++role[S] > 1)
      throw SetupError{-1, "preconditioner: a contact face serves more than one port"};
    if (K == S) throw SetupError{-1, "preconditioner: port source and sink faces coincide"};
    rep[K] = S;
    off_port[K] = k;
  }
  // conductor components over mesh branches
  std::vector<int> comp(nn, -1);
  {
    std::vector<std::vector<int>> adj(nn);
    for (int e = 0; e < b; ++e)
      if (m.bu[e] != m.bv[e]) {
        adj[m.bu[e]].push_back(m.bv[e]);
        adj[m.bv[e]].push_back(m.bu[e]);
      }
    int nc = 0;
    for (int r = 0; r < nn; ++r) {
      if (comp[r] >= 0) continue;
      std::deque<int> dq{r};
      comp[r] = nc;
      while (!dq.empty()) {
        int x = dq.front();
        dq.pop_front();
        for (int y : adj[x])
          if (comp[y] < 0) { comp[y] = nc; dq.push_back(y); }
      }
      ++nc;
    }
    ps.ncomp = nc;
  }
  // merged-node adjacency (mesh branches whose ends are different supernodes)
  std::vector<std::vector<int>> madj(nn);
  for (int e = 0; e < b; ++e) {
    int a = rep[m.bu[e]], c = rep[m.bv[e]];
    if (a != c) { madj[a].push_back(c); madj[c].push_back(a); }
  }
  for (auto &v : madj) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  }
  // ground: lowest merged node of each conductor
  std::vector<int> ground(ps.ncomp, -1);
  for (int x = 0; x < nn; ++x)
    if (rep[x] == x && ground[comp[x]] < 0) ground[comp[x]] = x;
  // RCM per conductor
  std::vector<int> unk(nn, -1);
  ps.comp_off.assign(ps.ncomp + 1, 0);
  int next = 0;
  // supernodes (a port's source node with its sink merged in) tie the two
  // ends of a conductor together; they are ordered after the band
  std::vector<uint8_t> dense(nn, 0);
  for (int k = 0; k < p; ++k) dense[m.bv[b + k]] = 1;
  std::vector<std::vector<int>> members(ps.ncomp), dmembers(ps.ncomp);
  for (int x = 0; x < nn; ++x)
    if (rep[x] == x && x != ground[comp[x]]) (dense[x] ? dmembers : members)[comp[x]].push_back(x);
  ps.comp_mid.assign(ps.ncomp, 0);
  std::vector<int> mark(nn, -1), dist(nn, -1);
  auto deg = [&](int x) {
    int d = 0;
    for (int y : madj[x]) d += (y != ground[comp[x]] && !dense[y]);
    return d;
  };
  for (int c = 0; c < ps.ncomp; ++c) {
    ps.comp_off[c] = next;
    auto &mem = members[c];
    if (mem.empty()) {
      ps.comp_mid[c] = next;
      for (int x : dmembers[c]) unk[x] = next++;
      continue;
    }
    int gnd = ground[c];
    auto bfs = [&](int start, std::vector<int> &ord) {
      ord.clear();
      ord.push_back(start);
      mark[start] = start * 2 + c;  // unique stamp per call
      size_t h = 0;
      while (h < ord.size()) {
        int x = ord[h++];
        std::vector<int> nb;
        for (int y : madj[x])
          if (y != gnd && !dense[y] && mark[y] != start * 2 + c) nb.push_back(y);
        std::sort(nb.begin(), nb.end(), [&](int a, int bq) {
          int da = deg(a), db = deg(bq);
          return da != db ? da < db : a < bq;
        });
        for (int y : nb)
          if (mark[y] != start * 2 + c) { mark[y] = start * 2 + c; ord.push_back(y); }
      }
    };
    // pseudo-peripheral start: min degree, then the last node of two BFS sweeps
    int s0 = mem[0];
    for (int x : mem)
      if (deg(x) < deg(s0)) s0 = x;
    std::vector<int> ord;
    for (int it = 0; it < 2; ++it) {
      bfs(s0, ord);
      for (int x : mem) mark[x] = -1;
      s0 = ord.back();
    }
    bfs(s0, ord);
    for (int x : mem) mark[x] = -1;
    // unreachable members (a conductor split only by a grounded node) follow
    std::vector<int> seen(ord.begin(), ord.end());
    std::sort(seen.begin(), seen.end());
    for (int x : mem)
      if (!std::binary_search(seen.begin(), seen.end(), x)) ord.push_back(x);
    std::reverse(ord.begin(), ord.end());
    for (int x : ord) unk[x] = next++;
    ps.comp_mid[c] = next;
    for (int x : dmembers[c]) unk[x] = next++;
  }
  ps.comp_off[ps.ncomp] = next;
  ps.nu = next;
  const int nu = ps.nu;
  // the band's widest row: nested dissection instead when it is too wide
  // (or always, nd_mode 1)
  int wband = 0;
  for (int x = 0; x < nn; ++x) {
    if (unk[x] < 0 || dense[x]) continue;
    for (int y : madj[x])
      if (unk[y] >= 0 && !dense[y]) wband = std::max(wband, std::abs(unk[x] - unk[y]));
  }
  ps.nd = nd_mode == 1 || wband > ND_BAND_MAX;
  if (ps.nd) {
    // node coordinates: mean centroid of a node's triangles
    std::vector<double> xyz(3 * (size_t)nn, 0.0);
    std::vector<int> cnt(nn, 0);
    for (int t = 0; t < m.n; ++t) {
      const int x = rep[m.node_of_tri[t]];
      for (int d = 0; d < 3; ++d) xyz[3 * x + d] += m.cen[3 * t + d];
      cnt[x]++;
    }
    for (int x = 0; x < nn; ++x)
      if (cnt[x])
        for (int d = 0; d < 3; ++d) xyz[3 * x + d] /= cnt[x];
    // band-member adjacency without ground and port supernodes
    std::vector<std::vector<int>> badj(nn);
    for (int x = 0; x < nn; ++x) {
      if (rep[x] != x || dense[x] || x == ground[comp[x]]) continue;
      for (int y : madj[x])
        if (y != ground[comp[y]] && !dense[y]) badj[x].push_back(y);
    }
    std::fill(unk.begin(), unk.end(), -1);
    next = 0;
    ps.nsn = 0;
    ps.sn_start.clear();
    ps.sn_parent.clear();
    std::vector<int> stamp(nn, 0);
    for (int c = 0; c < ps.ncomp; ++c) {
      ps.comp_off[c] = next;
      nd_order_conductor(badj, xyz, members[c], dmembers[c], stamp, next, unk, ps);
      ps.comp_mid[c] = ps.comp_off[c];
    }
    ps.comp_off[ps.ncomp] = next;
    if (next != nu) throw SetupError{-4, "internal: nested dissection lost unknowns"};
    std::vector<std::vector<int>> uadj(nu);
    for (int x = 0; x < nn; ++x) {
      if (unk[x] < 0) continue;
      for (int y : madj[x])
        if (unk[y] >= 0) uadj[unk[x]].push_back(unk[y]);
    }
    nd_symbolic(uadj, ps);
    // no band structure
    ps.first.resize(nu);
    std::iota(ps.first.begin(), ps.first.end(), 0);
    ps.env_off.assign(nu + 1, 0);
    ps.clast = ps.first;
    ps.col_off.assign(nu + 1, 0);
    ps.W = ps.Wc = 0;
    ps.pr = ps.pc = 1;
  }
  // envelope
  if (!ps.nd) {
  ps.first.assign(nu, 0);
  for (int x = 0; x < nn; ++x) {
    if (unk[x] < 0) continue;
    int i = unk[x], f = i;
    for (int y : madj[x])
      if (unk[y] >= 0) f = std::min(f, unk[y]);
    ps.first[i] = f;
  }
  std::vector<uint8_t> band(nu, 1);
  for (int c = 0; c < ps.ncomp; ++c)
    for (int i = ps.comp_mid[c]; i < ps.comp_off[c + 1]; ++i) band[i] = 0;
  ps.env_off.assign(nu + 1, 0);
  ps.W = 0;
  for (int i = 0; i < nu; ++i) {
    ps.env_off[i + 1] = ps.env_off[i] + (i - ps.first[i]);
    if (band[i]) ps.W = std::max(ps.W, i - ps.first[i]);
  }
  // column profile over band rows only (supernode rows are handled apart)
  ps.clast.resize(nu);
  for (int j = 0; j < nu; ++j) ps.clast[j] = j;
  for (int i = 0; i < nu; ++i)
    if (band[i])
      for (int j = ps.first[i]; j < i; ++j) ps.clast[j] = std::max(ps.clast[j], i);
  ps.col_off.assign(nu + 1, 0);
  ps.Wc = 0;
  for (int j = 0; j < nu; ++j) {
    ps.col_off[j + 1] = ps.col_off[j] + (ps.clast[j] - j);
    ps.Wc = std::max(ps.Wc, ps.clast[j] - j);
  }
  if (ps.W <= 63 && ps.Wc <= 63) {
    ps.pr = ps.pc = 64;
  } else {
    ps.pr = std::max(ps.W, 1);
    ps.pc = std::max(ps.Wc, 1);
  }
  }
  // branches
  ps.br_ru.resize(b);
  ps.br_rv.resize(b);
  ps.br_link.assign(b, -1);
  ps.br_offu.resize(b);
  ps.br_offv.resize(b);
  for (int i = 0; i < m.l; ++i)
    if (m.links[i] < b) ps.br_link[m.links[i]] = i;
  std::vector<int> cnt(nu + 1, 0);
  for (int e = 0; e < b; ++e) {
    int a = rep[m.bu[e]], c = rep[m.bv[e]];
    ps.br_ru[e] = unk[a];
    ps.br_rv[e] = unk[c];
    ps.br_offu[e] = off_port[m.bu[e]];
    ps.br_offv[e] = off_port[m.bv[e]];
    if (a != c) {
      if (unk[a] >= 0) cnt[unk[a] + 1]++;
      if (unk[c] >= 0) cnt[unk[c] + 1]++;
    }
  }
  for (int i = 0; i < nu; ++i) cnt[i + 1] += cnt[i];
  ps.inc_off = cnt;
  ps.inc_br.resize(cnt[nu]);
  ps.inc_sg.resize(cnt[nu]);
  {
    std::vector<int> f(cnt.begin(), cnt.end() - 1);
    for (int e = 0; e < b; ++e) {
      int a = rep[m.bu[e]], c = rep[m.bv[e]];
      if (a == c) continue;
      if (unk[a] >= 0) { ps.inc_br[f[unk[a]]] = e; ps.inc_sg[f[unk[a]]++] = 1; }
      if (unk[c] >= 0) { ps.inc_br[f[unk[c]]] = e; ps.inc_sg[f[unk[c]]++] = -1; }
    }
  }
  // source nodes: incident mesh branches (unmerged)
  ps.src_off.assign(p + 1, 0);
  ps.src_br.clear();
  ps.src_sg.clear();
  for (int k = 0; k < p; ++k) {
    int S = m.bv[b + k];
    for (int e = 0; e < b; ++e) {
      if (m.bu[e] == m.bv[e]) continue;
      if (m.bu[e] == S) { ps.src_br.push_back(e); ps.src_sg.push_back(1); }
      else if (m.bv[e] == S) { ps.src_br.push_back(e); ps.src_sg.push_back(-1); }
    }
    ps.src_off[k + 1] = (int)ps.src_br.size();
  }
  ps.link_kind.resize(m.l);
  for (int i = 0; i < m.l; ++i) ps.link_kind[i] = m.links[i] < b ? m.links[i] : -(m.links[i] - b + 1);
  ps.port_loop = m.port_loop;
}

bool factor_precond(const HostModel &m, const PrecondStruct &ps, double omega, double sigma, double mu_r,
                    std::vector<cd> &rowpad, std::vector<cd> &diag, std::vector<cd> &yinv, std::vector<cd> &colpad,
                    std::vector<cd> &env) {
  const int b = m.b, nu = ps.nu;
  double a = std::sqrt(omega * MU0 * mu_r / (2.0 * sigma));
  cd zs(a, a), jw(0.0, omega * MU0 * mu_r / (4.0 * M_PI));
  yinv.assign(b, 0.0);
  for (int e = 0; e < b; ++e) {
    double g = 0;
    for (int q = 0; q < 5; ++q)
      if (m.gram_col[5 * e + q] == e) g += m.gram_val[5 * e + q];
    cd D = zs * g + jw * m.kdiag[e];
    if (std::abs(D) == 0.0) return false;
    yinv[e] = 1.0 / D;
  }
  env.assign(ps.env_off[nu], 0.0);
  diag.assign(nu, 0.0);
  for (int e = 0; e < b; ++e) {
    int ru = ps.br_ru[e], rv = ps.br_rv[e];
    bool self = (ru == rv) && ru >= 0;
    if (self) continue;
    // a branch whose two ends are the same supernode (ground included) does
    // not enter the nodal matrix
    if (ru < 0 && rv < 0) continue;
    cd y = yinv[e];
    if (ru >= 0) diag[ru] += y;
    if (rv >= 0) diag[rv] += y;
    if (ru >= 0 && rv >= 0) {
      int i = std::max(ru, rv), j = std::min(ru, rv);
      env[ps.env_off[i] + (j - ps.first[i])] -= y;
    }
  }
  // envelope LDL^T, row by row: w_k = L_ik D_k (supernode rows are the widest)
  int wmax = 1;
  for (int i = 0; i < nu; ++i) wmax = std::max(wmax, i - ps.first[i] + 1);
  std::vector<cd> w(wmax);
  for (int i = 0; i < nu; ++i) {
    int fi = ps.first[i];
    cd *Li = &env[ps.env_off[i]];
    for (int j = fi; j < i; ++j) {
      int fj = ps.first[j];
      const cd *Lj = &env[ps.env_off[j]];
      cd u = Li[j - fi];
      for (int k = std::max(fi, fj); k < j; ++k) u -= w[k - fi] * Lj[k - fj];
      w[j - fi] = u;
      Li[j - fi] = u / diag[j];
    }
    cd d = diag[i];
    for (int k = fi; k < i; ++k) d -= w[k - fi] * Li[k - fi];
    if (std::abs(d) == 0.0 || !std::isfinite(d.real()) || !std::isfinite(d.imag())) return false;
    diag[i] = d;
  }
  const int W = std::max(ps.W, 1), pr = ps.pr, pc = ps.pc;
  rowpad.assign((size_t)nu * pr, 0.0);
  colpad.assign((size_t)nu * pc, 0.0);
  for (int i = 0; i < nu; ++i) {
    if (i - ps.first[i] > W) continue;             // supernode row: kept in env only
    if (ps.clast[i] < i) continue;
    bool is_band = true;
    for (int c = 0; c < ps.ncomp; ++c)
      if (i >= ps.comp_mid[c] && i < ps.comp_off[c + 1]) is_band = false;
    if (!is_band) continue;
    for (int j = ps.first[i]; j < i; ++j) {
      cd v = env[ps.env_off[i] + (j - ps.first[i])];
      rowpad[(size_t)i * pr + (i - 1 - j)] = v;
      colpad[(size_t)j * pc + (i - j - 1)] = v;
    }
  }
  return true;
}

// ---------------------------------------------------------------------------
// device side
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cmul2(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cdiv2(double2 a, double2 b) {
  double den = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}

// known part of branch e's current: (off_u - off_v + s_e) / D_e
__device__ __forceinline__ double2 branch_known(const PrecondDev &d, const double2 *y, const double2 *yinv,
                                                int e) {
  double2 s = make_double2(0, 0);
  int lk = d.br_link[e];
  if (lk >= 0) s = y[lk];
  int ou = d.br_offu[e], ov = d.br_offv[e];
  if (ou >= 0) { double2 v = y[d.port_loop[ou]]; s.x -= v.x; s.y -= v.y; }
  if (ov >= 0) { double2 v = y[d.port_loop[ov]]; s.x += v.x; s.y += v.y; }
  return cmul2(s, yinv[e]);
}

__global__ void k_pre_rhs(PrecondDev d, const int *fidx, const double2 *y, double2 *work) {
  int r = blockIdx.y;
  int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= d.nu) return;
  const double2 *yr = y + (size_t)r * d.l;
  const double2 *yinv = d.yinv + (size_t)fidx[r] * d.b;
  double gx = 0, gy = 0;
  for (int q = d.inc_off[x]; q < d.inc_off[x + 1]; ++q) {
    double2 c = branch_known(d, yr, yinv, d.inc_br[q]);
    double sg = d.inc_sg[q];
    gx += sg * c.x;
    gy += sg * c.y;
  }
  work[(size_t)r * d.nu + x] = make_double2(-gx, -gy);
}

// Orders a wavefront's global stores of the solution vector before its later
// loads of it.  Every solve workgroup is one wavefront and the only one that
// touches its (conductor, right-hand side) slice, so workgroup scope is
// enough; a device-scope fence would write back and invalidate the L2 of the
// XCD each time.
__device__ __forceinline__ void slice_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }

__device__ __forceinline__ double2 wave_sum(double2 v) {
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

// One wavefront per (conductor, RHS).  Band rows [lo, mid): unit-lower
// forward solve column by column (y_i = acc_i, then acc_k -= L_ki y_i) and
// transposed backward solve row by row (x_i final, then z_j -= L_ij x_i),
// both as scatters into a circular LDS window of WP entries, so the
// row-to-row chain holds no reductions; L is read in padded layouts, PF rows
// per block, the next block's values fetched while the current one is
// solved.  Supernode rows [mid, hi) come last: forward as dot products over
// their full rows, backward as scatters over their full rows.
constexpr int PF = 16;

// The solve runs as one wavefront, whose LDS operations complete in program
// order; this fence keeps the compiler from reordering LDS accesses across
// rows without waiting on outstanding global stores (which a workgroup
// barrier would).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef decltype(__builtin_amdgcn_raw_buffer_load_b128(__amdgpu_buffer_rsrc_t(), 0, 0, 0)) b128_t;

// Band factor rows are read with buffer loads (per-lane VGPR offset, uniform
// SGPR row offset): they count only against vmcnt, so waiting on the LDS
// window never waits on the prefetch of the next rows (flat loads would), and
// the hardware returns zero beyond the factor's size.
__device__ __forceinline__ double2 band_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

// Between the two band sweeps (one wavefront): forward over the supernode
// rows, y_s = b_s - sum_j L_sj y_j over each full row; z = y / D; then the
// transposed scatter of the supernode rows, last row first.  Each lane loads
// SB entries before using any, so that several loads are in flight.
constexpr int SB = 8;
__device__ void ldl_middle(const PrecondDev &d, int f, double2 *x, int lo, int mid, int hi, int lane) {
  const double2 *full = d.full + (size_t)f * d.nnz_full;
  const double2 *dg = d.diag + (size_t)f * d.nu;
  const double2 zero = make_double2(0, 0);
  for (int s = mid; s < hi; ++s) {
    const int fs = d.first[s];
    const double2 *Ls = full + d.env_off[s];
    double2 acc = zero;
    for (int j0 = fs; j0 < s; j0 += 64 * SB) {
      double2 lv[SB], yv[SB];
#pragma unroll
      for (int q = 0; q < SB; ++q) {
        const int j = j0 + q * 64 + lane;
        lv[q] = j < s ? Ls[j - fs] : zero;
        yv[q] = j < s ? x[j] : zero;
      }
#pragma unroll
      for (int q = 0; q < SB; ++q) {
        acc.x += lv[q].x * yv[q].x - lv[q].y * yv[q].y;
        acc.y += lv[q].x * yv[q].y + lv[q].y * yv[q].x;
      }
    }
    acc = wave_sum(acc);
    if (lane == 0) {
      const double2 bs = x[s];
      x[s] = make_double2(bs.x - acc.x, bs.y - acc.y);
    }
    slice_fence();
    __syncthreads();
  }
  for (int i0 = lo; i0 < hi; i0 += 64 * SB) {
    double2 xv[SB], dv[SB];
#pragma unroll
    for (int q = 0; q < SB; ++q) {
      const int i = i0 + q * 64 + lane;
      xv[q] = i < hi ? x[i] : zero;
      dv[q] = i < hi ? dg[i] : make_double2(1, 0);
    }
#pragma unroll
    for (int q = 0; q < SB; ++q) {
      const int i = i0 + q * 64 + lane;
      if (i < hi) x[i] = cdiv2(xv[q], dv[q]);
    }
  }
  slice_fence();
  __syncthreads();
  for (int s = hi - 1; s >= mid; --s) {
    const int fs = d.first[s];
    const double2 *Ls = full + d.env_off[s];
    const double2 xs = x[s];
    for (int j0 = fs; j0 < s; j0 += 64 * SB) {
      double2 lv[SB], t[SB];
#pragma unroll
      for (int q = 0; q < SB; ++q) {
        const int j = j0 + q * 64 + lane;
        lv[q] = j < s ? Ls[j - fs] : zero;
        t[q] = j < s ? x[j] : zero;
      }
#pragma unroll
      for (int q = 0; q < SB; ++q) {
        const int j = j0 + q * 64 + lane;
        if (j < s) {
          t[q].x -= lv[q].x * xs.x - lv[q].y * xs.y;
          t[q].y -= lv[q].x * xs.y + lv[q].y * xs.x;
          x[j] = t[q];
        }
      }
    }
    slice_fence();
    __syncthreads();
  }
}

template <int WP>
__global__ void __launch_bounds__(64) k_ldl_solve(PrecondDev d, const int *fidx, double2 *work, int R) {
  __shared__ double2 win[WP];
  const int lb = (int)xcd_block(blockIdx.x, gridDim.x), c = lb / R, r = lb - c * R, lane = threadIdx.x;
  const int lo = d.comp_off[c], hi = d.comp_off[c + 1], mid = d.comp_mid[c];
  if (lo >= hi) return;
  const int f = fidx[r];
  const int W = max(d.W, 1), Wc = max(d.Wc, 1), pr = d.pr, pc = d.pc;
  const double2 *rowp = d.env + (size_t)f * d.nu * pr;
  const double2 *colp = d.colenv + (size_t)f * d.nu * pc;
  double2 *x = work + (size_t)r * d.nu;
  const double2 zero = make_double2(0, 0);
  const unsigned row_bytes = (unsigned)d.nu * (unsigned)pr * 16u, col_bytes = (unsigned)d.nu * (unsigned)pc * 16u;
  const __amdgpu_buffer_rsrc_t rrow = __builtin_amdgcn_make_buffer_rsrc((void *)rowp, (short)0, (int)row_bytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t rcol = __builtin_amdgcn_make_buffer_rsrc((void *)colp, (short)0, (int)col_bytes, 0x00020000);
  const unsigned lane16 = (unsigned)lane * 16u;
  double2 cur[PF], nxt[PF];
  // ---- forward, band rows
  if (lo < mid) {
    int loaded_hi = lo;
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const double2 v = band_load(rcol, lane16, (unsigned)(lo + q) * (unsigned)pc * 16u);
      cur[q] = (lo + q < mid && lane < Wc) ? v : zero;
    }
    for (int i0 = lo; i0 < mid; i0 += PF) {
      const int nb = min(PF, mid - i0);
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int i = i0 + PF + q;
        const double2 v = band_load(rcol, lane16, (unsigned)i * (unsigned)pc * 16u);
        nxt[q] = (i < mid && lane < Wc) ? v : zero;
      }
      const int need = min(mid, i0 + nb + Wc);
      while (loaded_hi < need) {
        const int cnt = min(64, need - loaded_hi);
        if (lane < cnt) win[(loaded_hi + lane) & (WP - 1)] = x[loaded_hi + lane];
        loaded_hi += cnt;
      }
      wave_sync();
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        if (q < nb) {
        const int i = i0 + q;
        const double2 yi = win[i & (WP - 1)];
        if (lane == 0) x[i] = yi;
        if (lane < Wc && i + 1 + lane < mid) {
          double2 &t = win[(i + 1 + lane) & (WP - 1)];
          t.x -= cur[q].x * yi.x - cur[q].y * yi.y;
          t.y -= cur[q].x * yi.y + cur[q].y * yi.x;
        }
        for (int t2 = 64 + lane; t2 < Wc && i + 1 + t2 < mid; t2 += 64) {   // columns taller than 64
          double2 l2 = colp[(size_t)i * pc + t2];
          double2 &t = win[(i + 1 + t2) & (WP - 1)];
          t.x -= l2.x * yi.x - l2.y * yi.y;
          t.y -= l2.x * yi.y + l2.y * yi.x;
        }
        wave_sync();
        }
      }
#pragma unroll
      for (int q = 0; q < PF; ++q) cur[q] = nxt[q];
    }
  }
  slice_fence();
  __syncthreads();
  ldl_middle(d, f, x, lo, mid, hi, lane);
  // ---- backward, band rows
  if (lo < mid) {
    int loaded = mid;  // window holds z_j for j in [loaded, mid)
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int i = mid - 1 - q;
      const double2 v = band_load(rrow, lane16, (unsigned)max(i, 0) * (unsigned)pr * 16u);
      cur[q] = (i >= lo && lane < W) ? v : zero;
    }
    for (int i0 = mid - 1; i0 >= lo; i0 -= PF) {
      const int nb = min(PF, i0 - lo + 1);
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int i = i0 - PF - q;
        const double2 v = band_load(rrow, lane16, (unsigned)max(i, 0) * (unsigned)pr * 16u);
        nxt[q] = (i >= lo && lane < W) ? v : zero;
      }
      const int target = max(lo, i0 - (nb - 1) - W);
      while (loaded > target) {
        const int cnt = min(64, loaded - target);
        const int j = loaded - 1 - lane;
        if (lane < cnt) win[j & (WP - 1)] = x[j];
        loaded -= cnt;
      }
      wave_sync();
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        if (q < nb) {
        const int i = i0 - q;
        const double2 xi = win[i & (WP - 1)];
        if (lane == 0) x[i] = xi;
        if (lane < W && i - 1 - lane >= lo) {
          double2 &t = win[(i - 1 - lane) & (WP - 1)];
          t.x -= cur[q].x * xi.x - cur[q].y * xi.y;
          t.y -= cur[q].x * xi.y + cur[q].y * xi.x;
        }
        for (int t2 = 64 + lane; t2 < W && i - 1 - t2 >= lo; t2 += 64) {
          double2 l2 = rowp[(size_t)i * pr + t2];
          double2 &t = win[(i - 1 - t2) & (WP - 1)];
          t.x -= l2.x * xi.x - l2.y * xi.y;
          t.y -= l2.x * xi.y + l2.y * xi.x;
        }
        wave_sync();
        }
      }
#pragma unroll
      for (int q = 0; q < PF; ++q) cur[q] = nxt[q];
    }
  }
}

// Register-window variant (band widths W, Wc <= 63, factor layouts padded to
// 64 entries).  The pending partial sums of the band substitution live one
// per lane in a circular window: lane l holds the row whose position
// (forward: row - lo, backward: mid - 1 - row) is l mod 64.  Step p reads the
// finished value of position p from lane p mod 64 (readlane with a uniform
// lane index), subtracts its product with the factor from every lane (one
// complex FMA; the factor row is loaded rotated by p, so lane l takes the
// entry of its own row and the zero padding masks everything outside the
// band).  Lane p mod 64 itself takes the unit entry kept in the layouts' last
// padding slot, which turns its sum into exactly zero; from there it gathers
// the updates of position p + 64, whose right-hand side is added once per
// block.  No LDS, no barrier, no lane shifts, no per-step selects; solved
// values are collected one per lane (writelane) and stored 64 rows at a time.
// Rows past the band read from beyond the factor buffer, which the buffer
// load returns as zeros.
__device__ __forceinline__ double dbl_lane(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// v_writelane (the compiler intrinsic has no builtin spelling): returns old
// with lane l set to the uniform val
__device__ int amdgcn_writelane(int val, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

// v with lane l replaced by the uniform value u
__device__ __forceinline__ double dbl_put(double v, double u, int l) {
  const long long b = __builtin_bit_cast(long long, v), c = __builtin_bit_cast(long long, u);
  const int lo = amdgcn_writelane((int)(c & 0xffffffffll), l, (int)(b & 0xffffffffll));
  const int hi = amdgcn_writelane((int)(c >> 32), l, (int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

constexpr int RP = 32;   // rows of factor data in flight per buffer

// The forward and backward band sweeps of one conductor for NR right-hand
// sides of the same frequency (x[j] their slices of the work vector): the
// factor rows are loaded once and feed NR independent substitution chains,
// whose instructions the scheduler interleaves.
template <int NR>
__device__ __forceinline__ void band_sweeps(const PrecondDev &d, int f, double2 *const (&x)[NR], int lo, int mid,
                                            int hi, int lane) {
  const double2 *rowp = d.env + (size_t)f * d.nu * 64;
  const double2 *colp = d.colenv + (size_t)f * d.nu * 64;
  const double2 zero = make_double2(0, 0);
  const unsigned bytes = (unsigned)d.nu * 1024u;
  const __amdgpu_buffer_rsrc_t rrow = __builtin_amdgcn_make_buffer_rsrc((void *)rowp, (short)0, (int)bytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t rcol = __builtin_amdgcn_make_buffer_rsrc((void *)colp, (short)0, (int)bytes, 0x00020000);
  const int nb = mid - lo;
  // ---- forward, band rows: y = L^-1 b, column by column
  if (nb > 0) {
    double ax[NR], ay[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      const double2 v = lane < nb ? x[j][lo + lane] : zero;
      ax[j] = v.x;
      ay[j] = v.y;
    }
    // right-hand side entering at step p (lane p mod 64) for the RP steps of
    // the block starting at p0: position p + 64
    auto bload = [&](int j, int p0) -> double2 {
      const int pl = (lane - p0) & 63, row = lo + p0 + pl + 64;
      return (pl < RP && row < mid) ? x[j][row] : zero;
    };
    double2 Lc[RP], Ln[RP], bc[NR], bn[NR];
#pragma unroll
    for (int q = 0; q < RP; ++q)
      Lc[q] = band_load(rcol, (unsigned)((lane - q - 1) & 63) * 16u, q < nb ? (unsigned)(lo + q) * 1024u : bytes);
    double yx[NR], yy[NR], vx[NR], vy[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      bc[j] = bload(j, 0);
      yx[j] = yy[j] = 0;
      // value of the current position, read one step ahead from the updated
      // window (the hand-over of lane p mod 64 does not touch lane p + 1)
      vx[j] = dbl_lane(ax[j], 0);
      vy[j] = dbl_lane(ay[j], 0);
    }
    for (int p0 = 0; p0 < nb; p0 += RP) {
      // positions [p0 - 64, p0) done: store them before this block's prefetch,
      // so no wait on the store drains the prefetch (vmcnt is in order)
      if (p0 > 0 && (p0 & 63) == 0)
#pragma unroll
        for (int j = 0; j < NR; ++j) x[j][lo + p0 - 64 + lane] = make_double2(yx[j], yy[j]);
#pragma unroll
      for (int q = 0; q < RP; ++q) {
        const int p = p0 + RP + q;
        Ln[q] = band_load(rcol, (unsigned)((lane - p - 1) & 63) * 16u, p < nb ? (unsigned)(lo + p) * 1024u : bytes);
      }
#pragma unroll
      for (int j = 0; j < NR; ++j) bn[j] = bload(j, p0 + RP);
      __builtin_amdgcn_sched_barrier(0);
      const int sb = p0 & 63;
#pragma unroll
      for (int q = 0; q < RP; ++q) {
        const int s = sb + q;
        const double2 L = Lc[q];   // lane s: the unit self entry, so its sum becomes exactly 0
#pragma unroll
        for (int j = 0; j < NR; ++j) {
          double fx = fma(-L.x, vx[j], ax[j]), fy = fma(-L.x, vy[j], ay[j]);
          fx = fma(L.y, vy[j], fx);
          fy = fma(-L.y, vx[j], fy);
          yx[j] = dbl_put(yx[j], vx[j], s);   // (vx, vy): the finished value of position s
          yy[j] = dbl_put(yy[j], vy[j], s);
          vx[j] = dbl_lane(fx, (s + 1) & 63);
          vy[j] = dbl_lane(fy, (s + 1) & 63);
          ax[j] = fx;
          ay[j] = fy;
        }
      }
      // the lanes finished in this block start position p + 64: their sums
      // so far are the updates it already received, to which its right-hand
      // side is added (bc is zero in every other lane)
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        ax[j] += bc[j].x;
        ay[j] += bc[j].y;
        bc[j] = bn[j];
      }
#pragma unroll
      for (int q = 0; q < RP; ++q) Lc[q] = Ln[q];
    }
    {  // the last, partial batch
      const int b0 = (nb - 1) & ~63;
      if (b0 + lane < nb)
#pragma unroll
        for (int j = 0; j < NR; ++j) x[j][lo + b0 + lane] = make_double2(yx[j], yy[j]);
    }
  }
  slice_fence();
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NR; ++j) ldl_middle(d, f, x[j], lo, mid, hi, lane);
  // ---- backward, band rows: x = L^-T z, row by row from the last
  if (nb > 0) {
    double ax[NR], ay[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      const int row = mid - 1 - lane;
      const double2 v = row >= lo ? x[j][row] : zero;
      ax[j] = v.x;
      ay[j] = v.y;
    }
    auto bload = [&](int j, int p0) -> double2 {
      const int pl = (lane - p0) & 63, row = mid - 1 - (p0 + pl + 64);
      return (pl < RP && row >= lo) ? x[j][row] : zero;
    };
    double2 Lc[RP], Ln[RP], bc[NR], bn[NR];
#pragma unroll
    for (int q = 0; q < RP; ++q)
      Lc[q] = band_load(rrow, (unsigned)((lane - q - 1) & 63) * 16u, q < nb ? (unsigned)(mid - 1 - q) * 1024u : bytes);
    double ox[NR], oy[NR], vx[NR], vy[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      bc[j] = bload(j, 0);
      ox[j] = oy[j] = 0;
      vx[j] = dbl_lane(ax[j], 0);
      vy[j] = dbl_lane(ay[j], 0);
    }
    for (int p0 = 0; p0 < nb; p0 += RP) {
      if (p0 > 0 && (p0 & 63) == 0)
#pragma unroll
        for (int j = 0; j < NR; ++j) x[j][mid - 1 - (p0 - 64 + lane)] = make_double2(ox[j], oy[j]);
#pragma unroll
      for (int q = 0; q < RP; ++q) {
        const int p = p0 + RP + q;
        Ln[q] = band_load(rrow, (unsigned)((lane - p - 1) & 63) * 16u, p < nb ? (unsigned)(mid - 1 - p) * 1024u : bytes);
      }
#pragma unroll
      for (int j = 0; j < NR; ++j) bn[j] = bload(j, p0 + RP);
      __builtin_amdgcn_sched_barrier(0);
      const int sb = p0 & 63;
#pragma unroll
      for (int q = 0; q < RP; ++q) {
        const int s = sb + q;
        const double2 L = Lc[q];   // lane s: the unit self entry, so its sum becomes exactly 0
#pragma unroll
        for (int j = 0; j < NR; ++j) {
          double fx = fma(-L.x, vx[j], ax[j]), fy = fma(-L.x, vy[j], ay[j]);
          fx = fma(L.y, vy[j], fx);
          fy = fma(-L.y, vx[j], fy);
          ox[j] = dbl_put(ox[j], vx[j], s);   // (vx, vy): the finished value of position s
          oy[j] = dbl_put(oy[j], vy[j], s);
          vx[j] = dbl_lane(fx, (s + 1) & 63);
          vy[j] = dbl_lane(fy, (s + 1) & 63);
          ax[j] = fx;
          ay[j] = fy;
        }
      }
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        ax[j] += bc[j].x;
        ay[j] += bc[j].y;
        bc[j] = bn[j];
      }
#pragma unroll
      for (int q = 0; q < RP; ++q) Lc[q] = Ln[q];
    }
    {  // the last, partial batch
      const int b0 = (nb - 1) & ~63;
      if (b0 + lane < nb)
#pragma unroll
        for (int j = 0; j < NR; ++j) x[j][mid - 1 - (b0 + lane)] = make_double2(ox[j], oy[j]);
    }
  }
}

// One wavefront per (conductor, right-hand side) or, with NR = 2, per
// (conductor, pair of consecutive right-hand sides): a pair of the same
// frequency shares its factor-row loads; a pair of two frequencies (or a
// last single right-hand side) is solved one after the other.
template <int NR>
__global__ void __launch_bounds__(64) k_ldl_solve_reg(PrecondDev d, const int *fidx, double2 *work, int R) {
  const int ng = (R + NR - 1) / NR;
  const int lb = (int)xcd_block(blockIdx.x, gridDim.x), c = lb / ng, r = (lb - c * ng) * NR, lane = threadIdx.x;
  const int lo = d.comp_off[c], hi = d.comp_off[c + 1], mid = d.comp_mid[c];
  if (lo >= hi) return;
  double2 *xa = work + (size_t)r * d.nu;
  const int f = fidx[r];
  if (NR == 2 && r + 1 < R && fidx[r + 1] == f) {
    double2 *const xs[2] = {xa, work + (size_t)(r + 1) * d.nu};
    band_sweeps<2>(d, f, xs, lo, mid, hi, lane);
    return;
  }
  {
    double2 *const xs[1] = {xa};
    band_sweeps<1>(d, f, xs, lo, mid, hi, lane);
  }
  if (NR == 2 && r + 1 < R) {
    slice_fence();
    __syncthreads();
    double2 *const xs[1] = {work + (size_t)(r + 1) * d.nu};
    band_sweeps<1>(d, fidx[r + 1], xs, lo, mid, hi, lane);
  }
}

// Band-solve plan: the register window when both band widths fit one wave
// (ldl_plan 1 selects the LDS window).
static bool ldl_reg_plan(const PrecondDev &d) { return d.ldl_plan == 0 && d.W <= 63 && d.Wc <= 63; }

__global__ void k_pre_out(PrecondDev d, const int *fidx, const double2 *y, const double2 *work, double2 *z) {
  int r = blockIdx.y;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.l) return;
  const double2 *yr = y + (size_t)r * d.l;
  const double2 *yinv = d.yinv + (size_t)fidx[r] * d.b;
  const double2 *ph = work + (size_t)r * d.nu;
  auto cur = [&](int e) {
    double2 c = branch_known(d, yr, yinv, e);
    int ru = d.br_ru[e], rv = d.br_rv[e];
    if (ru != rv) {
      double2 pu = ru >= 0 ? ph[ru] : make_double2(0, 0);
      double2 pv = rv >= 0 ? ph[rv] : make_double2(0, 0);
      double2 dp = cmul2(make_double2(pu.x - pv.x, pu.y - pv.y), yinv[e]);
      c.x += dp.x;
      c.y += dp.y;
    }
    return c;
  };
  int kind = d.link_kind[i];
  double2 out;
  if (kind >= 0) {
    out = cur(kind);
  } else {
    int k = -kind - 1;
    double ox = 0, oy = 0;
    for (int q = d.src_off[k]; q < d.src_off[k + 1]; ++q) {
      double2 c = cur(d.src_br[q]);
      double sg = d.src_sg[q];
      ox += sg * c.x;
      oy += sg * c.y;
    }
    out = make_double2(ox, oy);
  }
  z[(size_t)r * d.l + i] = out;
}

// ---------------------------------------------------------------------------
// nested-dissection solve: one workgroup per (supernode of a level,
// right-hand side), levels by height.  Forward (leaves first): the
// supernode's front vector in LDS is its right-hand side entries plus its
// children's update vectors (extend-add by their positions in its front);
// unit-lower solve with its pivot block; its own update vector = the
// front's structure part minus L21 y, kept for its parent.  Backward (root
// first): z = y / D - L21^T x(structure) with the ancestors' final values,
// then the transposed unit-lower solve.  Deterministic: every sum has a
// fixed order (no atomics).
// ---------------------------------------------------------------------------
constexpr int ND_T = 256;

__global__ void __launch_bounds__(ND_T) k_nd_fwd(PrecondDev d, const int *fidx, double2 *work, int q0, int R) {
  extern __shared__ double2 ndF[];
  const int lb = (int)xcd_block(blockIdx.x, gridDim.x), qf = lb / R, r = lb - qf * R, tid = threadIdx.x;
  const int s = d.lvl_sn[q0 + qf];
  const int f = fidx[r];
  const int sa = d.sn_start[s], ns = d.sn_start[s + 1] - sa;
  const int64_t so = d.st_off[s];
  const int nst = (int)(d.st_off[s + 1] - so);
  double2 *x = work + (size_t)r * d.nu;
  double2 *u = d.uvec + (size_t)r * d.nst_tot;
  for (int i = tid; i < ns; i += ND_T) ndF[i] = x[sa + i];
  for (int t = tid; t < nst; t += ND_T) ndF[ns + t] = make_double2(0, 0);
  __syncthreads();
  for (int q = d.ch_off[s]; q < d.ch_off[s + 1]; ++q) {
    const int c = d.ch_ids[q];
    const int64_t co = d.st_off[c];
    const int nc = (int)(d.st_off[c + 1] - co);
    for (int t = tid; t < nc; t += ND_T) {
      const int p = d.st_pos[co + t];
      const double2 v = u[co + t];
      ndF[p].x += v.x;
      ndF[p].y += v.y;
    }
    __syncthreads();
  }
  const double2 *L = d.l11 + (size_t)f * d.nl11 + d.l11_off[s];   // by columns
  for (int k = 0; k < ns; ++k) {
    const double2 yk = ndF[k];
    const double2 *Lk = L + (size_t)k * ns;
    for (int i = k + 1 + tid; i < ns; i += ND_T) {
      const double2 l = Lk[i];
      ndF[i].x -= l.x * yk.x - l.y * yk.y;
      ndF[i].y -= l.x * yk.y + l.y * yk.x;
    }
    __syncthreads();
  }
  const double2 *L21 = d.l21 + (size_t)f * d.nl21 + d.l21_off[s];   // [k][t]
  for (int t = tid; t < nst; t += ND_T) {
    double2 acc = ndF[ns + t];
    for (int k = 0; k < ns; ++k) {
      const double2 l = L21[(size_t)k * nst + t], yk = ndF[k];
      acc.x -= l.x * yk.x - l.y * yk.y;
      acc.y -= l.x * yk.y + l.y * yk.x;
    }
    u[so + t] = acc;
  }
  for (int i = tid; i < ns; i += ND_T) x[sa + i] = ndF[i];
}

__global__ void __launch_bounds__(ND_T) k_nd_bwd(PrecondDev d, const int *fidx, double2 *work, int q0, int R) {
  extern __shared__ double2 ndF[];
  const int lb = (int)xcd_block(blockIdx.x, gridDim.x), qf = lb / R, r = lb - qf * R, tid = threadIdx.x;
  const int s = d.lvl_sn[q0 + qf];
  const int f = fidx[r];
  const int sa = d.sn_start[s], ns = d.sn_start[s + 1] - sa;
  const int64_t so = d.st_off[s];
  const int nst = (int)(d.st_off[s + 1] - so);
  double2 *x = work + (size_t)r * d.nu;
  const double2 *dg = d.diag + (size_t)f * d.nu;
  for (int t = tid; t < nst; t += ND_T) ndF[ns + t] = x[d.st_ids[so + t]];
  __syncthreads();
  const double2 *L21 = d.l21 + (size_t)f * d.nl21 + d.l21_off[s];   // [k][t]
  for (int i = tid; i < ns; i += ND_T) {
    double2 z = cdiv2(x[sa + i], dg[sa + i]);
    const double2 *Li = L21 + (size_t)i * nst;
    for (int t = 0; t < nst; ++t) {
      const double2 l = Li[t], v = ndF[ns + t];
      z.x -= l.x * v.x - l.y * v.y;
      z.y -= l.x * v.y + l.y * v.x;
    }
    ndF[i] = z;
  }
  __syncthreads();
  const double2 *Lt = d.l11t + (size_t)f * d.nl11 + d.l11_off[s];   // by rows
  for (int k = ns - 1; k > 0; --k) {
    const double2 xk = ndF[k];
    const double2 *Lk = Lt + (size_t)k * ns;   // row k: L(k, i), i < k
    for (int i = tid; i < k; i += ND_T) {
      const double2 l = Lk[i];
      ndF[i].x -= l.x * xk.x - l.y * xk.y;
      ndF[i].y -= l.x * xk.y + l.y * xk.x;
    }
    __syncthreads();
  }
  for (int i = tid; i < ns; i += ND_T) x[sa + i] = ndF[i];
}

static void nd_solve(const PrecondDev &d, const int *fidx, double2 *work, int R, hipStream_t st) {
  static int lds_cap = -1;
  if (lds_cap < 0) {
    int dev = 0, q = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&q, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) q = 65536;
    lds_cap = q;
    if (hipFuncSetAttribute((const void *)k_nd_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, q) != hipSuccess ||
        hipFuncSetAttribute((const void *)k_nd_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, q) != hipSuccess) {
      (void)hipGetLastError();
      lds_cap = 65536;
    }
  }
  for (int h = 0; h < d.nlvl; ++h) {
    const size_t lds = sizeof(double2) * (size_t)std::max(1, d.lvl_front_host[h]);
    if (lds > (size_t)lds_cap) throw SetupError{-1, "nested-dissection front larger than LDS"};
    const int q0 = d.lvl_off_host[h], n = d.lvl_off_host[h + 1] - q0;
    // one workgroup per (front, right-hand side), a front's right-hand
    // sides consecutive on one XCD (they share its factor blocks)
    if (n > 0) k_nd_fwd<<<dim3((unsigned)n * (unsigned)R), ND_T, lds, st>>>(d, fidx, work, q0, R);
  }
  for (int h = d.nlvl - 1; h >= 0; --h) {
    const size_t lds = sizeof(double2) * (size_t)std::max(1, d.lvl_front_host[h]);
    const int q0 = d.lvl_off_host[h], n = d.lvl_off_host[h + 1] - q0;
    if (n > 0) k_nd_bwd<<<dim3((unsigned)n * (unsigned)R), ND_T, lds, st>>>(d, fidx, work, q0, R);
  }
}

void precond_apply(const PrecondDev &d, const int *fidx, const double2 *y, double2 *z, double2 *work, int R,
                   hipStream_t st) {
  k_pre_rhs<<<dim3((d.nu + 255) / 256, R), 256, 0, st>>>(d, fidx, y, work);
  if (d.nd) {
    nd_solve(d, fidx, work, R, st);
    k_pre_out<<<dim3((d.l + 255) / 256, R), 256, 0, st>>>(d, fidx, y, work, z);
    return;
  }
  // the window must hold max(W, Wc) + PF entries: a block of PF rows reaches
  // W (backward) or Wc (forward) beyond its last row while its own rows are
  // still pending
  // one workgroup per (conductor, right-hand side), the right-hand sides of
  // a conductor consecutive on one XCD: right-hand sides of one frequency
  // (adjacent in the solver's order) then read the same factor rows
  // through that XCD's L2
  const dim3 g((unsigned)d.ncomp * (unsigned)R);
  const int span = std::max(d.W, d.Wc) + PF;
  if ((double)d.nu * std::max(d.pr, d.pc) * 16.0 + 1024.0 >= 2147483647.0)
    throw SetupError{-1, "preconditioner band larger than 2 GB per frequency"};
  // the circular LDS window of the widest solve holds 4096 entries
  if (!ldl_reg_plan(d) && span >= 4096) throw SetupError{-1, "preconditioner band too wide for the band solve"};
  if (ldl_reg_plan(d) && d.ncomp * R >= 4 * 1024)
    // many more chains than SIMDs (one wavefront per SIMD at 256 VGPRs):
    // two right-hand sides per wavefront halve the rounds
    k_ldl_solve_reg<2><<<dim3((unsigned)d.ncomp * (unsigned)((R + 1) / 2)), 64, 0, st>>>(d, fidx, work, R);
  else if (ldl_reg_plan(d))
    k_ldl_solve_reg<1><<<g, 64, 0, st>>>(d, fidx, work, R);
  else if (span < 128)
    k_ldl_solve<128><<<g, 64, 0, st>>>(d, fidx, work, R);
  else if (span < 512)
    k_ldl_solve<512><<<g, 64, 0, st>>>(d, fidx, work, R);
  else if (span < 2048)
    k_ldl_solve<2048><<<g, 64, 0, st>>>(d, fidx, work, R);
  else
    k_ldl_solve<4096><<<g, 64, 0, st>>>(d, fidx, work, R);
  k_pre_out<<<dim3((d.l + 255) / 256, R), 256, 0, st>>>(d, fidx, y, work, z);
}


// ---------------------------------------------------------------------------
// device factorization of L_w, one workgroup per (conductor, frequency)
// ---------------------------------------------------------------------------
constexpr int FACT_T = 256;

// 1/D_e with D_e = Z_s G_ee + (j omega mu / 4 pi) K_ee (Eq. Zb's diagonal)
__global__ void k_fac_yinv(FactorArgs a) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x, f = blockIdx.y;
  if (e >= a.b) return;
  const double om = a.omega[f];
  const double zr = sqrt(om * MU0 * a.mu_r / (2.0 * a.sigma));   // Z_s = zr (1 + j)
  const double jw = om * MU0 * a.mu_r / (4.0 * M_PI);
  const double g = a.gdiag[e];
  const double2 D = make_double2(zr * g, zr * g + jw * a.kdiag[e]);
  double2 y = make_double2(0, 0);
  if (D.x == 0.0 && D.y == 0.0)
    a.status[a.nf * a.ncomp + f] = 1;
  else
    y = cdiv2(make_double2(1, 0), D);
  a.yinv[(size_t)f * a.b + e] = y;
}

// Row i of L_w = N D^-1 N^T: band rows into the padded row layout, supernode
// rows into their envelope; the diagonal separately.  One thread per row
// gathers its incident branches (no atomics); the padded column layout is
// cleared for the factorization to fill.
__global__ void k_fac_assemble(FactorArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, f = blockIdx.y;
  if (i >= a.nu) return;
  int lo = 0, hi = a.ncomp;            // conductor of row i
  while (hi - lo > 1) {
    const int m = (lo + hi) >> 1;
    if (a.comp_off[m] <= i) lo = m; else hi = m;
  }
  const bool super = i >= a.comp_mid[lo];
  const double2 *yi = a.yinv + (size_t)f * a.b;
  double2 *rowp = a.env + ((size_t)f * a.nu + i) * a.pr;
  double2 *colp = a.colenv + ((size_t)f * a.nu + i) * a.pc;
  double2 *fr = a.full + (size_t)f * a.nnz_full + a.env_off[i];
  const int fi = a.first[i];
  const double2 zero = make_double2(0, 0);
  for (int t = 0; t < a.pr; ++t) rowp[t] = zero;
  for (int t = 0; t < a.pc; ++t) colp[t] = zero;
  // 64-entry layouts (band width at most 63): the last slot, never part of
  // the band, holds 1 (the register-window solve's self entry)
  if (a.pr == 64) rowp[63] = make_double2(1.0, 0.0);
  if (a.pc == 64) colp[63] = make_double2(1.0, 0.0);
  if (super)
    for (int k = 0; k < i - fi; ++k) fr[k] = zero;
  double2 dsum = zero;
  for (int q = a.inc_off[i]; q < a.inc_off[i + 1]; ++q) {
    const int e = a.inc_br[q];
    const double2 y = yi[e];
    dsum.x += y.x;
    dsum.y += y.y;
    const int o = a.br_ru[e] == i ? a.br_rv[e] : a.br_ru[e];
    if (o >= 0 && o < i) {
      double2 &t = super ? fr[o - fi] : rowp[i - 1 - o];
      t.x -= y.x;
      t.y -= y.y;
    }
  }
  a.diag[(size_t)f * a.nu + i] = dsum;
}

__device__ __forceinline__ bool bad_pivot(double2 d) {
  return !(isfinite(d.x) && isfinite(d.y)) || (d.x == 0.0 && d.y == 0.0);
}

// Right-looking LDL^T over the band rows [lo, mid) of one conductor: step j
// takes d_j and column j of L (l_ij = a_ij / d_j, i = j+1 .. j+W) and applies
// the rank-one update a_ik -= l_ij (d_j l_kj) to the (W x W) trailing window.
// The window holds rows j .. j+W (circular slots, row slot x offset i - k);
// after step j, row j+W+1 enters row j's slot (it receives no update before
// step j+1).  Each supernode row s keeps a circular window of its entries in
// columns j .. j+W and is updated the same way; the supernode block itself is
// factored last.  L is written in place over the assembled values: row i's
// assembled entries are read when it enters the window, before any of its L
// entries is stored.
__global__ void __launch_bounds__(FACT_T) k_ldl_factor(FactorArgs a) {
  extern __shared__ double2 fsm[];
  const int c = blockIdx.x, f = blockIdx.y, tid = threadIdx.x;
  const int lo = a.comp_off[c], mid = a.comp_mid[c], hi = a.comp_off[c + 1];
  const int ns = hi - mid;
  const int W = a.W, Wp = a.W + 1, Wc = a.Wc, pr = a.pr, pc = a.pc;
  double2 *env = a.env + (size_t)f * a.nu * pr;
  double2 *col = a.colenv + (size_t)f * a.nu * pc;
  double2 *full = a.full + (size_t)f * a.nnz_full;
  double2 *dg = a.diag + (size_t)f * a.nu;
  double2 *lcol = fsm, *ucol = fsm + Wp, *lsn = ucol + Wp, *usn = lsn + FACT_NS, *S = usn + FACT_NS;
  double2 *win = S + FACT_NS * FACT_NS, *swin = win + Wp * Wp;
  const double2 zero = make_double2(0, 0);
  // window rows lo .. lo+W (slot = row - lo)
  for (int idx = tid; idx < Wp * Wp; idx += FACT_T) {
    const int q = idx / Wp, o = idx - q * Wp, i = lo + q;
    double2 v = zero;
    if (i < mid) v = o == 0 ? dg[i] : env[(size_t)i * pr + (o - 1)];
    win[idx] = v;
  }
  for (int idx = tid; idx < ns * Wp; idx += FACT_T) {
    const int s = idx / Wp, q = idx - s * Wp, k = lo + q, row = mid + s, fs = a.first[row];
    swin[idx] = (k < mid && k >= fs) ? full[a.env_off[row] + (k - fs)] : zero;
  }
  for (int idx = tid; idx < ns * ns; idx += FACT_T) {
    const int s = idx / ns, s2 = idx - s * ns, row = mid + s, k = mid + s2, fs = a.first[row];
    double2 v = zero;
    if (s2 == s)
      v = dg[row];
    else if (s2 < s && k >= fs)
      v = full[a.env_off[row] + (k - fs)];
    S[s * FACT_NS + s2] = v;
  }
  __syncthreads();
  const int npair = W * (W + 1) / 2;
  int sj = 0;
  bool bad = false;
  for (int j = lo; j < mid; ++j) {
    const double2 d = win[sj * Wp];
    if (bad_pivot(d)) {     // uniform: every thread read the same value
      bad = true;
      break;
    }
    // column j of L, and of the supernode rows
    for (int t = tid; t <= W + ns; t += FACT_T) {
      if (t == 0) {
        dg[j] = d;
      } else if (t <= W) {
        const int i = j + t;
        double2 u = zero, l = zero;
        if (i < mid) {
          int si = sj + t;
          if (si >= Wp) si -= Wp;
          u = win[si * Wp + t];
          l = cdiv2(u, d);
          env[(size_t)i * pr + (t - 1)] = l;
        }
        ucol[t] = u;
        lcol[t] = l;
        if (t <= Wc) col[(size_t)j * pc + (t - 1)] = l;
      } else {
        const int s = t - W - 1, row = mid + s, fs = a.first[row];
        const double2 u = swin[s * Wp + sj], l = cdiv2(u, d);
        usn[s] = u;
        lsn[s] = l;
        if (j >= fs) full[a.env_off[row] + (j - fs)] = l;
      }
    }
    __syncthreads();
    // trailing update: pair (t, t2), 1 <= t2 <= t <= W, is entry (j+t, j+t2)
    for (int p = tid; p < npair; p += FACT_T) {
      int r0 = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
      while ((r0 + 1) * (r0 + 2) / 2 <= p) ++r0;
      while (r0 * (r0 + 1) / 2 > p) --r0;
      const int t = r0 + 1, t2 = p - r0 * (r0 + 1) / 2 + 1;
      if (j + t < mid) {
        int si = sj + t;
        if (si >= Wp) si -= Wp;
        double2 &w = win[si * Wp + (t - t2)];
        const double2 l = lcol[t], u = ucol[t2];
        w.x -= l.x * u.x - l.y * u.y;
        w.y -= l.x * u.y + l.y * u.x;
      }
    }
    for (int p = tid; p < ns * W; p += FACT_T) {
      const int s = p / W, t = p - s * W + 1;
      if (j + t < mid) {
        int sk = sj + t;
        if (sk >= Wp) sk -= Wp;
        double2 &w = swin[s * Wp + sk];
        const double2 l = lsn[s], u = ucol[t];
        w.x -= l.x * u.x - l.y * u.y;
        w.y -= l.x * u.y + l.y * u.x;
      }
    }
    for (int p = tid; p < ns * ns; p += FACT_T) {
      const int s = p / ns, s2 = p - s * ns;
      if (s2 <= s) {
        double2 &w = S[s * FACT_NS + s2];
        const double2 l = lsn[s], u = usn[s2];
        w.x -= l.x * u.x - l.y * u.y;
        w.y -= l.x * u.y + l.y * u.x;
      }
    }
    // row j+W+1 (and the supernode entries of column j+W+1) into slot sj
    const int inew = j + Wp;
    for (int o = tid; o < Wp; o += FACT_T) {
      double2 v = zero;
      if (inew < mid) v = o == 0 ? dg[inew] : env[(size_t)inew * pr + (o - 1)];
      win[sj * Wp + o] = v;
    }
    for (int s = tid; s < ns; s += FACT_T) {
      const int row = mid + s, fs = a.first[row];
      swin[s * Wp + sj] = (inew < mid && inew >= fs) ? full[a.env_off[row] + (inew - fs)] : zero;
    }
    __syncthreads();
    if (++sj == Wp) sj = 0;
  }
  __syncthreads();
  if (tid != 0) return;
  // supernode block: dense right-looking LDL^T (u values stay in S)
  for (int s = 0; s < ns && !bad; ++s) {
    const double2 d = S[s * FACT_NS + s];
    if (bad_pivot(d)) {
      bad = true;
      break;
    }
    dg[mid + s] = d;
    for (int s2 = s + 1; s2 < ns; ++s2) {
      const double2 u = S[s2 * FACT_NS + s], l = cdiv2(u, d);
      const int row = mid + s2, k = mid + s, fs = a.first[row];
      if (k >= fs) full[a.env_off[row] + (k - fs)] = l;
      for (int s3 = s + 1; s3 <= s2; ++s3) {
        double2 &w = S[s2 * FACT_NS + s3];
        const double2 v = S[s3 * FACT_NS + s];
        w.x -= l.x * v.x - l.y * v.y;
        w.y -= l.x * v.y + l.y * v.x;
      }
    }
  }
  if (bad) a.status[f * a.ncomp + c] = 2;
}

__global__ void k_fill_int(int *p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

static size_t factor_lds_bytes(int W) {
  const size_t Wp = (size_t)W + 1;
  return (2 * Wp + 2 * FACT_NS + FACT_NS * FACT_NS + Wp * Wp + FACT_NS * Wp) * sizeof(double2);
}

static bool factor_allow_lds(const void *fn, size_t bytes) {
  if (bytes <= 65536) return true;
  int dev = 0, q = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&q, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) q = 65536;
  if (bytes > (size_t)std::min(q, 131072)) return false;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return true;
}

bool factor_device_ok(const PrecondStruct &ps) {
  for (int c = 0; c < ps.ncomp; ++c)
    if (ps.comp_off[c + 1] - ps.comp_mid[c] > FACT_NS) return false;
  return factor_allow_lds((const void *)k_ldl_factor, factor_lds_bytes(std::max(ps.W, 1)));
}

void factor_precond_device(const FactorArgs &a, hipStream_t st) {
  const int nst = a.nf * a.ncomp + a.nf;
  k_fill_int<<<(nst + 255) / 256, 256, 0, st>>>(a.status, nst, 0);
  k_fac_yinv<<<dim3((a.b + 255) / 256, a.nf), 256, 0, st>>>(a);
  k_fac_assemble<<<dim3((a.nu + 255) / 256, a.nf), 256, 0, st>>>(a);
  k_ldl_factor<<<dim3(a.ncomp, a.nf), FACT_T, factor_lds_bytes(a.W), st>>>(a);
  hip_ok(hipGetLastError(), "factor launch");
}

}  // namespace pfft
