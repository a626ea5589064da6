// C ABI: context setup, device upload, kernel spectrum, pFFT matvec.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>

#include "engine.h"
#include "learned.h"

namespace pfft {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

void hip_ok(hipError_t e, const char *what) {
  if (e != hipSuccess) {
    int code = (e == hipErrorOutOfMemory) ? PFFT_ENOMEM : PFFT_EDEVICE;
    throw DeviceError{code, std::string(what) + ": " + hipGetErrorString(e)};
  }
}

static constexpr double MU0 = 4e-7 * M_PI;

void StageTimer::begin(int s, hipStream_t st) {
  if (!on) return;
  end(st);
  hip_ok(hipEventCreate(&open_ev), "hipEventCreate");
  hip_ok(hipEventRecord(open_ev, st), "hipEventRecord");
  open_stage = s;
}

void StageTimer::end(hipStream_t st) {
  if (!on || open_stage < 0) return;
  hipEvent_t e;
  hip_ok(hipEventCreate(&e), "hipEventCreate");
  hip_ok(hipEventRecord(e, st), "hipEventRecord");
  pending.push_back(Rec{open_stage, open_ev, e});
  open_stage = -1;
  open_ev = nullptr;
}

void StageTimer::collect() {
  for (auto &r : pending) {
    hip_ok(hipEventSynchronize(r.b), "hipEventSynchronize");
    float t = 0;
    hip_ok(hipEventElapsedTime(&t, r.a, r.b), "hipEventElapsedTime");
    ms[r.stage] += t;
    calls[r.stage] += 1;
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  pending.clear();
}

struct TimerHook : PassHook {
  StageTimer *t;
  explicit TimerHook(StageTimer *tt) : t(tt) {}
  void pass(int k, hipStream_t st) override { t->begin(ST_FFT_X + k, st); }
  void done(hipStream_t st) override { t->end(st); }
};

}  // namespace pfft

using namespace pfft;

void *pfft_ctx::dalloc(size_t bytes) {
  void *p = nullptr;
  if (bytes == 0) bytes = 16;
  hip_ok(hipMalloc(&p, bytes), "hipMalloc");
  allocs.push_back(p);
  dev_bytes += bytes;
  return p;
}

template <typename V>
static V *upload(pfft_ctx *c, const std::vector<V> &h, hipStream_t st) {
  V *d = (V *)c->dalloc(h.size() * sizeof(V));
  if (!h.empty()) hip_ok(hipMemcpyAsync(d, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice, st), "upload");
  hip_ok(hipStreamSynchronize(st), "upload sync");
  return d;
}

size_t pfft_ctx::per_rhs_bytes() const {
  size_t vs = grid_fp64 ? sizeof(double2) : sizeof(float2);
  size_t N = (size_t)m.dims[0] * m.dims[1] * m.dims[2];
  const size_t grid = (9 + (convolve_uses_t2(gm, grid_fp64) ? 12 : 0)) * N;
  return 16 * ((size_t)m.b * 2 + (m.nn + 1) + 4 * (size_t)m.n + 2) + vs * (4 * (size_t)m.n + grid);
}

int pfft_ctx::chunk_for(int R) const {
  int cap = max_chunk;
  if (cap <= 0) cap = (int)std::max<size_t>(1, ws_budget / per_rhs_bytes());
  return std::max(1, std::min(R, cap));
}

void pfft_ctx::ensure_workspace(Workspace &w, int R) {
  if (R <= w.R) return;
  if (w.fixed) throw DeviceError{PFFT_ENOMEM, "fixed scratch too small for the chunk"};
  for (void *p : w.allocs) hipFree(p);
  w.allocs.clear();
  auto al = [&](size_t bytes) {
    void *p = nullptr;
    hip_ok(hipMalloc(&p, bytes ? bytes : 16), "hipMalloc workspace");
    w.allocs.push_back(p);
    return p;
  };
  size_t vs = grid_fp64 ? sizeof(double2) : sizeof(float2);
  size_t N = (size_t)m.dims[0] * m.dims[1] * m.dims[2];
  w.alpha = (double2 *)al(sizeof(double2) * (size_t)R * m.b);
  w.yb = (double2 *)al(sizeof(double2) * (size_t)R * m.b);
  w.scan = (double2 *)al(sizeof(double2) * (size_t)R * (m.nn + 1));
  w.part = (double2 *)al(sizeof(double2) * scan_partials_size(m.nn + 1, R));
  // U also holds the transposed loop vector inside the loop transforms
  w.U = (double2 *)al(sizeof(double2) * (size_t)R * std::max<size_t>((size_t)m.n * 4, (size_t)m.l));
  w.coef = (double2 *)al(sizeof(double2) * 2 * (size_t)R);
  w.J = al(vs * (size_t)R * m.n * 4);
  w.Q = al(vs * (size_t)R * 3 * N);
  w.T1 = al(vs * (size_t)R * 6 * N);
  w.T2 = convolve_uses_t2(gm, grid_fp64) ? al(vs * (size_t)R * 12 * N) : nullptr;
  w.R = R;
  w.coef_on_device.clear();
}

void pfft_ctx::release_workspaces() {
  for (Workspace &w : ws) {
    if (w.fixed) continue;
    for (void *p : w.allocs) hipFree(p);
    w = Workspace();
  }
}

void pfft_ctx::matvec(int R, const double *omega, int space, int flags, const double2 *x, double2 *y,
                      hipStream_t st) {
  const int dim = space == 1 ? m.l : m.b;
  run_split(R, st, [&](int r0, int rn, hipStream_t s2, Workspace &w) {
    matvec_range(w, rn, omega ? omega + r0 : nullptr, space, flags, x + (size_t)r0 * dim, y + (size_t)r0 * dim, s2);
  });
}

void pfft_ctx::matvec_range(Workspace &w, int R, const double *omega, int space, int flags, const double2 *x,
                            double2 *y, hipStream_t st, const PostOut *post) {
  const int dim = space == 1 ? m.l : m.b;
  const int Rc = w.fixed ? std::min(w.R, R) : chunk_for(R);
  ensure_workspace(w, Rc);
  if (!w.T2 && !(flags & PFFT_NEAR_ONLY) && convolve_uses_t2(gm, grid_fp64)) {
    if (w.fixed) throw DeviceError{PFFT_ENOMEM, "the fixed scratch was carved without the unfused FFT buffer"};
    // a plan change since the workspace was sized now needs the unfused passes' buffer
    const size_t vs = grid_fp64 ? sizeof(double2) : sizeof(float2);
    void *p = nullptr;
    hip_ok(hipMalloc(&p, vs * (size_t)w.R * 12 * m.dims[0] * m.dims[1] * m.dims[2]), "hipMalloc workspace");
    w.allocs.push_back(p);
    w.T2 = p;
  }
  int mode = 0;
  if (!(flags & PFFT_NEAR_ONLY)) mode |= 1;
  if (!(flags & PFFT_FAR_ONLY)) mode |= 2;
  if (space == 1) mode |= 4;
  w.host_coef.resize(2 * (size_t)Rc);
  for (int r0 = 0; r0 < R; r0 += Rc) {
    int Rn = std::min(Rc, R - r0);
    const double2 *xc = x + (size_t)r0 * dim;
    double2 *yc = y + (size_t)r0 * dim;
    const double2 *alpha;
    TimerHook hook(&timer);
    PassHook *hk = timer.on ? &hook : nullptr;
    if (space == 1) {
      timer.begin(ST_LOOP_TO_BRANCH, st);
      loop_to_branch(lm, xc, w.alpha, w.scan, w.part, w.U, Rn, st);   // U is free until interpolation
    } else {
      timer.begin(ST_LOOP_TO_BRANCH, st);
      transpose(xc, w.alpha, Rn, m.b, st);
    }
    alpha = w.alpha;
    if (mode & 1) {
      if (grid_fp64) {
        timer.begin(ST_TRI_CURRENT, st);
        tri_currents<double>(gm, alpha, (double2 *)w.J, Rn, st);
        timer.begin(ST_PROJECT, st);
        project<double>(gm, (double2 *)w.J, (double2 *)w.Q, Rn, st);
        timer.end(st);
        convolve<double>(gm, (double2 *)w.Q, (double2 *)w.T1, (double2 *)w.T2, Rn, st, hk);
        timer.begin(ST_INTERP, st);
        interp_tri<double>(gm, (double2 *)w.Q, w.U, Rn, st, w.T1);
      } else {
        timer.begin(ST_TRI_CURRENT, st);
        tri_currents<float>(gm, alpha, (float2 *)w.J, Rn, st);
        timer.begin(ST_PROJECT, st);
        project<float>(gm, (float2 *)w.J, (float2 *)w.Q, Rn, st);
        timer.end(st);
        convolve<float>(gm, (float2 *)w.Q, (float2 *)w.T1, (float2 *)w.T2, Rn, st, hk);
        timer.begin(ST_INTERP, st);
        interp_tri<float>(gm, (float2 *)w.Q, w.U, Rn, st, w.T1);
      }
    }
    double2 *zs = w.coef, *jw = w.coef + Rc;
    if (space == 1) {
      for (int r = 0; r < Rn; ++r) {
        double om = omega[r0 + r];
        double a = std::sqrt(om * MU0 * mu_r / (2.0 * sigma));
        w.host_coef[r] = make_double2(a, a);
        w.host_coef[Rc + r] = make_double2(0.0, om * MU0 * mu_r / (4.0 * M_PI));
      }
      timer.end(st);
      // per-RHS coefficients: uploaded only when they change, so a product
      // captured in a graph holds no host-to-device copy
      const bool single = Rn == R;
      if (!single || w.coef_on_device != w.host_coef) {
        hip_ok(hipMemcpyAsync(w.coef, w.host_coef.data(), sizeof(double2) * 2 * Rc, hipMemcpyHostToDevice, st),
               "coef upload");
        if (single) w.coef_on_device = w.host_coef;
        else w.coef_on_device.clear();
      }
      timer.begin(ST_COMBINE, st);
      combine(cm, alpha, w.U, zs, jw, w.yb, Rn, mode, st);
      timer.begin(ST_BRANCH_TO_LOOP, st);
      branch_to_loop(lm, w.yb, yc, w.scan, w.part, w.U, Rn, st);   // U was last read by combine
      if (post) {
        PostOut o = *post;
        if (o.Ib) o.Ib += (size_t)r0 * (m.b + m.p);
        if (o.Vb) o.Vb += (size_t)r0 * m.b;
        if (o.J) o.J += (size_t)r0 * m.n * 3;
        if (o.phi) o.phi += (size_t)r0 * m.n;
        post_outputs(gm, lm, o, xc, alpha, w.yb, w.scan, Rn, st);
      }
    } else {
      timer.begin(ST_COMBINE, st);
      combine(cm, alpha, w.U, zs, jw, w.yb, Rn, mode, st);
      timer.begin(ST_BRANCH_TO_LOOP, st);
      transpose(w.yb, yc, m.b, Rn, st);
    }
    timer.end(st);
  }
  hip_ok(hipGetLastError(), "matvec launch");
}

// ---------------------------------------------------------------------------
// setup: host model -> device maps
// ---------------------------------------------------------------------------
static void build_device(pfft_ctx *c, hipStream_t st) {
  HostModel &m = c->m;
  const int nn = m.nn, b = m.b, n = m.n, l = m.l;
  // ---- A^T maps
  std::vector<int> inj_cnt(nn + 1, 0);
  for (int i = 0; i < l; ++i) {
    int e = m.links[i];
    if (m.bu[e] == m.bv[e]) continue;
    inj_cnt[m.pre[m.bv[e]] + 1]++;
    inj_cnt[m.pre[m.bu[e]] + 1]++;
  }
  for (int k = 0; k < nn; ++k) inj_cnt[k + 1] += inj_cnt[k];
  std::vector<int> inj_link(inj_cnt[nn]);
  std::vector<int8_t> inj_sgn(inj_cnt[nn]);
  {
    std::vector<int> f(inj_cnt.begin(), inj_cnt.end() - 1);
    for (int i = 0; i < l; ++i) {
      int e = m.links[i];
      if (m.bu[e] == m.bv[e]) continue;
      int kv = m.pre[m.bv[e]], ku = m.pre[m.bu[e]];
      inj_link[f[kv]] = i;
      inj_sgn[f[kv]++] = 1;
      inj_link[f[ku]] = i;
      inj_sgn[f[ku]++] = -1;
    }
  }
  std::vector<int> link_of_branch(b + m.p, -1);
  for (int i = 0; i < l; ++i) link_of_branch[m.links[i]] = i;
  std::vector<int> child_of_twig(b + m.p, -1);
  for (int y = 0; y < nn; ++y)
    if (m.parent_branch[y] >= 0) child_of_twig[m.parent_branch[y]] = y;
  std::vector<int> br_a(b), br_lo(b, 0), br_hi(b, 0);
  std::vector<int8_t> br_sg(b, 0);
  for (int e = 0; e < b; ++e) {
    if (!m.twig[e]) {
      br_a[e] = link_of_branch[e];
    } else {
      int y = child_of_twig[e];
      br_a[e] = -1;
      br_lo[e] = m.pre[y];
      br_hi[e] = m.pre[y] + m.sub[y];
      br_sg[e] = (m.bu[e] == y) ? 1 : -1;
    }
  }
  // ---- A maps
  std::vector<int> pos_branch(nn, -1);
  std::vector<int8_t> pos_sign(nn, 0);
  std::vector<int> end_cnt(nn + 1, 0);
  for (int k = 0; k < nn; ++k) {
    int z = m.order[k];
    int e = m.parent_branch[z];
    if (e >= 0) {
      pos_branch[k] = e;
      pos_sign[k] = (m.bu[e] == z) ? 1 : -1;
      int kend = m.pre[z] + m.sub[z];
      if (kend < nn) end_cnt[kend + 1]++;
    }
  }
  for (int k = 0; k < nn; ++k) end_cnt[k + 1] += end_cnt[k];
  std::vector<int> end_pos(end_cnt[nn]);
  {
    std::vector<int> f(end_cnt.begin(), end_cnt.end() - 1);
    for (int k = 0; k < nn; ++k) {
      int z = m.order[k];
      if (m.parent_branch[z] < 0) continue;
      int kend = m.pre[z] + m.sub[z];
      if (kend < nn) end_pos[f[kend]++] = k;
    }
  }
  // per position k, the signed branch voltages that make up D[k] before the
  // scan: its own twig (sign s_k) then, negated, the twig of every node
  // whose subtree ends at k; code = 2 e + (sign < 0)
  std::vector<int> dd_off(nn + 1, 0), dd_code;
  dd_code.reserve((size_t)nn + end_pos.size());
  for (int k = 0; k < nn; ++k) {
    if (pos_branch[k] >= 0) dd_code.push_back(2 * pos_branch[k] + (pos_sign[k] < 0 ? 1 : 0));
    for (int q = end_cnt[k]; q < end_cnt[k + 1]; ++q) {
      const int j = end_pos[q];
      dd_code.push_back(2 * pos_branch[j] + (pos_sign[j] > 0 ? 1 : 0));
    }
    dd_off[k + 1] = (int)dd_code.size();
  }
  std::vector<int> link_upos(l, -1), link_vpos(l, -1);
  for (int i = 0; i < l; ++i) {
    int e = m.links[i];
    if (m.bu[e] != m.bv[e]) {
      link_upos[i] = m.pre[m.bu[e]];
      link_vpos[i] = m.pre[m.bv[e]];
    }
  }
  LoopMaps &lm = c->lm;
  lm.nn = nn;
  lm.b = b;
  lm.l = l;
  lm.inj_off = upload(c, inj_cnt, st);
  lm.inj_link = upload(c, inj_link, st);
  lm.inj_sgn = upload(c, inj_sgn, st);
  lm.br_a = upload(c, br_a, st);
  lm.br_lo = upload(c, br_lo, st);
  lm.br_hi = upload(c, br_hi, st);
  lm.br_sg = upload(c, br_sg, st);
  lm.dd_off = upload(c, dd_off, st);
  lm.dd_code = upload(c, dd_code, st);
  lm.link_branch = upload(c, m.links, st);
  lm.link_upos = upload(c, link_upos, st);
  lm.link_vpos = upload(c, link_vpos, st);
  // ---- grid maps
  GridMaps &g = c->gm;
  g.n = n;
  g.b = b;
  for (int d = 0; d < 3; ++d) g.dims[d] = m.dims[d];
  const long N = (long)m.dims[0] * m.dims[1] * m.dims[2];
  g.N = (int)N;
  std::vector<double> inv2A(n);
  for (int t = 0; t < n; ++t) inv2A[t] = 1.0 / (2.0 * m.area[t]);
  g.tri_edge = upload(c, m.tri_edge, st);
  g.tri_sign = upload(c, m.tri_sign, st);
  g.inv2A = upload(c, inv2A, st);
  g.pl = upload(c, m.pl, st);
  g.anchor = upload(c, m.anchor, st);
  std::vector<int> pg_off(N + 1, 0);
  auto node_of = [&](int t, int k) {
    int i = k >> 4, j = (k >> 2) & 3, q = k & 3;
    return ((long)(m.anchor[3 * t] + i) * m.dims[1] + (m.anchor[3 * t + 1] + j)) * m.dims[2] +
           (m.anchor[3 * t + 2] + q);
  };
  for (int t = 0; t < n; ++t)
    for (int k = 0; k < 64; ++k) pg_off[node_of(t, k) + 1]++;
  for (long q = 0; q < N; ++q) pg_off[q + 1] += pg_off[q];
  std::vector<int> pg_tri(pg_off[N]);
  std::vector<double> pg_w(4 * (size_t)pg_off[N]);
  {
    std::vector<int> f(pg_off.begin(), pg_off.end() - 1);
    for (int t = 0; t < n; ++t)
      for (int k = 0; k < 64; ++k) {
        long node = node_of(t, k);
        int q = f[node]++;
        pg_tri[q] = t;
        pg_w[4 * (size_t)q] = m.M0[64 * (size_t)t + k];
        for (int cc = 0; cc < 3; ++cc) pg_w[4 * (size_t)q + 1 + cc] = m.M1[192 * (size_t)t + 3 * k + cc];
      }
  }
  std::vector<double> tri_w(256 * (size_t)n);
  for (int t = 0; t < n; ++t)
    for (int k = 0; k < 64; ++k) {
      tri_w[256 * (size_t)t + 4 * k] = m.M0[64 * (size_t)t + k];
      for (int cc = 0; cc < 3; ++cc) tri_w[256 * (size_t)t + 4 * k + 1 + cc] = m.M1[192 * (size_t)t + 3 * k + cc];
    }
  // projection tiles: TZ x TY x TX nodes with z fastest (the Q layout), each
  // listing the triangles whose 4 x 4 x 4 stencil meets it.  16 x 8 x 4
  // nodes: a tile's z runs are whole 128-byte lines of the FP32 grid, and
  // on the package traces its triangle lists overflow the staging area for
  // 0.3% of the gather entries (32 x 4 x 4 tiles: 7.9%)
  {
    const int TZ = std::min(m.dims[2], 16), TY = std::min(m.dims[1], 8);
    const int TX = std::min(m.dims[0], std::max(1, 512 / (TY * TZ)));
    const int nt3[3] = {(m.dims[0] + TX - 1) / TX, (m.dims[1] + TY - 1) / TY, (m.dims[2] + TZ - 1) / TZ};
    const int T3[3] = {TX, TY, TZ};
    const long ntile = (long)nt3[0] * nt3[1] * nt3[2];
    std::vector<int> tt_off(ntile + 1, 0);
    auto tiles_of = [&](int t, auto &&fn) {
      int lo[3], hi[3];
      for (int d = 0; d < 3; ++d) {
        lo[d] = m.anchor[3 * t + d] / T3[d];
        hi[d] = std::min(nt3[d] - 1, (m.anchor[3 * t + d] + 3) / T3[d]);
      }
      for (int a = lo[0]; a <= hi[0]; ++a)
        for (int b2 = lo[1]; b2 <= hi[1]; ++b2)
          for (int c2 = lo[2]; c2 <= hi[2]; ++c2) fn(((long)a * nt3[1] + b2) * nt3[2] + c2);
    };
    for (int t = 0; t < n; ++t) tiles_of(t, [&](long T) { tt_off[T + 1]++; });
    for (long T = 0; T < ntile; ++T) tt_off[T + 1] += tt_off[T];
    std::vector<int> tt_tri(tt_off[ntile]);
    {
      std::vector<int> f(tt_off.begin(), tt_off.end() - 1);
      for (int t = 0; t < n; ++t) tiles_of(t, [&](long T) { tt_tri[f[T]++] = t; });
    }
    std::vector<int> pg_loc(pg_tri.size());
    for (long node = 0; node < N; ++node) {
      const int z = (int)(node % m.dims[2]), y = (int)((node / m.dims[2]) % m.dims[1]),
                x = (int)(node / ((long)m.dims[2] * m.dims[1]));
      const long T = ((long)(x / TX) * nt3[1] + y / TY) * nt3[2] + z / TZ;
      const int *b0 = tt_tri.data() + tt_off[T], *b1 = tt_tri.data() + tt_off[T + 1];
      for (int q = pg_off[node]; q < pg_off[node + 1]; ++q) {
        const int *it = std::lower_bound(b0, b1, pg_tri[q]);
        if (it == b1 || *it != pg_tri[q]) throw SetupError{PFFT_EINVAL, "projection tile lists inconsistent"};
        pg_loc[q] = (int)(it - b0);
      }
    }
    // nodes of each tile by descending gather length (ties by local index)
    const int TN = TX * TY * TZ;
    std::vector<uint16_t> tn_perm((size_t)ntile * TN);
    {
      std::vector<std::pair<int, int>> key(TN);
      for (long T = 0; T < ntile; ++T) {
        const int tz = (int)(T % nt3[2]), ty = (int)((T / nt3[2]) % nt3[1]), tx = (int)(T / ((long)nt3[2] * nt3[1]));
        for (int u = 0; u < TN; ++u) {
          const int iz = u % TZ, iy = (u / TZ) % TY, ix = u / (TZ * TY);
          const int x = tx * TX + ix, y = ty * TY + iy, z = tz * TZ + iz;
          int len = -1;
          if (x < m.dims[0] && y < m.dims[1] && z < m.dims[2]) {
            const long node = ((long)x * m.dims[1] + y) * m.dims[2] + z;
            len = pg_off[node + 1] - pg_off[node];
          }
          key[u] = {-len, u};
        }
        std::sort(key.begin(), key.end());
        for (int u = 0; u < TN; ++u) tn_perm[(size_t)T * TN + u] = (uint16_t)key[u].second;
      }
    }
    for (int d = 0; d < 3; ++d) {
      g.tile[d] = T3[d];
      g.ntile[d] = nt3[d];
    }
    g.tn_perm = upload(c, tn_perm, st);
    // LDS: tcap triangles x 16 (FP32) or 2 (FP64) right-hand sides x 4
    // moments at a 528- or 144-byte pitch, at most 120 KB (or 53 KB)
    {
      int tmax = 1;
      for (long T = 0; T < ntile; ++T) tmax = std::max(tmax, tt_off[T + 1] - tt_off[T]);
      g.tcap = c->grid_fp64 ? 376 : std::min(tmax, 232);
    }
    // sliced gather lists in the tile's node order
    {
      const int nwave = (TN + 63) / 64;
      const size_t ns_ = (size_t)ntile * nwave;
      std::vector<int> ps_off(ns_ + 1, 0), ps_k(ns_, 0);
      auto node_at = [&](long T, int u) -> long {
        const int tz = (int)(T % nt3[2]), ty = (int)((T / nt3[2]) % nt3[1]), tx = (int)(T / ((long)nt3[2] * nt3[1]));
        const int v = tn_perm[(size_t)T * TN + u];
        const int iz = v % TZ, iy = (v / TZ) % TY, ix = v / (TZ * TY);
        const int x = tx * TX + ix, y = ty * TY + iy, z = tz * TZ + iz;
        if (x >= m.dims[0] || y >= m.dims[1] || z >= m.dims[2]) return -1;
        return ((long)x * m.dims[1] + y) * m.dims[2] + z;
      };
      for (long T = 0; T < ntile; ++T)
        for (int w = 0; w < nwave; ++w) {
          int K = 0;
          for (int ln = 0; ln < 64 && w * 64 + ln < TN; ++ln) {
            const long node = node_at(T, w * 64 + ln);
            if (node >= 0) K = std::max(K, pg_off[node + 1] - pg_off[node]);
          }
          const size_t sidx = (size_t)T * nwave + w;
          ps_k[sidx] = K;
          ps_off[sidx + 1] = ps_off[sidx] + 64 * K;
        }
      std::vector<int> ps_ent(ps_off[ns_], 0);
      std::vector<double> ps_w(4 * (size_t)ps_off[ns_], 0.0);
      for (long T = 0; T < ntile; ++T)
        for (int w = 0; w < nwave; ++w) {
          const size_t sidx = (size_t)T * nwave + w;
          for (int ln = 0; ln < 64 && w * 64 + ln < TN; ++ln) {
            const long node = node_at(T, w * 64 + ln);
            if (node < 0) continue;
            for (int k = 0; k < pg_off[node + 1] - pg_off[node]; ++k) {
              const int q = pg_off[node] + k;
              const size_t at = (size_t)ps_off[sidx] + 64 * (size_t)k + ln;
              ps_ent[at] = pg_loc[q] < g.tcap ? pg_loc[q] : -1 - pg_tri[q];
              for (int cc = 0; cc < 4; ++cc) ps_w[4 * at + cc] = pg_w[4 * (size_t)q + cc];
            }
          }
        }
      g.nwave = nwave;
      g.ps_off = upload(c, ps_off, st);
      g.ps_k = upload(c, ps_k, st);
      g.ps_ent = upload(c, ps_ent, st);
      if (c->grid_fp64) {
        g.ps_w = upload(c, ps_w, st);
      } else {
        std::vector<float> a(ps_w.begin(), ps_w.end());
        g.ps_w = upload(c, a, st);
      }
    }
    g.fft_plan = c->plans.fft;
    g.proj_plan = c->plans.proj;
    g.proj_rhs = c->plans.proj_rhs;
    g.tt_off = upload(c, tt_off, st);
    g.tt_tri = upload(c, tt_tri, st);
    g.pg_loc = upload(c, pg_loc, st);
  }
  {
    std::vector<int> act, act_of(N, -1);
    for (long node = 0; node < N; ++node)
      if (pg_off[node + 1] > pg_off[node]) {
        act_of[node] = (int)act.size();
        act.push_back((int)node);
      }
    g.nact = (int)act.size();
    g.act = upload(c, act, st);
    g.act_of = upload(c, act_of, st);
    // masks of the pruned FFT passes
    const int Nx = m.dims[0], Ny = m.dims[1], Nz = m.dims[2];
    const long C = (long)Ny * Nz;
    if (Nx % 32 == 0 && C % 32 == 0) {
      const int wpc = Nx / 32;
      std::vector<uint32_t> xm((size_t)C * wpc, 0u), ca((size_t)(C / 32), 0u);
      std::vector<uint64_t> zm(Nz, 0u);
      std::vector<uint8_t> cg((size_t)(C / 32), 0);
      for (int node : act) {
        const int z = node % Nz, y = (node / Nz) % Ny, x = node / (Nz * Ny);
        const long col = (long)y * Nz + z;
        xm[(size_t)col * wpc + x / 32] |= 1u << (x % 32);
        if (Ny <= 64) zm[z] |= 1ull << y;
        cg[col / 32] = 1;
        ca[col / 32] |= 1u << (col % 32);
      }
      g.xmask = upload(c, xm, st);
      g.zmask = Ny <= 64 ? upload(c, zm, st) : nullptr;
      g.cgrp = upload(c, cg, st);
      g.colact = upload(c, ca, st);
    }
    g.prune = c->plans.prune;
    if (!c->grid_fp64 && (Nx == 32 || Nx == 64 || Nx == 128 || Nx == 256)) {
      const int M = Nx / 4;
      std::vector<float2> tw(16 * (size_t)M);
      for (int r = 0; r < 8; ++r) {
        const int q = r & 3, h = r >> 2, k2 = (q >> 1) | ((q & 1) << 1);
        const double sg = (q & 1) ? -1.0 : 1.0;
        for (int mm = 0; mm < M; ++mm) {
          // exact angle reduction: the exponents modulo 2 Nx
          const long ef = ((long)(2 * k2 + h) * mm) % (2 * Nx);
          const long ei = ((long)2 * k2 * mm + (long)h * k2) % (2 * Nx);
          const double af = -2.0 * M_PI * (double)ef / (2.0 * Nx), ai = 2.0 * M_PI * (double)ei / (2.0 * Nx);
          const double si = sg / (2.0 * Nx);
          tw[(size_t)r * M + mm] = make_float2((float)(sg * std::cos(af)), (float)(sg * std::sin(af)));
          tw[(size_t)(8 + r) * M + mm] = make_float2((float)(si * std::cos(ai)), (float)(si * std::sin(ai)));
        }
      }
      g.xtw = upload(c, tw, st);
    }
  }
  {
    // triangles sorted by anchor (then index); runs of one anchor cut into
    // groups of INTERP_GROUP, in Z-order (Morton) of their anchors: the
    // groups that run at the same time on an XCD then cover a compact block
    // of the grid and share most of their stencil nodes in its L2
    std::vector<int> ord(n);
    for (int t = 0; t < n; ++t) ord[t] = t;
    auto spread3 = [](uint64_t v) {   // bit i of v to bit 3 i
      uint64_t r = 0;
      for (int i = 0; i < 21; ++i) r |= ((v >> i) & 1ull) << (3 * i);
      return r;
    };
    std::vector<uint64_t> mkey(n);
    for (int t = 0; t < n; ++t)
      mkey[t] = (spread3((uint64_t)m.anchor[3 * t]) << 2) | (spread3((uint64_t)m.anchor[3 * t + 1]) << 1) |
                spread3((uint64_t)m.anchor[3 * t + 2]);
    auto key = [&](int t) { return mkey[t]; };
    std::sort(ord.begin(), ord.end(), [&](int a2, int b2) {
      const uint64_t ka = key(a2), kb = key(b2);
      return ka != kb ? ka < kb : a2 < b2;
    });
    std::vector<int> ig_off{0};
    for (int i = 1; i < n; ++i)
      if (key(ord[i]) != key(ord[i - 1]) || i - ig_off.back() == INTERP_GROUP) ig_off.push_back(i);
    ig_off.push_back(n);
    g.nig = n > 0 ? (int)ig_off.size() - 1 : 0;
    g.ig_off = upload(c, ig_off, st);
    g.ig_tri = upload(c, ord, st);
    // the active-node positions of each group's 64 stencil nodes (k = 16 i +
    // 4 j + l for node anchor + (i, j, l)); every stencil node is active
    std::vector<int> act_pos(N, -1);
    for (long node = 0, a = 0; node < N; ++node)
      if (pg_off[node + 1] > pg_off[node]) act_pos[node] = (int)a++;
    std::vector<int> ig_act((size_t)g.nig * 64);
    for (int q = 0; q < g.nig; ++q) {
      const int t = ord[ig_off[q]];
      for (int k = 0; k < 64; ++k) {
        const long node = ((long)(m.anchor[3 * t] + k / 16) * m.dims[1] + (m.anchor[3 * t + 1] + (k / 4) % 4)) *
                              m.dims[2] + (m.anchor[3 * t + 2] + k % 4);
        ig_act[(size_t)q * 64 + k] = act_pos[node];
      }
    }
    g.ig_act = upload(c, ig_act, st);
  }
  g.pg_off = upload(c, pg_off, st);
  g.pg_tri = upload(c, pg_tri, st);
  if (c->grid_fp64) {
    g.pg_w = upload(c, pg_w, st);
    g.tri_w = upload(c, tri_w, st);
    g.tri_wd = (const double *)g.tri_w;
  } else {
    std::vector<float> a(pg_w.begin(), pg_w.end()), bb(tri_w.begin(), tri_w.end());
    g.pg_w = upload(c, a, st);
    g.tri_w = upload(c, bb, st);
    g.tri_wd = upload(c, tri_w, st);
  }
  // ---- kernel spectrum: FFT of the circulant-embedded grid Green's function
  {
    int d2[3] = {2 * m.dims[0], 2 * m.dims[1], 2 * m.dims[2]};
    size_t tot = (size_t)d2[0] * d2[1] * d2[2];
    std::vector<double2> H(tot);
    for (int i = 0; i < d2[0]; ++i) {
      double ox = (i < m.dims[0] ? i : i - d2[0]) * m.h[0];
      bool ux = i == m.dims[0];
      for (int j = 0; j < d2[1]; ++j) {
        double oy = (j < m.dims[1] ? j : j - d2[1]) * m.h[1];
        bool uy = j == m.dims[1];
        for (int k = 0; k < d2[2]; ++k) {
          double oz = (k < m.dims[2] ? k : k - d2[2]) * m.h[2];
          bool uz = k == m.dims[2];
          double R = std::sqrt(ox * ox + oy * oy + oz * oz);
          double v = (ux || uy || uz || R == 0.0) ? 0.0 : 1.0 / R;
          H[((size_t)i * d2[1] + j) * d2[2] + k] = make_double2(v, 0.0);
        }
      }
    }
    double2 *dH = nullptr;
    hip_ok(hipMalloc(&dH, tot * sizeof(double2)), "hipMalloc spectrum");
    hip_ok(hipMemcpyAsync(dH, H.data(), tot * sizeof(double2), hipMemcpyHostToDevice, st), "upload H");
    fft3_full_fp64(dH, d2, st);
    size_t oct = (size_t)(m.dims[0] + 1) * (m.dims[1] + 1) * (m.dims[2] + 1);
    if (c->grid_fp64) {
      double *gh = (double *)c->dalloc(oct * sizeof(double));
      fold_spectrum<double>(dH, gh, m.dims, st);
      g.ghat = gh;
    } else {
      float *gh = (float *)c->dalloc(oct * sizeof(float));
      fold_spectrum<float>(dH, gh, m.dims, st);
      g.ghat = gh;
    }
    hip_ok(hipStreamSynchronize(st), "spectrum");
    hipFree(dH);
  }
  // ---- combine maps
  CombineMaps &cm = c->cm;
  cm.b = b;
  cm.n = n;
  std::vector<int> efar_t(2 * (size_t)b);
  std::vector<double> efar_s(2 * (size_t)b), efar_pl(6 * (size_t)b);
  for (int e = 0; e < b; ++e)
    for (int side = 0; side < 2; ++side) {
      int t = side == 0 ? m.tplus[e] : m.tminus[e];
      int i = 0;
      while (m.tri_edge[3 * t + i] != e) ++i;
      efar_t[2 * e + side] = t;
      efar_s[2 * e + side] = m.tri_sign[3 * t + i] / (2.0 * m.area[t]);
      for (int d = 0; d < 3; ++d) efar_pl[6 * (size_t)e + 3 * side + d] = m.pl[9 * t + 3 * i + d];
    }
  cm.efar_t = upload(c, efar_t, st);
  cm.efar_s = upload(c, efar_s, st);
  cm.efar_pl = upload(c, efar_pl, st);
  cm.nf_rowptr = upload(c, m.nf_rowptr, st);
  cm.nf_col = upload(c, m.nf_col, st);
  cm.nf_val = upload(c, m.nf_val, st);
  cm.gram_col = upload(c, m.gram_col, st);
  cm.gram_val = upload(c, m.gram_val, st);
  // near-field row tiles: the widest tile (rows a power of two, at most 32)
  // whose column lists all fit the LDS staging area of the tiled product
  cm.ctile = 0;
  cm.ctr = 0;
  cm.cmax = 0;
  cm.comb_plan = c->plans.comb;
  cm.crc = 16;
  // dense row tiles of 32 rows for the matrix-core product, built when the
  // tiles are at least half full (near fields are geometric neighbourhoods,
  // so consecutive rows share most columns)
  cm.dn_tiles = 0;
  cm.near_dense = c->plans.near_dense;
  if (b > 0) {
    const int nt = (b + 31) / 32;
    std::vector<std::vector<int>> cols(nt);
    std::vector<int> nu(nt);
#pragma omp parallel for schedule(dynamic, 64)
    for (int T = 0; T < nt; ++T) {
      const int64_t q0 = m.nf_rowptr[(size_t)T * 32], q1 = m.nf_rowptr[std::min(b, (T + 1) * 32)];
      std::vector<int> u(m.nf_col.begin() + q0, m.nf_col.begin() + q1);
      std::sort(u.begin(), u.end());
      u.erase(std::unique(u.begin(), u.end()), u.end());
      nu[T] = (int)u.size();
      const int pad = u.empty() ? 0 : u[0];
      while (u.size() % 16 != 0 || u.empty()) u.push_back(pad);
      cols[T] = std::move(u);
    }
    std::vector<int64_t> off(nt + 1, 0);
    for (int T = 0; T < nt; ++T) off[T + 1] = off[T] + (int64_t)cols[T].size();
    const double fill = (double)m.nf_rowptr[b] / (32.0 * (double)off[nt]);
    if (fill >= 0.5) {
      std::vector<int> dcol(off[nt]);
      std::vector<double> dval(32 * (size_t)off[nt], 0.0);
#pragma omp parallel for schedule(dynamic, 64)
      for (int T = 0; T < nt; ++T) {
        std::copy(cols[T].begin(), cols[T].end(), dcol.begin() + off[T]);
        double *V = dval.data() + 32 * off[T];
        for (int e = T * 32; e < std::min(b, (T + 1) * 32); ++e)
          for (int64_t q = m.nf_rowptr[e]; q < m.nf_rowptr[e + 1]; ++q) {
            const int k = (int)(std::lower_bound(cols[T].begin(), cols[T].begin() + nu[T], m.nf_col[q]) -
                                cols[T].begin());
            V[((size_t)(k / 4) * 32 + (e - T * 32)) * 4 + k % 4] = m.nf_val[q];
          }
      }
      cm.dn_off = upload(c, off, st);
      cm.dn_col = upload(c, dcol, st);
      cm.dn_val = upload(c, dval, st);
      cm.dn_tiles = nt;
    }
  }
  // (right-hand sides, rows) per workgroup, in order of preference; every
  // candidate has at least 128 threads (near fields with long rows, such as
  // the package traces' 580 nonzeros a row, take 4 right-hand sides over 64
  // or 32 rows; without a fit the gather kernel runs)
  static const int cand[][2] = {{16, 32}, {16, 16}, {16, 8}, {8, 32}, {8, 16}, {4, 64}, {4, 32}};
  for (int trial = 0; trial < 7 && cm.ctile == 0 && b > 0; ++trial) {
    const int rc = cand[trial][0], tr = cand[trial][1];
    const int ucap = combine_tile_cap(rc);
    const int nt = (b + tr - 1) / tr;
    std::vector<int> ct_off(nt + 1, 0);
    std::vector<std::vector<int>> cols(nt);
    // a candidate fails at its first tile whose column list overflows the
    // staging area; the other threads then stop sorting
    int over = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int T = 0; T < nt; ++T) {
      int seen;
#pragma omp atomic read
      seen = over;
      if (seen) continue;
      const int64_t q0 = m.nf_rowptr[(size_t)T * tr], q1 = m.nf_rowptr[std::min(b, (T + 1) * tr)];
      std::vector<int> u(m.nf_col.begin() + q0, m.nf_col.begin() + q1);
      std::sort(u.begin(), u.end());
      u.erase(std::unique(u.begin(), u.end()), u.end());
      if ((int)u.size() > ucap) {
#pragma omp atomic write
        over = 1;
      }
      cols[T] = std::move(u);
    }
    if (over) continue;
    int umax = 0;
    for (int T = 0; T < nt; ++T) {
      umax = std::max(umax, (int)cols[T].size());
      ct_off[T + 1] = ct_off[T] + (int)cols[T].size();
    }
    cm.crc = rc;
    std::vector<int> ct_col(ct_off[nt]);
    std::vector<uint16_t> slot(m.nf_col.size());
#pragma omp parallel for schedule(dynamic, 64)
    for (int T = 0; T < nt; ++T) {
      std::copy(cols[T].begin(), cols[T].end(), ct_col.begin() + ct_off[T]);
      for (int e = T * tr; e < std::min(b, (T + 1) * tr); ++e)
        for (int64_t q = m.nf_rowptr[e]; q < m.nf_rowptr[e + 1]; ++q)
          slot[q] = (uint16_t)(std::lower_bound(cols[T].begin(), cols[T].end(), m.nf_col[q]) - cols[T].begin());
    }
    cm.ctr = tr;
    cm.ctile = nt;
    cm.cmax = umax;
    cm.ct_off = upload(c, ct_off, st);
    cm.ct_col = upload(c, ct_col, st);
    cm.nf_slot = upload(c, slot, st);
  }
}

// ---------------------------------------------------------------------------
// Fixed scratch of the no-allocation product (pfft_matvec_noalloc).  Each GPU
// holds its own copy of this array from the first use of the library until
// the process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns with that device current (kept per device).
// ---------------------------------------------------------------------------
static constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::map<int, void *> g_scratch_addr;

// the current device's scratch address (looked up once per device)
static void *device_scratch(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) return it->second;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    throw DeviceError{PFFT_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
  g_scratch_addr[dev] = p;
  return p;
}

// Lays out the product workspace for R right-hand sides from base (256-byte
// aligned pieces) and returns its size; assigns the pointers when w is given.
static size_t carve_workspace(const pfft_ctx *c, int R, unsigned char *base, Workspace *w) {
  const HostModel &m = c->m;
  const size_t vs = c->grid_fp64 ? sizeof(double2) : sizeof(float2);
  const size_t N = (size_t)m.dims[0] * m.dims[1] * m.dims[2];
  const bool t2 = convolve_uses_t2(c->gm, c->grid_fp64);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    void *p = base ? base + off : nullptr;
    off += (std::max<size_t>(bytes, 16) + 255) & ~(size_t)255;
    return p;
  };
  void *alpha = take(sizeof(double2) * (size_t)R * m.b);
  void *yb = take(sizeof(double2) * (size_t)R * m.b);
  void *scan = take(sizeof(double2) * (size_t)R * (m.nn + 1));
  void *part = take(sizeof(double2) * scan_partials_size(m.nn + 1, R));
  void *U = take(sizeof(double2) * (size_t)R * std::max<size_t>((size_t)m.n * 4, (size_t)m.l));
  void *coef = take(sizeof(double2) * 2 * (size_t)R);
  void *J = take(vs * (size_t)R * m.n * 4);
  void *Q = take(vs * (size_t)R * 3 * N);
  void *T1 = take(vs * (size_t)R * 6 * N);
  void *T2 = t2 ? take(vs * (size_t)R * 12 * N) : nullptr;
  if (w) {
    w->alpha = (double2 *)alpha;
    w->yb = (double2 *)yb;
    w->scan = (double2 *)scan;
    w->part = (double2 *)part;
    w->U = (double2 *)U;
    w->coef = (double2 *)coef;
    w->J = J;
    w->Q = Q;
    w->T1 = T1;
    w->T2 = T2;
    w->R = R;
    w->fixed = true;
    w->allocs.clear();
    w->coef_on_device.clear();   // another call may have changed the scratch
  }
  return off;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *pfft_last_error(void) { return g_err.c_str(); }

pfft_status pfft_ctx_get(const pfft_ctx *c, const char *name, void *dst, int64_t cap_bytes, int64_t *len_bytes) {
  if (!c || !name || !len_bytes) {
    set_error("pfft_ctx_get: null argument");
    return PFFT_EINVAL;
  }
  const std::string k(name);
  int64_t n = -1;
  try {
    n = model_get(c->m, k, dst, cap_bytes);
  } catch (const SetupError &e) {
    set_error("pfft_ctx_get: " + e.msg);
    return (pfft_status)e.code;
  }
  if (n < 0) {
    set_error("pfft_ctx_get: unknown array " + k);
    return PFFT_EINVAL;
  }
  *len_bytes = n;
  if (dst && cap_bytes < n) {
    set_error("pfft_ctx_get: buffer too small");
    return PFFT_EINVAL;
  }
  return PFFT_OK;
}

pfft_status pfft_setup(const pfft_problem *pb, void *hip_stream, pfft_ctx **out) {
  if (!pb || !out) {
    set_error("pfft_setup: null argument");
    return PFFT_EINVAL;
  }
  *out = nullptr;
  pfft_ctx *c = nullptr;
  try {
    c = new pfft_ctx();
    c->grid_fp64 = pb->grid_fp64 ? 1 : 0;
    c->sigma = pb->sigma;
    c->mu_r = pb->mu_r > 0 ? pb->mu_r : 1.0;
    c->max_chunk = pb->max_rhs_chunk;
    if (!(pb->sigma > 0)) throw SetupError{PFFT_EINVAL, "sigma must be positive"};
    if (!(pb->near_kappa > 0)) throw SetupError{PFFT_EINVAL, "near_kappa must be positive"};
    SetupOptions opt;
    for (int d = 0; d < 3; ++d) opt.grid[d] = pb->grid[d];
    opt.stencil = pb->stencil;
    opt.kappa = pb->near_kappa;
    opt.contact_zs = pb->contact_zs;
    opt.device_blocks = 1;
    opt.stream = hip_stream;
    build_model(c->m, pb->V, pb->nv, pb->T, pb->nt, pb->nport, pb->src_off, pb->src_tri, pb->snk_off,
                pb->snk_tri, opt);
    hip_ok(hipGetDevice(&c->device), "hipGetDevice");
    c->scratch = device_scratch(c->device);
    {
      const auto t0 = std::chrono::steady_clock::now();
      build_device(c, (hipStream_t)hip_stream);
      c->m.setup_ms[7] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    {
      // product workspaces may take half of the memory left after setup
      // (the rest is for the Krylov bases and preconditioner factors)
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) == hipSuccess) c->ws_budget = std::max(c->ws_budget, fr / 2);
    }
    *out = c;
    return PFFT_OK;
  } catch (const SetupError &e) {
    set_error("pfft_setup: " + e.msg);
    delete c;
    return (pfft_status)e.code;
  } catch (const DeviceError &e) {
    set_error("pfft_setup: " + e.msg);
    delete c;
    return (pfft_status)e.code;
  } catch (const std::bad_alloc &) {
    set_error("pfft_setup: host allocation failed");
    delete c;
    return PFFT_ENOMEM;
  }
}

pfft_status pfft_sizes(const pfft_ctx *c, int64_t out[10]) {
  if (!c || !out) {
    set_error("pfft_sizes: null argument");
    return PFFT_EINVAL;
  }
  const HostModel &m = c->m;
  out[0] = m.n;
  out[1] = m.nn;
  out[2] = m.b;
  out[3] = m.l;
  out[4] = m.s;
  out[5] = m.p;
  out[6] = m.nf_rowptr.empty() ? 0 : m.nf_rowptr.back();
  out[7] = (int64_t)m.dims[0] * m.dims[1] * m.dims[2];
  out[8] = m.npairs;
  out[9] = (int64_t)c->dev_bytes;
  return PFFT_OK;
}

pfft_status pfft_matvec(pfft_ctx *c, int32_t nrhs, const double *omega, int32_t space, int32_t flags,
                        const void *x_dev, void *y_dev, void *hip_stream) {
  if (!c || !x_dev || !y_dev || nrhs < 0 || (space != 0 && space != 1)) {
    set_error("pfft_matvec: bad argument");
    return PFFT_EINVAL;
  }
  if (space == 1 && !omega && nrhs > 0) {
    set_error("pfft_matvec: loop space needs omega");
    return PFFT_EINVAL;
  }
  if ((flags & PFFT_FAR_ONLY) && (flags & PFFT_NEAR_ONLY)) {
    set_error("pfft_matvec: FAR_ONLY and NEAR_ONLY are exclusive");
    return PFFT_EINVAL;
  }
  const int pre_flags = PFFT_PRECOND | PFFT_PRECOND_ONLY | PFFT_LEARNED_ONLY;
  if ((flags & pre_flags) && space != 1) {
    set_error("pfft_matvec: preconditioner flags need loop space");
    return PFFT_EINVAL;
  }
  if (x_dev == y_dev) {
    set_error("pfft_matvec: x and y must not alias");
    return PFFT_EINVAL;
  }
  if (nrhs == 0) return PFFT_OK;
  try {
    hip_ok(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t st = (hipStream_t)hip_stream;
    if (flags & pre_flags) {
      return pfft_internal_precond_matvec(c, nrhs, omega, flags, (const double2 *)x_dev, (double2 *)y_dev, st);
    }
    c->matvec(nrhs, omega, space, flags, (const double2 *)x_dev, (double2 *)y_dev, st);
    return PFFT_OK;
  } catch (const DeviceError &e) {
    set_error("pfft_matvec: " + e.msg);
    return (pfft_status)e.code;
  } catch (const SetupError &e) {
    set_error("pfft_matvec: " + e.msg);
    return (pfft_status)e.code;
  }
}

pfft_status pfft_matvec_noalloc(pfft_ctx *c, int32_t nrhs, const double *omega, int32_t space, int32_t flags,
                                const void *x_dev, void *y_dev, void *hip_stream) {
  if (!c || !x_dev || !y_dev || nrhs < 0 || (space != 0 && space != 1)) {
    set_error("pfft_matvec_noalloc: bad argument");
    return PFFT_EINVAL;
  }
  if (space == 1 && !omega && nrhs > 0) {
    set_error("pfft_matvec_noalloc: loop space needs omega");
    return PFFT_EINVAL;
  }
  if ((flags & PFFT_FAR_ONLY) && (flags & PFFT_NEAR_ONLY)) {
    set_error("pfft_matvec_noalloc: FAR_ONLY and NEAR_ONLY are exclusive");
    return PFFT_EINVAL;
  }
  if (flags & (PFFT_PRECOND | PFFT_PRECOND_ONLY | PFFT_LEARNED_ONLY)) {
    set_error("pfft_matvec_noalloc: the preconditioner flags need per-frequency factors (use pfft_matvec)");
    return PFFT_EINVAL;
  }
  if (x_dev == y_dev) {
    set_error("pfft_matvec_noalloc: x and y must not alias");
    return PFFT_EINVAL;
  }
  if (nrhs == 0) return PFFT_OK;
  const size_t one = carve_workspace(c, 1, nullptr, nullptr);
  if (one > NOALLOC_SCRATCH_BYTES) {
    set_error("pfft_matvec_noalloc: one right-hand side needs " + std::to_string(one) +
              " bytes of scratch; the fixed scratch holds " + std::to_string(NOALLOC_SCRATCH_BYTES));
    return PFFT_ENOMEM;
  }
  try {
    hip_ok(hipSetDevice(c->device), "hipSetDevice");
    // the largest chunk that fits (workspace size grows with R)
    int rfit = 1;
    while (rfit < nrhs) {
      const int nx = std::min(2 * rfit, (int)nrhs);
      if (carve_workspace(c, nx, nullptr, nullptr) > NOALLOC_SCRATCH_BYTES) break;
      rfit = nx;
    }
    carve_workspace(c, rfit, (unsigned char *)c->scratch, &c->ws_fixed);
    c->matvec_range(c->ws_fixed, nrhs, omega, space, flags, (const double2 *)x_dev, (double2 *)y_dev,
                    (hipStream_t)hip_stream);
    return PFFT_OK;
  } catch (const DeviceError &e) {
    set_error("pfft_matvec_noalloc: " + e.msg);
    return (pfft_status)e.code;
  } catch (const SetupError &e) {
    set_error("pfft_matvec_noalloc: " + e.msg);
    return (pfft_status)e.code;
  }
}

pfft_status pfft_postprocess(pfft_ctx *c, int32_t nrhs, const double *omega, const void *Il_dev, void *Vl_dev,
                             void *Ib_dev, void *Vb_dev, void *J_dev, void *phi_dev, void *hip_stream) {
  if (!c || nrhs < 0 || (nrhs > 0 && (!omega || !Il_dev))) {
    set_error("pfft_postprocess: bad argument");
    return PFFT_EINVAL;
  }
  if (nrhs == 0) return PFFT_OK;
  double2 *scratch = nullptr;
  try {
    hip_ok(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t st = (hipStream_t)hip_stream;
    const HostModel &m = c->m;
    if (!c->d_tri_pos) {
      // reference node of each conductor: the sink of its lowest-numbered
      // port, else its root (lowest node)
      std::vector<int> root(m.nn);
      for (int k = 0; k < m.nn; ++k) {
        const int z = m.order[k];   // preorder: a parent precedes its children
        root[z] = m.parent[z] < 0 ? z : root[m.parent[z]];
      }
      std::vector<int> ref(m.nn, -1);
      for (int k = m.p - 1; k >= 0; --k) ref[root[m.bu[m.b + k]]] = m.bu[m.b + k];
      std::vector<int> tpos(m.n), tref(m.n);
      for (int t = 0; t < m.n; ++t) {
        const int z = m.node_of_tri[t], r = root[z];
        tpos[t] = m.pre[z];
        tref[t] = m.pre[ref[r] >= 0 ? ref[r] : r];
      }
      c->d_tri_pos = upload(c, tpos, st);
      c->d_tri_ref = upload(c, tref, st);
      c->d_port_loop = upload(c, m.port_loop, st);
    }
    PostOut o;
    o.Ib = (double2 *)Ib_dev;
    o.Vb = (double2 *)Vb_dev;
    o.J = (double2 *)J_dev;
    o.phi = (double2 *)phi_dev;
    o.p = m.p;
    o.port_loop = c->d_port_loop;
    o.tri_pos = c->d_tri_pos;
    o.tri_ref = c->d_tri_ref;
    double2 *vl = (double2 *)Vl_dev;
    if (!vl) {
      hip_ok(hipMalloc(&scratch, (size_t)nrhs * m.l * sizeof(double2)), "hipMalloc post scratch");
      vl = scratch;
    }
    c->matvec_range(c->ws[0], nrhs, omega, 1, 0, (const double2 *)Il_dev, vl, st, &o);
    if (scratch) {
      hip_ok(hipStreamSynchronize(st), "post sync");
      hipFree(scratch);
    }
    return PFFT_OK;
  } catch (const DeviceError &e) {
    if (scratch) hipFree(scratch);
    set_error("pfft_postprocess: " + e.msg);
    return (pfft_status)e.code;
  } catch (const SetupError &e) {
    if (scratch) hipFree(scratch);
    set_error("pfft_postprocess: " + e.msg);
    return (pfft_status)e.code;
  }
}

pfft_status pfft_profile(pfft_ctx *c, int32_t enable) {
  if (!c) {
    set_error("pfft_profile: null context");
    return PFFT_EINVAL;
  }
  try {
    c->timer.collect();
    c->timer.on = enable != 0;
    for (int i = 0; i < ST_COUNT; ++i) {
      c->timer.ms[i] = 0;
      c->timer.calls[i] = 0;
    }
    return PFFT_OK;
  } catch (const DeviceError &e) {
    set_error("pfft_profile: " + e.msg);
    return (pfft_status)e.code;
  }
}

pfft_status pfft_stage_times(pfft_ctx *c, double ms[16], int64_t calls[16]) {
  if (!c || !ms || !calls) {
    set_error("pfft_stage_times: null argument");
    return PFFT_EINVAL;
  }
  try {
    c->timer.collect();
    for (int i = 0; i < 16; ++i) {
      ms[i] = i < ST_COUNT ? c->timer.ms[i] : 0.0;
      calls[i] = i < ST_COUNT ? c->timer.calls[i] : 0;
    }
    return PFFT_OK;
  } catch (const DeviceError &e) {
    set_error("pfft_stage_times: " + e.msg);
    return (pfft_status)e.code;
  }
}

pfft_status extract_RL(int32_t nfreq, int32_t nport, const double *freq_hz, const void *Y, double *R_out,
                       double *L_out) {
  if (nfreq < 0 || nport <= 0 || !freq_hz || !Y || !R_out || !L_out) {
    set_error("extract_RL: bad argument");
    return PFFT_EINVAL;
  }
  typedef std::complex<double> cd;
  const cd *Yc = (const cd *)Y;
  const int p = nport;
  std::vector<cd> a(p * p), inv(p * p);
  for (int f = 0; f < nfreq; ++f) {
    for (int i = 0; i < p * p; ++i) a[i] = Yc[(size_t)f * p * p + i];
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < p; ++j) inv[i * p + j] = (i == j) ? 1.0 : 0.0;
    // Gauss-Jordan with partial pivoting
    for (int k = 0; k < p; ++k) {
      int piv = k;
      for (int i = k + 1; i < p; ++i)
        if (std::abs(a[i * p + k]) > std::abs(a[piv * p + k])) piv = i;
      if (std::abs(a[piv * p + k]) == 0.0) {
        set_error("extract_RL: singular admittance matrix");
        return PFFT_EINVAL;
      }
      if (piv != k)
        for (int j = 0; j < p; ++j) {
          std::swap(a[k * p + j], a[piv * p + j]);
          std::swap(inv[k * p + j], inv[piv * p + j]);
        }
      cd d = a[k * p + k];
      for (int j = 0; j < p; ++j) {
        a[k * p + j] /= d;
        inv[k * p + j] /= d;
      }
      for (int i = 0; i < p; ++i) {
        if (i == k) continue;
        cd fct = a[i * p + k];
        if (fct == 0.0) continue;
        for (int j = 0; j < p; ++j) {
          a[i * p + j] -= fct * a[k * p + j];
          inv[i * p + j] -= fct * inv[k * p + j];
        }
      }
    }
    double om = 2.0 * M_PI * freq_hz[f];
    for (int i = 0; i < p * p; ++i) {
      R_out[(size_t)f * p * p + i] = inv[i].real();
      L_out[(size_t)f * p * p + i] = om > 0 ? inv[i].imag() / om : 0.0;
    }
  }
  return PFFT_OK;
}

}  // extern "C"

void pfft_ctx_free(pfft_ctx *c);

namespace {
int *option_slot(pfft_ctx *c, const std::string &name) {
  if (name == "fft_plan") return &c->plans.fft;
  if (name == "ldl_plan") return &c->plans.ldl;
  if (name == "project_plan") return &c->plans.proj;
  if (name == "project_rhs") return &c->plans.proj_rhs;
  if (name == "graphs") return &c->plans.graphs;
  if (name == "stream_split") return &c->plans.stream_split;
  if (name == "factor_plan") return &c->plans.factor;
  if (name == "combine_plan") return &c->plans.comb;
  if (name == "fft_prune") return &c->plans.prune;
  if (name == "near_dense") return &c->plans.near_dense;
  if (name == "nd_plan") return &c->plans.nd;
  return nullptr;
}
void sync_plans(pfft_ctx *c) {
  c->gm.fft_plan = c->plans.fft;
  c->gm.proj_plan = c->plans.proj;
  c->gm.proj_rhs = c->plans.proj_rhs;
  c->gm.prune = c->plans.prune;
  c->cm.comb_plan = c->plans.comb;
  c->cm.near_dense = c->plans.near_dense;
}
}  // namespace

extern "C" pfft_status pfft_set_option(pfft_ctx *c, const char *name, int64_t value) {
  if (!c || !name) {
    set_error("pfft_set_option: bad argument");
    return PFFT_EINVAL;
  }
  // the learned correction's convergence judge, parts per million of the
  // per-step residual factor (0 disables it)
  if (std::string(name) == "learned_judge_ppm") {
    if (value < 0 || value >= 1000000) {
      set_error("pfft_set_option: learned_judge_ppm must lie in [0, 1e6)");
      return PFFT_EINVAL;
    }
    learned_set_judge(c, (double)value * 1e-6);
    return PFFT_OK;
  }
  int *slot = option_slot(c, name);
  if (!slot || value < 0 || value > 1) {
    set_error(std::string("pfft_set_option: unknown option or value: ") + name);
    return PFFT_EINVAL;
  }
  *slot = (int)value;
  sync_plans(c);
  return PFFT_OK;
}

extern "C" pfft_status pfft_get_option(pfft_ctx *c, const char *name, int64_t *value) {
  if (!c || !name || !value) {
    set_error("pfft_get_option: bad argument");
    return PFFT_EINVAL;
  }
  // read-only: the near-field tile shape chosen at setup (0 when the gather
  // kernel runs)
  if (std::string(name) == "combine_tile_rows") {
    *value = c->cm.ctile > 0 ? c->cm.ctr : 0;
    return PFFT_OK;
  }
  if (std::string(name) == "combine_tile_rhs") {
    *value = c->cm.ctile > 0 ? c->cm.crc : 0;
    return PFFT_OK;
  }
  // read-only: whether the preconditioner built so far uses nested
  // dissection (-1 before the first preconditioned product or solve)
  if (std::string(name) == "precond_nd") {
    *value = precond_uses_nd(c);
    return PFFT_OK;
  }
  if (std::string(name) == "learned_judge_ppm") {
    *value = (int64_t)std::llround(learned_judge_factor(c) * 1e6);
    return PFFT_OK;
  }
  int *slot = option_slot(c, name);
  if (!slot) {
    set_error(std::string("pfft_get_option: unknown option: ") + name);
    return PFFT_EINVAL;
  }
  *value = *slot;
  return PFFT_OK;
}

// Times the preconditioned loop-space product (the FGMRES step) for each
// value of each plan option in turn on device-resident synthetic vectors,
// keeps the fastest value of each, and writes a JSON report.
extern "C" pfft_status pfft_autotune(pfft_ctx *c, int32_t nrhs, const double *omega, int32_t reps,
                                     char *report, int64_t cap, void *hip_stream) {
  if (!c || nrhs <= 0 || !omega || reps <= 0) {
    set_error("pfft_autotune: bad argument");
    return PFFT_EINVAL;
  }
  double2 *x = nullptr, *y = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  try {
    hip_ok(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t n = (size_t)nrhs * c->m.l;
    hip_ok(hipMalloc(&x, n * sizeof(double2)), "hipMalloc autotune x");
    hip_ok(hipMalloc(&y, n * sizeof(double2)), "hipMalloc autotune y");
    {  // deterministic non-trivial input (x_i = (sin i, cos 2i))
      std::vector<double2> h(n);
      for (size_t i = 0; i < n; ++i) h[i] = make_double2(std::sin(0.37 * (double)i), std::cos(0.71 * (double)i));
      hip_ok(hipMemcpy(x, h.data(), n * sizeof(double2), hipMemcpyHostToDevice), "autotune x");
    }
    hip_ok(hipEventCreate(&e0), "event");
    hip_ok(hipEventCreate(&e1), "event");
    auto time_step = [&]() {
      pfft_status s0 = pfft_internal_precond_matvec(c, nrhs, omega, PFFT_PRECOND, x, y, st);
      if (s0 != PFFT_OK) throw DeviceError{s0, "autotune product"};
      std::vector<float> t(reps);
      for (int k = 0; k < reps; ++k) {
        hip_ok(hipEventRecord(e0, st), "event");
        pfft_internal_precond_matvec(c, nrhs, omega, PFFT_PRECOND, x, y, st);
        hip_ok(hipEventRecord(e1, st), "event");
        hip_ok(hipEventSynchronize(e1), "event sync");
        hip_ok(hipEventElapsedTime(&t[k], e0, e1), "event time");
      }
      std::sort(t.begin(), t.end());
      return (double)t[reps / 2];
    };
    std::string js = "{";
    const char *names[7] = {"fft_plan", "ldl_plan", "project_plan", "project_rhs", "combine_plan", "stream_split",
                            "near_dense"};
    for (int o = 0; o < 7; ++o) {
      int *slot = option_slot(c, names[o]);
      double best = 1e300;
      int arg = *slot;
      js += std::string(o ? ", " : "") + "\"" + names[o] + "\": {";
      for (int v = 0; v <= 1; ++v) {
        *slot = v;
        sync_plans(c);
        const double ms = time_step();
        js += (v ? ", " : "") + std::string("\"") + std::to_string(v) + "\": " + std::to_string(ms);
        if (ms < best) {
          best = ms;
          arg = v;
        }
      }
      *slot = arg;
      sync_plans(c);
      js += ", \"chosen\": " + std::to_string(arg) + "}";
    }
    js += "}";
    // the trials sized workspaces for every plan (the unfused FFT passes'
    // buffer, a second stream's workspace); the chosen plans allocate their
    // own at the next product
    hip_ok(hipStreamSynchronize(st), "autotune sync");
    c->release_workspaces();
    if (report && cap > 0) {
      const size_t k = std::min<size_t>((size_t)cap - 1, js.size());
      memcpy(report, js.data(), k);
      report[k] = 0;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(x);
    hipFree(y);
    return PFFT_OK;
  } catch (const DeviceError &e) {
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (x) hipFree(x);
    if (y) hipFree(y);
    set_error("pfft_autotune: " + e.msg);
    return (pfft_status)e.code;
  } catch (const SetupError &e) {
    if (x) hipFree(x);
    if (y) hipFree(y);
    set_error("pfft_autotune: " + e.msg);
    return (pfft_status)e.code;
  }
}

extern "C" void pfft_destroy(pfft_ctx *c) {
  if (!c) return;
  pfft_ctx_free(c);
}
