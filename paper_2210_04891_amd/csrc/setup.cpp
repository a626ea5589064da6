// Host setup of the pFFT loop-analysis model (FP64).
//
//  * topology and modified RWG basis            -- Sec. II-C, Eqs. RWG, ExpandJ
//  * circuit graph, BFS spanning forest, links  -- Sec. II-D Table I, Sec. III
//  * Gram blocks of the basis                   -- second term of Eq. Zb
//  * grid, stencils, projection moments         -- Sec. IV-B step 1
//  * near pairs, direct integrals, grid blocks  -- Sec. IV-B step 4, Eq. Lb
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <numeric>
#include <unordered_map>

#include "model.h"

namespace pfft {

static void fail(int code, const std::string &msg) { throw SetupError{code, msg}; }

static double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static inline void sub3(const double *a, const double *b, double *c) {
  c[0] = a[0] - b[0]; c[1] = a[1] - b[1]; c[2] = a[2] - b[2];
}
static inline double dot3(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static inline void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// ---------------------------------------------------------------------------
// mesh topology
// ---------------------------------------------------------------------------
static void build_topology(HostModel &m) {
  const int n = m.n;
  m.area.resize(n);
  m.cen.resize(3 * n);
  for (int t = 0; t < n; ++t) {
    const double *p0 = &m.V[3 * m.T[3 * t]], *p1 = &m.V[3 * m.T[3 * t + 1]], *p2 = &m.V[3 * m.T[3 * t + 2]];
    double e1[3], e2[3], c[3];
    sub3(p1, p0, e1);
    sub3(p2, p0, e2);
    cross3(e1, e2, c);
    m.area[t] = 0.5 * std::sqrt(dot3(c, c));
    if (!(m.area[t] > 0.0)) fail(-2, "degenerate triangle " + std::to_string(t));
    for (int d = 0; d < 3; ++d) m.cen[3 * t + d] = (p0[d] + p1[d] + p2[d]) / 3.0;
  }
  struct Half { int64_t key; int t, i; };
  std::vector<Half> hs(3 * (size_t)n);
  for (int t = 0; t < n; ++t)
    for (int i = 0; i < 3; ++i) {
      int a = m.T[3 * t + (i + 1) % 3], b = m.T[3 * t + (i + 2) % 3];
      if (a == b) fail(-2, "degenerate triangle " + std::to_string(t));
      int lo = std::min(a, b), hi = std::max(a, b);
      hs[3 * t + i] = Half{(int64_t)lo * m.nv + hi, t, i};
    }
  std::sort(hs.begin(), hs.end(), [](const Half &x, const Half &y) {
    return x.key != y.key ? x.key < y.key : x.t < y.t;
  });
  m.tri_edge.assign(3 * n, -1);
  m.tri_sign.assign(3 * n, 0);
  m.tplus.clear();
  m.tminus.clear();
  size_t k = 0;
  while (k < hs.size()) {
    size_t j = k;
    while (j < hs.size() && hs[j].key == hs[k].key) ++j;
    if (j - k != 2) fail(-2, "edge shared by " + std::to_string(j - k) + " triangles (mesh must be a closed 2-manifold)");
    int e = (int)m.tplus.size();
    m.tplus.push_back(hs[k].t);
    m.tminus.push_back(hs[k + 1].t);
    m.tri_edge[3 * hs[k].t + hs[k].i] = e;
    m.tri_sign[3 * hs[k].t + hs[k].i] = 1;
    m.tri_edge[3 * hs[k + 1].t + hs[k + 1].i] = e;
    m.tri_sign[3 * hs[k + 1].t + hs[k + 1].i] = -1;
    k = j;
  }
  m.b = (int)m.tplus.size();
  m.pl.resize(9 * (size_t)n);
  for (int t = 0; t < n; ++t)
    for (int i = 0; i < 3; ++i)
      for (int d = 0; d < 3; ++d) m.pl[9 * t + 3 * i + d] = m.V[3 * m.T[3 * t + i] + d] - m.cen[3 * t + d];
}

// ---------------------------------------------------------------------------
// circuit graph, spanning forest, loops (Sec. III)
// ---------------------------------------------------------------------------
static void build_circuit(HostModel &m, int nport, const int *src_off, const int *src_tri,
                          const int *snk_off, const int *snk_tri) {
  const int n = m.n;
  std::vector<int> rep(n);
  std::iota(rep.begin(), rep.end(), 0);
  std::vector<int> owner(n, -1);
  std::vector<std::vector<int>> sets;
  std::vector<int> port_src(nport), port_snk(nport);
  m.contact.assign(n, 0);
  for (int k = 0; k < nport; ++k) {
    for (int side = 0; side < 2; ++side) {
      const int *off = side == 0 ? src_off : snk_off;
      const int *tri = side == 0 ? src_tri : snk_tri;
      std::vector<int> S(tri + off[k], tri + off[k + 1]);
      if (S.empty()) fail(-1, "port " + std::to_string(k) + ": empty contact set");
      for (int t : S)
        if (t < 0 || t >= n) fail(-1, "port triangle id out of range");
      std::sort(S.begin(), S.end());
      S.erase(std::unique(S.begin(), S.end()), S.end());
      int sid = -1;
      for (size_t q = 0; q < sets.size(); ++q)
        if (sets[q] == S) sid = (int)q;
      if (sid < 0) {
        for (int t : S)
          if (owner[t] >= 0) fail(-2, "overlapping contact sets");
        sid = (int)sets.size();
        sets.push_back(S);
        for (int t : S) { owner[t] = sid; rep[t] = S[0]; m.contact[t] = 1; }
      }
      (side == 0 ? port_src : port_snk)[k] = S[0];
    }
  }
  // compact node ids, increasing with the representative triangle id
  std::vector<int> idx(n, -1);
  int nn = 0;
  for (int t = 0; t < n; ++t)
    if (rep[t] == t) idx[t] = nn++;
  m.nn = nn;
  m.node_of_tri.resize(n);
  for (int t = 0; t < n; ++t) m.node_of_tri[t] = idx[rep[t]];
  const int b = m.b;
  m.p = nport;
  m.bu.resize(b + nport);
  m.bv.resize(b + nport);
  for (int e = 0; e < b; ++e) {
    m.bu[e] = m.node_of_tri[m.tplus[e]];
    m.bv[e] = m.node_of_tri[m.tminus[e]];
  }
  for (int k = 0; k < nport; ++k) {
    m.bu[b + k] = idx[port_snk[k]];
    m.bv[b + k] = idx[port_src[k]];
  }
  // adjacency over mesh branches that are not self-loops, sorted (neighbour, branch)
  std::vector<int> deg(nn + 1, 0);
  for (int e = 0; e < b; ++e)
    if (m.bu[e] != m.bv[e]) { deg[m.bu[e] + 1]++; deg[m.bv[e] + 1]++; }
  for (int i = 0; i < nn; ++i) deg[i + 1] += deg[i];
  std::vector<std::pair<int, int>> adj(deg[nn]);
  std::vector<int> fill(deg.begin(), deg.end() - 1);
  for (int e = 0; e < b; ++e) {
    int u = m.bu[e], v = m.bv[e];
    if (u == v) continue;
    adj[fill[u]++] = {v, e};
    adj[fill[v]++] = {u, e};
  }
  for (int i = 0; i < nn; ++i) std::sort(adj.begin() + deg[i], adj.begin() + deg[i + 1]);
  m.parent.assign(nn, -2);
  m.parent_branch.assign(nn, -1);
  std::vector<int> comp(nn, -1);
  m.twig.assign(b + nport, 0);
  int ncomp = 0;
  std::vector<int> roots;
  std::deque<int> dq;
  for (int r = 0; r < nn; ++r) {
    if (comp[r] >= 0) continue;
    comp[r] = ncomp;
    m.parent[r] = -1;
    roots.push_back(r);
    dq.push_back(r);
    while (!dq.empty()) {
      int x = dq.front();
      dq.pop_front();
      for (int q = deg[x]; q < deg[x + 1]; ++q) {
        int y = adj[q].first, e = adj[q].second;
        if (comp[y] < 0) {
          comp[y] = ncomp;
          m.parent[y] = x;
          m.parent_branch[y] = e;
          m.twig[e] = 1;
          dq.push_back(y);
        }
      }
    }
    ++ncomp;
  }
  m.s = ncomp;
  for (int k = 0; k < nport; ++k)
    if (comp[m.bu[b + k]] != comp[m.bv[b + k]])
      fail(-2, "port " + std::to_string(k) + ": source and sink on different conductors");
  m.links.clear();
  for (int e = 0; e < b + nport; ++e)
    if (!m.twig[e]) m.links.push_back(e);
  m.l = (int)m.links.size();
  m.port_loop.assign(nport, -1);
  for (int i = 0; i < m.l; ++i)
    if (m.links[i] >= b) m.port_loop[m.links[i] - b] = i;
  // depth-first preorder of the forest (children in increasing node order)
  std::vector<int> cdeg(nn + 1, 0);
  for (int y = 0; y < nn; ++y)
    if (m.parent[y] >= 0) cdeg[m.parent[y] + 1]++;
  for (int i = 0; i < nn; ++i) cdeg[i + 1] += cdeg[i];
  std::vector<int> child(cdeg[nn]);
  std::vector<int> cf(cdeg.begin(), cdeg.end() - 1);
  for (int y = 0; y < nn; ++y)
    if (m.parent[y] >= 0) child[cf[m.parent[y]]++] = y;
  m.pre.assign(nn, -1);
  m.sub.assign(nn, 1);
  m.order.clear();
  m.order.reserve(nn);
  std::vector<std::pair<int, int>> st;
  for (int r : roots) {
    st.push_back({r, cdeg[r]});
    m.pre[r] = (int)m.order.size();
    m.order.push_back(r);
    while (!st.empty()) {
      auto &top = st.back();
      int x = top.first;
      if (top.second < cdeg[x + 1]) {
        int y = child[top.second++];
        m.pre[y] = (int)m.order.size();
        m.order.push_back(y);
        st.push_back({y, cdeg[y]});
      } else {
        m.sub[x] = (int)m.order.size() - m.pre[x];
        st.pop_back();
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Gram blocks: int_t (r - a).(r - b) dS = A[(c-a).(c-b) + sum_k |v_k - c|^2 / 12]
// ---------------------------------------------------------------------------
static void build_gram(HostModel &m, int contact_zs) {
  const int n = m.n, b = m.b;
  m.gram.resize(9 * (size_t)n);
  for (int t = 0; t < n; ++t) {
    const double *pl = &m.pl[9 * t];
    double spread = (dot3(pl, pl) + dot3(pl + 3, pl + 3) + dot3(pl + 6, pl + 6)) / 12.0;
    double A = m.area[t];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double raw = A * (dot3(pl + 3 * i, pl + 3 * j) + spread);
        m.gram[9 * t + 3 * i + j] = raw * m.tri_sign[3 * t + i] * m.tri_sign[3 * t + j] / (4.0 * A * A);
      }
  }
  m.gram_col.assign(5 * (size_t)b, 0);
  m.gram_val.assign(5 * (size_t)b, 0.0);
  for (int e = 0; e < b; ++e) {
    int cnt = 0;
    int *cols = &m.gram_col[5 * e];
    double *vals = &m.gram_val[5 * e];
    auto add = [&](int col, double v) {
      for (int q = 0; q < cnt; ++q)
        if (cols[q] == col) { vals[q] += v; return; }
      cols[cnt] = col;
      vals[cnt++] = v;
    };
    for (int side = 0; side < 2; ++side) {
      int t = side == 0 ? m.tplus[e] : m.tminus[e];
      double w = (m.contact[t] && !contact_zs) ? 0.0 : 1.0;
      int i = 0;
      while (m.tri_edge[3 * t + i] != e) ++i;
      for (int j = 0; j < 3; ++j) add(m.tri_edge[3 * t + j], w * m.gram[9 * t + 3 * i + j]);
    }
    for (int q = cnt; q < 5; ++q) { cols[q] = e; vals[q] = 0.0; }
  }
}

// ---------------------------------------------------------------------------
// grid and projection moments (Sec. IV-B step 1)
// ---------------------------------------------------------------------------
static const double D7_L[7][3] = {
    {1.0 / 3, 1.0 / 3, 1.0 / 3},
    {0.059715871789770, 0.470142064105115, 0.470142064105115},
    {0.470142064105115, 0.059715871789770, 0.470142064105115},
    {0.470142064105115, 0.470142064105115, 0.059715871789770},
    {0.797426985353087, 0.101286507323456, 0.101286507323456},
    {0.101286507323456, 0.797426985353087, 0.101286507323456},
    {0.101286507323456, 0.101286507323456, 0.797426985353087}};
static const double D7_W[7] = {0.225, 0.132394152788506, 0.132394152788506, 0.132394152788506,
                               0.125939180544827, 0.125939180544827, 0.125939180544827};

static void lagrange4(double x, double L[4]) {
  // nodes 0, 1, 2, 3
  L[0] = -(x - 1) * (x - 2) * (x - 3) / 6.0;
  L[1] = x * (x - 2) * (x - 3) / 2.0;
  L[2] = -x * (x - 1) * (x - 3) / 2.0;
  L[3] = x * (x - 1) * (x - 2) / 6.0;
}

static void build_grid(HostModel &m, const SetupOptions &opt) {
  if (opt.stencil != 4) fail(-1, "only stencil order 4 is supported");
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int v = 0; v < m.nv; ++v)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], m.V[3 * v + d]);
      hi[d] = std::max(hi[d], m.V[3 * v + d]);
    }
  double hmax = 0;
  for (int d = 0; d < 3; ++d) {
    m.dims[d] = opt.grid[d];
    if (m.dims[d] < 8 || m.dims[d] > 512) fail(-1, "grid dimension out of range [8, 512]");
    if ((m.dims[d] & (m.dims[d] - 1)) != 0) fail(-1, "grid dimensions must be powers of two");
    double ext = hi[d] - lo[d];
    m.h[d] = ext > 0 ? ext / (m.dims[d] - opt.stencil) : 0.0;
    hmax = std::max(hmax, m.h[d]);
  }
  for (int d = 0; d < 3; ++d) {
    if (m.h[d] <= 0) m.h[d] = hmax;
    m.x0[d] = lo[d] - 0.5 * (opt.stencil - 1) * m.h[d];
  }
  const int n = m.n;
  m.anchor.resize(3 * (size_t)n);
  m.M0.assign(64 * (size_t)n, 0.0);
  m.M1.assign(192 * (size_t)n, 0.0);
#pragma omp parallel for schedule(static)
  for (int t = 0; t < n; ++t) {
    int a[3];
    for (int d = 0; d < 3; ++d) {
      int ai = (int)std::floor((m.cen[3 * t + d] - m.x0[d]) / m.h[d]) - 1;
      a[d] = std::min(std::max(ai, 0), m.dims[d] - 4);
      m.anchor[3 * t + d] = a[d];
    }
    const double *P[3] = {&m.V[3 * m.T[3 * t]], &m.V[3 * m.T[3 * t + 1]], &m.V[3 * m.T[3 * t + 2]]};
    for (int q = 0; q < 7; ++q) {
      double r[3], L[3][4];
      for (int d = 0; d < 3; ++d) {
        r[d] = D7_L[q][0] * P[0][d] + D7_L[q][1] * P[1][d] + D7_L[q][2] * P[2][d];
        lagrange4((r[d] - m.x0[d]) / m.h[d] - a[d], L[d]);
      }
      double wq = D7_W[q] * m.area[t];
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
          for (int k = 0; k < 4; ++k) {
            int g = (i * 4 + j) * 4 + k;
            double W = wq * L[0][i] * L[1][j] * L[2][k];
            m.M0[64 * (size_t)t + g] += W;
            for (int c = 0; c < 3; ++c) m.M1[192 * (size_t)t + 3 * g + c] += W * (r[c] - m.cen[3 * t + c]);
          }
    }
  }
}

// ---------------------------------------------------------------------------
// near pairs, exact minus grid blocks, edge-level CSR (Sec. IV-B step 4)
// ---------------------------------------------------------------------------
static void build_nearfield(HostModel &m, const SetupOptions &opt) {
  const double tl0 = now_ms();
  const int n = m.n;
  const double hmax = std::max(m.h[0], std::max(m.h[1], m.h[2]));
  const double rad = opt.kappa * 3.0 * hmax;
  const double rbox = std::sqrt(16.0 * (m.h[0] * m.h[0] + m.h[1] * m.h[1] + m.h[2] * m.h[2]));
  const double cell = std::max(rad, rbox) * (1 + 1e-12);
  // cell lists over centroids
  double lo[3] = {1e300, 1e300, 1e300};
  for (int t = 0; t < n; ++t)
    for (int d = 0; d < 3; ++d) lo[d] = std::min(lo[d], m.cen[3 * t + d]);
  std::vector<std::array<int64_t, 3>> cidx(n);
  std::unordered_map<int64_t, std::vector<int>> cells;
  auto ckey = [](int64_t a, int64_t b, int64_t c) { return (a * 2097152 + b) * 2097152 + c; };
  for (int t = 0; t < n; ++t) {
    for (int d = 0; d < 3; ++d) cidx[t][d] = (int64_t)std::floor((m.cen[3 * t + d] - lo[d]) / cell);
    cells[ckey(cidx[t][0], cidx[t][1], cidx[t][2])].push_back(t);
  }
  // triangles around each vertex: a pair that shares a vertex is always near
  // (its singular entries are computed directly), whatever the grid spacing
  const int nvert = (int)(m.V.size() / 3);
  std::vector<int> vt_off(nvert + 1, 0), vt_tri(3 * (size_t)n);
  for (int k = 0; k < 3 * n; ++k) vt_off[m.T[k] + 1]++;
  for (int v = 0; v < nvert; ++v) vt_off[v + 1] += vt_off[v];
  {
    std::vector<int> fill(vt_off.begin(), vt_off.end() - 1);
    for (int k = 0; k < 3 * n; ++k) vt_tri[fill[m.T[k]]++] = k / 3;
  }
  std::vector<std::vector<int>> nb(n);
#pragma omp parallel for schedule(dynamic, 256)
  for (int t = 0; t < n; ++t) {
    auto &out = nb[t];
    for (int i = 0; i < 3; ++i) {
      const int v = m.T[3 * t + i];
      for (int k = vt_off[v]; k < vt_off[v + 1]; ++k) out.push_back(vt_tri[k]);
    }
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          auto it = cells.find(ckey(cidx[t][0] + dx, cidx[t][1] + dy, cidx[t][2] + dz));
          if (it == cells.end()) continue;
          for (int u : it->second) {
            bool box = true;
            for (int d = 0; d < 3; ++d) box = box && std::abs(m.anchor[3 * t + d] - m.anchor[3 * u + d]) <= 3;
            double dd[3];
            sub3(&m.cen[3 * t], &m.cen[3 * u], dd);
            double dist = std::sqrt(dot3(dd, dd));
            if (box || dist < rad || u == t) out.push_back(u);
          }
        }
    std::sort(out.begin(), out.end());
    out.erase(std::unique(out.begin(), out.end()), out.end());
  }
  m.near_off.assign(n + 1, 0);
  for (int t = 0; t < n; ++t) m.near_off[t + 1] = m.near_off[t] + (int)nb[t].size();
  m.near_tri.resize(m.near_off[n]);
  for (int t = 0; t < n; ++t) std::copy(nb[t].begin(), nb[t].end(), m.near_tri.begin() + m.near_off[t]);
  // unordered pairs t <= u and their (exact - grid) blocks
  std::vector<int64_t> poff(n + 1, 0);
  for (int t = 0; t < n; ++t) {
    int c = 0;
    for (int q = m.near_off[t]; q < m.near_off[t + 1]; ++q) c += m.near_tri[q] >= t;
    poff[t + 1] = poff[t] + c;
  }
  m.npairs = poff[n];
  const double tl1 = now_ms();
  std::vector<double> blk(9 * (size_t)m.npairs);   // scaled (exact - grid)
  // grid Green's function table over offsets within [-Dmax, Dmax]^3
  int Dm[3] = {0, 0, 0};
  for (int t = 0; t < n; ++t)
    for (int q = m.near_off[t]; q < m.near_off[t + 1]; ++q) {
      int u = m.near_tri[q];
      for (int d = 0; d < 3; ++d) Dm[d] = std::max(Dm[d], std::abs(m.anchor[3 * t + d] - m.anchor[3 * u + d]) + 3);
    }
  int S[3] = {2 * Dm[0] + 1, 2 * Dm[1] + 1, 2 * Dm[2] + 1};
  std::vector<double> Htab((size_t)S[0] * S[1] * S[2]);
  for (int i = 0; i < S[0]; ++i)
    for (int j = 0; j < S[1]; ++j)
      for (int k = 0; k < S[2]; ++k) {
        double x = (i - Dm[0]) * m.h[0], y = (j - Dm[1]) * m.h[1], z = (k - Dm[2]) * m.h[2];
        double R = std::sqrt(x * x + y * y + z * z);
        Htab[((size_t)i * S[1] + j) * S[2] + k] = R > 0 ? 1.0 / R : 0.0;
      }
  std::vector<double> radius(n);
  for (int t = 0; t < n; ++t) {
    double r = 0;
    for (int i = 0; i < 3; ++i) r = std::max(r, std::sqrt(dot3(&m.pl[9 * t + 3 * i], &m.pl[9 * t + 3 * i])));
    radius[t] = r;
  }
  // the pairs sorted by the outer rule their proximity asks for (class 0:
  // the pair shares a vertex; 1, 2, 3: separated, with the rule on 64, 16
  // or 4 sub-triangles of t as the gap shrinks relative to the triangles)
  NearPairList pl;
  {
    std::vector<int8_t> cls(m.npairs);
#pragma omp parallel for schedule(dynamic, 256)
    for (int t = 0; t < n; ++t) {
      int64_t pk = poff[t];
      for (int q = m.near_off[t]; q < m.near_off[t + 1]; ++q) {
        const int u = m.near_tri[q];
        if (u < t) continue;
        int shared = 0;
        for (int a = 0; a < 3; ++a)
          for (int c = 0; c < 3; ++c) shared += m.T[3 * t + a] == m.T[3 * u + c];
        double dd[3];
        sub3(&m.cen[3 * t], &m.cen[3 * u], dd);
        const double ratio = (std::sqrt(dot3(dd, dd)) - radius[t] - radius[u]) / std::max(radius[t], radius[u]);
        cls[pk++] = shared > 0 ? 0 : (ratio < 0.5 ? 1 : (ratio < 2.0 ? 2 : 3));
      }
    }
    int64_t cnt[4] = {0, 0, 0, 0};
    for (int64_t k = 0; k < m.npairs; ++k) cnt[cls[k]]++;
    int64_t pos[4] = {0, cnt[0], cnt[0] + cnt[1], cnt[0] + cnt[1] + cnt[2]};
    for (int c = 0; c < 4; ++c) pl.cls_end[c] = pos[c] + cnt[c];
    pl.t.resize(m.npairs);
    pl.u.resize(m.npairs);
    pl.idx.resize(m.npairs);
    for (int t = 0; t < n; ++t) {
      int64_t pk = poff[t];
      for (int q = m.near_off[t]; q < m.near_off[t + 1]; ++q) {
        const int u = m.near_tri[q];
        if (u < t) continue;
        const int64_t r = pos[cls[pk]]++;
        pl.t[r] = t;
        pl.u[r] = u;
        pl.idx[r] = pk++;
      }
    }
  }
  const int64_t ntouch = pl.cls_end[0];
  std::vector<double> exb(9 * (size_t)ntouch);     // scaled direct blocks of the touching pairs
  near_pair_blocks(m, pl, Htab, Dm, S, opt.device_blocks != 0, opt.stream, blk.data(), exb.data());
  // unordered pair -> its row in exb (touching pairs only)
  std::vector<int> touch_row(m.npairs, -1);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < ntouch; ++r) touch_row[pl.idx[r]] = (int)r;
  pl = NearPairList();
  const double tl2 = now_ms();
  // ordered entry q of t's list -> unordered block index and transpose flag
  std::vector<int64_t> qblk(m.near_tri.size());
  std::vector<uint8_t> qtr(m.near_tri.size());
#pragma omp parallel for schedule(static)
  for (int t = 0; t < n; ++t) {
    const int *beg = &m.near_tri[m.near_off[t]], *end = &m.near_tri[m.near_off[t + 1]];
    int64_t lb_t = std::lower_bound(beg, end, t) - beg;
    for (int q = m.near_off[t]; q < m.near_off[t + 1]; ++q) {
      int u = m.near_tri[q];
      if (u >= t) {
        qblk[q] = poff[t] + (q - m.near_off[t] - lb_t);
        qtr[q] = 0;
      } else {
        const int *ub = &m.near_tri[m.near_off[u]], *ue = &m.near_tri[m.near_off[u + 1]];
        int64_t pos_t = std::lower_bound(ub, ue, t) - ub;
        int64_t pos_u = std::lower_bound(ub, ue, u) - ub;
        qblk[q] = poff[u] + (pos_t - pos_u);
        qtr[q] = 1;
      }
    }
  }
  // (touching pairs are in every near list by construction; a miss is
  // reported after the parallel loop, never thrown inside it)
  int missing = 0;
  auto find_q = [&](int t, int u) -> int {
    const int *beg = &m.near_tri[m.near_off[t]], *end = &m.near_tri[m.near_off[t + 1]];
    const int *it = std::lower_bound(beg, end, u);
    if (it == end || *it != u) {
#pragma omp atomic write
      missing = 1;
      return -1;
    }
    return (int)(m.near_off[t] + (it - beg));
  };
  // diagonal of the exact K (for Z_b^N = diag(Z_b)): the two triangles of e
  // and both cross terms, all of them near pairs
  const int b = m.b;
  m.kdiag.assign(b, 0.0);
#pragma omp parallel for schedule(static)
  for (int e = 0; e < b; ++e) {
    int ts[2] = {m.tplus[e], m.tminus[e]};
    double acc = 0;
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 2; ++c) {
        int t = ts[a], u = ts[c];
        int q = find_q(t, u);
        if (q < 0) continue;
        int i = 0, j = 0;
        while (m.tri_edge[3 * t + i] != e) ++i;
        while (m.tri_edge[3 * u + j] != e) ++j;
        const int tr = touch_row[qblk[q]];
        if (tr < 0) {
#pragma omp atomic write
          missing = 1;
          continue;
        }
        const double *B = &exb[9 * (size_t)tr];
        acc += qtr[q] ? B[3 * j + i] : B[3 * i + j];
      }
    m.kdiag[e] = acc;
  }
  if (missing) fail(-4, "internal: touching pair missing from near list");
  // edge-level CSR: row e gathers the blocks of (t, u), t in {T+, T-}, u near t
  m.nf_rowptr.assign(b + 1, 0);
  std::vector<std::vector<int>> rcol(b);
  std::vector<std::vector<double>> rval(b);
#pragma omp parallel for schedule(dynamic, 64)
  for (int e = 0; e < b; ++e) {
    std::vector<std::pair<int, double>> acc;
    for (int side = 0; side < 2; ++side) {
      int t = side == 0 ? m.tplus[e] : m.tminus[e];
      int i = 0;
      while (m.tri_edge[3 * t + i] != e) ++i;
      for (int q = m.near_off[t]; q < m.near_off[t + 1]; ++q) {
        int u = m.near_tri[q];
        const double *B = &blk[9 * qblk[q]];
        bool tr = qtr[q];
        for (int j = 0; j < 3; ++j) acc.push_back({m.tri_edge[3 * u + j], tr ? B[3 * j + i] : B[3 * i + j]});
      }
    }
    std::sort(acc.begin(), acc.end(), [](const std::pair<int, double> &a, const std::pair<int, double> &c) {
      return a.first < c.first;
    });
    auto &cs = rcol[e];
    auto &vs = rval[e];
    for (auto &pr : acc) {
      if (!cs.empty() && cs.back() == pr.first)
        vs.back() += pr.second;
      else {
        cs.push_back(pr.first);
        vs.push_back(pr.second);
      }
    }
  }
  for (int e = 0; e < b; ++e) m.nf_rowptr[e + 1] = m.nf_rowptr[e] + (int64_t)rcol[e].size();
  m.nf_col.resize(m.nf_rowptr[b]);
  m.nf_val.resize(m.nf_rowptr[b]);
#pragma omp parallel for schedule(static)
  for (int e = 0; e < b; ++e) {
    std::copy(rcol[e].begin(), rcol[e].end(), m.nf_col.begin() + m.nf_rowptr[e]);
    std::copy(rval[e].begin(), rval[e].end(), m.nf_val.begin() + m.nf_rowptr[e]);
  }
  m.setup_ms[4] = tl1 - tl0;
  m.setup_ms[5] = tl2 - tl1;
  m.setup_ms[6] = now_ms() - tl2;
}

void build_model(HostModel &m, const double *V, int nv, const int *T, int n, int nport,
                 const int *src_off, const int *src_tri, const int *snk_off, const int *snk_tri,
                 const SetupOptions &opt) {
  if (nv <= 0 || n <= 0 || !V || !T) fail(-1, "empty mesh");
  if (nport < 0) fail(-1, "negative port count");
  if (nport > 0 && (!src_off || !src_tri || !snk_off || !snk_tri)) fail(-1, "null port arrays");
  m.nv = nv;
  m.n = n;
  m.V.assign(V, V + 3 * (size_t)nv);
  m.T.assign(T, T + 3 * (size_t)n);
  for (int k = 0; k < 3 * n; ++k)
    if (m.T[k] < 0 || m.T[k] >= nv) fail(-1, "vertex id out of range");
  auto t0 = now_ms();
  build_topology(m);
  auto t1 = now_ms();
  build_circuit(m, nport, src_off, src_tri, snk_off, snk_tri);
  auto t2 = now_ms();
  build_gram(m, opt.contact_zs);
  auto t3 = now_ms();
  build_grid(m, opt);
  auto t4 = now_ms();
  build_nearfield(m, opt);
  m.setup_ms[0] = t1 - t0;
  m.setup_ms[1] = t2 - t1;
  m.setup_ms[2] = t3 - t2;
  m.setup_ms[3] = t4 - t3;
}

}  // namespace pfft
