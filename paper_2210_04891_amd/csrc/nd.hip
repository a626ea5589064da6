// Nested-dissection ordering and supernodal (multifrontal) LDL^T of the
// nodal matrix L_w = N D^-1 N^T that applies the preconditioner of Eq. Precond
// (Sec. IV-A).  The paper factors P with a sparse direct solver; a
// conductor of a million nodes (the PDN-like configuration) has a reverse
// Cuthill-McKee band of about 700, too wide for a band factorization, while
// a surface mesh has small geometric separators.  Host code (OpenMP); the
// solve runs on the device (precond.hip).  Host code only, built with the
// HIP sources for the vector types its header shares with them.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>
#include <vector>

#include "precond.h"

namespace pfft {

typedef std::complex<double> cd;
static constexpr double MU0 = 4e-7 * M_PI;
static constexpr int ND_LEAF = 64;   // subdomains at most this large are not split further

// One conductor: recursive bisection of the node set S at the median of its
// widest coordinate; the separator is the lower half's nodes adjacent to the
// upper half.  Appends supernodes in postorder (halves first, separator
// last) to `out` as (node list, parent placeholder) and returns the roots of
// the subtree it built.
struct NdBuild {
  const std::vector<std::vector<int>> &adj;
  const std::vector<double> &xyz;
  std::vector<int> &stamp;
  int tick = 0;
  std::vector<std::vector<int>> nodes;   // per supernode, its nodes
  std::vector<std::vector<int>> kids;    // per supernode, its children
  NdBuild(const std::vector<std::vector<int>> &a, const std::vector<double> &x, std::vector<int> &st)
      : adj(a), xyz(x), stamp(st) {}

  int leaf(std::vector<int> S) {
    nodes.push_back(std::move(S));
    kids.emplace_back();
    return (int)nodes.size() - 1;
  }
  std::vector<int> split(std::vector<int> S) {
    if (S.empty()) return {};
    if ((int)S.size() <= ND_LEAF) return {leaf(std::move(S))};
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int x : S)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], xyz[3 * x + d]);
        hi[d] = std::max(hi[d], xyz[3 * x + d]);
      }
    int ax = 0;
    for (int d = 1; d < 3; ++d)
      if (hi[d] - lo[d] > hi[ax] - lo[ax]) ax = d;
    const size_t half = S.size() / 2;
    std::nth_element(S.begin(), S.begin() + half, S.end(), [&](int a, int b) {
      const double ca = xyz[3 * a + ax], cb = xyz[3 * b + ax];
      return ca != cb ? ca < cb : a < b;
    });
    // upper half marked; separator = lower-half nodes with an upper neighbour
    const int up = ++tick;
    for (size_t i = half; i < S.size(); ++i) stamp[S[i]] = up;
    std::vector<int> A, B(S.begin() + half, S.end()), sep;
    for (size_t i = 0; i < half; ++i) {
      const int x = S[i];
      bool cut = false;
      for (int y : adj[x])
        if (stamp[y] == up) { cut = true; break; }
      (cut ? sep : A).push_back(x);
    }
    if (sep.size() * 2 > S.size()) return {leaf(std::move(S))};   // no useful separator
    std::vector<int> ra = split(std::move(A)), rb = split(std::move(B));
    if (sep.empty()) {
      ra.insert(ra.end(), rb.begin(), rb.end());
      return ra;
    }
    const int s = leaf(std::move(sep));
    kids[s] = ra;
    kids[s].insert(kids[s].end(), rb.begin(), rb.end());
    return {s};
  }
};

// Orders conductor c's non-grounded nodes `mem` (band members) and its port
// supernodes `dmem` by nested dissection: unknowns from `next` on, in
// postorder; the supernode tree goes to ps (sn_start, sn_parent; children
// and structure come later from nd_symbolic).
void nd_order_conductor(const std::vector<std::vector<int>> &adj, const std::vector<double> &xyz,
                        const std::vector<int> &mem, const std::vector<int> &dmem, std::vector<int> &stamp,
                        int &next, std::vector<int> &unk, PrecondStruct &ps) {
  NdBuild nb(adj, xyz, stamp);
  std::vector<int> roots = nb.split(mem);
  int top = -1;
  if (!dmem.empty()) {
    top = nb.leaf(dmem);
    nb.kids[top] = roots;
    roots = {top};
  }
  // postorder numbering of the supernodes and their unknowns
  std::vector<int> sid(nb.nodes.size(), -1);
  std::vector<std::pair<int, int>> st;   // (supernode, state)
  for (int r : roots) {
    st.push_back({r, 0});
    while (!st.empty()) {
      auto &[s, k] = st.back();
      if (k < (int)nb.kids[s].size()) {
        const int ch = nb.kids[s][k++];
        st.push_back({ch, 0});
        continue;
      }
      const int me = ps.nsn++;
      sid[s] = me;
      ps.sn_start.push_back(next);
      for (int x : nb.nodes[s]) unk[x] = next++;
      ps.sn_parent.push_back(-1);
      st.pop_back();
    }
  }
  for (size_t s = 0; s < nb.nodes.size(); ++s)
    for (int ch : nb.kids[s]) ps.sn_parent[sid[ch]] = sid[s];
}

// Structure of every supernode from the unknown adjacency (uadj: neighbours
// of each unknown), children lists, levels by height, front sizes and value
// offsets.  The structure of s is every neighbour of its subtree numbered
// after s: its own neighbours and its children's structures.
void nd_symbolic(const std::vector<std::vector<int>> &uadj, PrecondStruct &ps) {
  const int nsn = ps.nsn;
  ps.sn_start.push_back(ps.nu);                      // closes the last range
  ps.ch_off.assign(nsn + 1, 0);
  for (int s = 0; s < nsn; ++s)
    if (ps.sn_parent[s] >= 0) ps.ch_off[ps.sn_parent[s] + 1]++;
  for (int s = 0; s < nsn; ++s) ps.ch_off[s + 1] += ps.ch_off[s];
  ps.ch_ids.assign(ps.ch_off[nsn], 0);
  {
    std::vector<int> f(ps.ch_off.begin(), ps.ch_off.end() - 1);
    for (int s = 0; s < nsn; ++s)
      if (ps.sn_parent[s] >= 0) ps.ch_ids[f[ps.sn_parent[s]]++] = s;
  }
  // structures bottom-up (children precede parents in the numbering)
  std::vector<std::vector<int>> st(nsn);
  ps.sn_height.assign(nsn, 0);
  for (int s = 0; s < nsn; ++s) {
    const int a = ps.sn_start[s], e = ps.sn_start[s + 1];
    std::vector<int> v;
    for (int i = a; i < e; ++i)
      for (int j : uadj[i])
        if (j >= e) v.push_back(j);
    for (int q = ps.ch_off[s]; q < ps.ch_off[s + 1]; ++q) {
      const int c = ps.ch_ids[q];
      for (int j : st[c])
        if (j >= e) v.push_back(j);
      ps.sn_height[s] = std::max(ps.sn_height[s], ps.sn_height[c] + 1);
    }
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    st[s] = std::move(v);
  }
  ps.st_off.assign(nsn + 1, 0);
  for (int s = 0; s < nsn; ++s) ps.st_off[s + 1] = ps.st_off[s] + (int64_t)st[s].size();
  ps.st_ids.resize(ps.st_off[nsn]);
  ps.st_pos.assign(ps.st_off[nsn], -1);
  ps.l11_off.assign(nsn + 1, 0);
  ps.l21_off.assign(nsn + 1, 0);
  ps.max_front = 0;
  for (int s = 0; s < nsn; ++s) {
    std::copy(st[s].begin(), st[s].end(), ps.st_ids.begin() + ps.st_off[s]);
    const int64_t ns = ps.sn_start[s + 1] - ps.sn_start[s], nst = (int64_t)st[s].size();
    ps.l11_off[s + 1] = ps.l11_off[s] + ns * ns;
    ps.l21_off[s + 1] = ps.l21_off[s] + ns * nst;
    ps.max_front = std::max(ps.max_front, (int)(ns + nst));
    // positions in the parent's front: its own unknowns first, then its
    // structure (every structure row of s lies in one of the two)
    const int p = ps.sn_parent[s];
    if (p < 0) {
      if (nst) throw SetupError{-4, "internal: structure above a root supernode"};
      continue;
    }
    const int pa = ps.sn_start[p], pe = ps.sn_start[p + 1];
    for (int64_t t = 0; t < nst; ++t) {
      const int u = st[s][t];
      int pos = -1;
      if (u >= pa && u < pe) {
        pos = u - pa;
      } else {
        auto it = std::lower_bound(st[p].begin(), st[p].end(), u);
        if (it != st[p].end() && *it == u) pos = (pe - pa) + (int)(it - st[p].begin());
      }
      if (pos < 0) throw SetupError{-4, "internal: structure row missing from the parent's front"};
      ps.st_pos[ps.st_off[s] + t] = pos;
    }
  }
  int hmax = 0;
  for (int s = 0; s < nsn; ++s) hmax = std::max(hmax, ps.sn_height[s]);
  ps.lvl_off.assign(hmax + 2, 0);
  for (int s = 0; s < nsn; ++s) ps.lvl_off[ps.sn_height[s] + 1]++;
  for (int h = 0; h <= hmax; ++h) ps.lvl_off[h + 1] += ps.lvl_off[h];
  ps.lvl_sn.resize(nsn);
  ps.lvl_front.assign(hmax + 1, 0);
  {
    std::vector<int> f(ps.lvl_off.begin(), ps.lvl_off.end() - 1);
    for (int s = 0; s < nsn; ++s) {
      const int h = ps.sn_height[s];
      ps.lvl_sn[f[h]++] = s;
      const int fr = (ps.sn_start[s + 1] - ps.sn_start[s]) + (int)(ps.st_off[s + 1] - ps.st_off[s]);
      ps.lvl_front[h] = std::max(ps.lvl_front[h], fr);
    }
  }
}

// Dense LDL^T of the first ns columns of the lower-triangular front F
// (nf x nf, row-major, only j <= i used), in panels of NB columns: within a
// panel rank-1 updates of the panel's columns; then one rank-NB update of
// the rest.  F keeps L below the diagonal of those columns and their pivots
// on it; the trailing nst x nst block becomes the update matrix.
static bool front_ldl(cd *F, int nf, int ns) {
  constexpr int NB = 32;
  std::vector<cd> W((size_t)nf * NB);   // W[i][k] = L_ik d_k for the panel
  for (int k0 = 0; k0 < ns; k0 += NB) {
    const int k1 = std::min(ns, k0 + NB), nb = k1 - k0;
    for (int k = k0; k < k1; ++k) {
      const cd d = F[(size_t)k * nf + k];
      if (std::abs(d) == 0.0 || !std::isfinite(d.real()) || !std::isfinite(d.imag())) return false;
      for (int i = k + 1; i < nf; ++i) {
        const cd w = F[(size_t)i * nf + k];
        W[(size_t)i * NB + (k - k0)] = w;
        F[(size_t)i * nf + k] = w / d;
      }
      // rank-1 update restricted to the panel's later columns
      for (int i = k + 1; i < nf; ++i) {
        const cd li = F[(size_t)i * nf + k];
        cd *Fi = F + (size_t)i * nf;
        const int jm = std::min(i, k1 - 1);
        for (int j = k + 1; j <= jm; ++j) Fi[j] -= li * W[(size_t)j * NB + (k - k0)];
      }
    }
    // trailing update: F[i][j] -= sum_k L_ik (L_jk d_k), i >= j >= k1
    auto row = [&](int i) {
      cd *Fi = F + (size_t)i * nf;
      const cd *Li = F + (size_t)i * nf + k0;
      for (int j = k1; j <= i; ++j) {
        const cd *Wj = &W[(size_t)j * NB];
        cd acc = 0.0;
        for (int k = 0; k < nb; ++k) acc += Li[k] * Wj[k];
        Fi[j] -= acc;
      }
    };
    const long work = (long)(nf - k1) * (nf - k1) * nb;
    if (work > (1L << 22) && !omp_in_parallel()) {
#pragma omp parallel for schedule(dynamic, 8)
      for (int i = k1; i < nf; ++i) row(i);
    } else {
      for (int i = k1; i < nf; ++i) row(i);
    }
  }
  return true;
}

bool factor_precond_nd(const HostModel &m, const PrecondStruct &ps, double omega, double sigma, double mu_r,
                       std::vector<cd> &l11, std::vector<cd> &l11t, std::vector<cd> &l21, std::vector<cd> &diag,
                       std::vector<cd> &yinv) {
  const int b = m.b, nu = ps.nu, nsn = ps.nsn;
  const double a = std::sqrt(omega * MU0 * mu_r / (2.0 * sigma));
  const cd zs(a, a), jw(0.0, omega * MU0 * mu_r / (4.0 * M_PI));
  yinv.assign(b, 0.0);
  for (int e = 0; e < b; ++e) {
    double g = 0;
    for (int q = 0; q < 5; ++q)
      if (m.gram_col[5 * e + q] == e) g += m.gram_val[5 * e + q];
    const cd D = zs * g + jw * m.kdiag[e];
    if (std::abs(D) == 0.0) return false;
    yinv[e] = 1.0 / D;
  }
  // lower triangle of L_w by columns: entries (i, j), i >= j
  std::vector<cd> dg(nu, 0.0);
  std::vector<std::vector<std::pair<int, cd>>> low(nu);
  for (int e = 0; e < b; ++e) {
    const int ru = ps.br_ru[e], rv = ps.br_rv[e];
    if (ru == rv) continue;   // same supernode (ground included): not in L_w
    const cd y = yinv[e];
    if (ru >= 0) dg[ru] += y;
    if (rv >= 0) dg[rv] += y;
    if (ru >= 0 && rv >= 0) low[std::min(ru, rv)].push_back({std::max(ru, rv), -y});
  }
  l11.assign(ps.l11_off[nsn], 0.0);
  l11t.assign(ps.l11_off[nsn], 0.0);
  l21.assign(ps.l21_off[nsn], 0.0);
  diag.assign(nu, 0.0);
  std::vector<std::vector<cd>> upd(nsn);   // update matrices (nst x nst, row-major) until the parent takes them
  int bad = 0;
  const int nlvl = (int)ps.lvl_off.size() - 1;
  for (int h = 0; h < nlvl; ++h) {
    const int q0 = ps.lvl_off[h], q1 = ps.lvl_off[h + 1];
    auto one = [&](int s) {
      const int sa = ps.sn_start[s], ns = ps.sn_start[s + 1] - sa;
      const int64_t so = ps.st_off[s];
      const int nst = (int)(ps.st_off[s + 1] - so), nf = ns + nst;
      const int *sid = ps.st_ids.data() + so;
      std::vector<cd> F((size_t)nf * nf, 0.0);
      auto pos = [&](int u) {
        if (u < sa + ns) return u - sa;
        return ns + (int)(std::lower_bound(sid, sid + nst, u) - sid);
      };
      for (int j = sa; j < sa + ns; ++j) {
        F[(size_t)(j - sa) * nf + (j - sa)] += dg[j];
        for (auto &pr : low[j]) {
          const int pi = pos(pr.first);
          F[(size_t)pi * nf + (j - sa)] += pr.second;
        }
      }
      for (int q = ps.ch_off[s]; q < ps.ch_off[s + 1]; ++q) {
        const int c = ps.ch_ids[q];
        const int64_t co = ps.st_off[c];
        const int nc = (int)(ps.st_off[c + 1] - co);
        const int *cp = ps.st_pos.data() + co;
        const std::vector<cd> &U = upd[c];
        for (int x = 0; x < nc; ++x)
          for (int y = 0; y <= x; ++y) F[(size_t)cp[x] * nf + cp[y]] += U[(size_t)x * nc + y];
      }
      for (int q = ps.ch_off[s]; q < ps.ch_off[s + 1]; ++q) std::vector<cd>().swap(upd[ps.ch_ids[q]]);
      if (!front_ldl(F.data(), nf, ns)) {
#pragma omp atomic
        ++bad;
        return;
      }
      cd *L11 = l11.data() + ps.l11_off[s], *L11t = l11t.data() + ps.l11_off[s];
      cd *L21 = l21.data() + ps.l21_off[s];
      for (int k = 0; k < ns; ++k) {
        diag[sa + k] = F[(size_t)k * nf + k];
        L11[(size_t)k * ns + k] = 1.0;
        L11t[(size_t)k * ns + k] = 1.0;
        for (int i = k + 1; i < ns; ++i) {
          L11[(size_t)k * ns + i] = F[(size_t)i * nf + k];    // by columns
          L11t[(size_t)i * ns + k] = F[(size_t)i * nf + k];   // by rows
        }
        for (int t = 0; t < nst; ++t) L21[(size_t)k * nst + t] = F[(size_t)(ns + t) * nf + k];
      }
      if (nst) {
        std::vector<cd> U((size_t)nst * nst);
        for (int x = 0; x < nst; ++x)
          for (int y = 0; y <= x; ++y) U[(size_t)x * nst + y] = F[(size_t)(ns + x) * nf + ns + y];
        upd[s] = std::move(U);
      }
    };
    if (q1 - q0 >= 16) {
#pragma omp parallel for schedule(dynamic, 1)
      for (int q = q0; q < q1; ++q) one(ps.lvl_sn[q]);
    } else {
      for (int q = q0; q < q1; ++q) one(ps.lvl_sn[q]);
    }
    if (bad) return false;
  }
  return true;
}

std::vector<int64_t> precond_info(const HostModel &m, int nd_mode) {
  PrecondStruct ps;
  build_precond_struct(m, ps, nd_mode);
  return {ps.nu, ps.W, ps.Wc, ps.nd ? 1 : 0, ps.nsn, ps.max_front,
          ps.nd ? (int64_t)ps.lvl_off.size() - 1 : 0};
}

double nd_solve_check(const HostModel &m, double omega) {
  PrecondStruct ps;
  build_precond_struct(m, ps, 1);
  std::vector<cd> l11, l11t, l21, dg, yinv;
  if (!factor_precond_nd(m, ps, omega, 5.8e7, 1.0, l11, l11t, l21, dg, yinv)) return -1.0;
  const int nu = ps.nu;
  std::vector<cd> b(nu), x(nu);
  for (int i = 0; i < nu; ++i) b[i] = cd(std::sin(0.37 * i + 0.1), std::cos(1.3 * i));
  x = b;
  std::vector<cd> u(ps.st_off[ps.nsn], 0.0);
  const int nlvl = (int)ps.lvl_off.size() - 1;
  for (int h = 0; h < nlvl; ++h)            // forward, leaves first
    for (int q = ps.lvl_off[h]; q < ps.lvl_off[h + 1]; ++q) {
      const int s = ps.lvl_sn[q], sa = ps.sn_start[s], ns = ps.sn_start[s + 1] - sa;
      const int64_t so = ps.st_off[s];
      const int nst = (int)(ps.st_off[s + 1] - so);
      std::vector<cd> F(ns + nst, 0.0);
      for (int i = 0; i < ns; ++i) F[i] = x[sa + i];
      for (int c = ps.ch_off[s]; c < ps.ch_off[s + 1]; ++c) {
        const int ch = ps.ch_ids[c];
        for (int64_t t = ps.st_off[ch]; t < ps.st_off[ch + 1]; ++t) F[ps.st_pos[t]] += u[t];
      }
      const cd *L = l11.data() + ps.l11_off[s];
      for (int k = 0; k < ns; ++k)
        for (int i = k + 1; i < ns; ++i) F[i] -= L[(size_t)k * ns + i] * F[k];
      const cd *L21 = l21.data() + ps.l21_off[s];
      for (int t = 0; t < nst; ++t) {
        cd acc = F[ns + t];
        for (int k = 0; k < ns; ++k) acc -= L21[(size_t)k * nst + t] * F[k];
        u[so + t] = acc;
      }
      for (int i = 0; i < ns; ++i) x[sa + i] = F[i];
    }
  for (int h = nlvl - 1; h >= 0; --h)       // backward, roots first
    for (int q = ps.lvl_off[h]; q < ps.lvl_off[h + 1]; ++q) {
      const int s = ps.lvl_sn[q], sa = ps.sn_start[s], ns = ps.sn_start[s + 1] - sa;
      const int64_t so = ps.st_off[s];
      const int nst = (int)(ps.st_off[s + 1] - so);
      std::vector<cd> z(ns);
      const cd *L21 = l21.data() + ps.l21_off[s];
      for (int i = 0; i < ns; ++i) {
        cd v = x[sa + i] / dg[sa + i];
        for (int t = 0; t < nst; ++t) v -= L21[(size_t)i * nst + t] * x[ps.st_ids[so + t]];
        z[i] = v;
      }
      const cd *Lt = l11t.data() + ps.l11_off[s];
      for (int k = ns - 1; k > 0; --k)
        for (int i = 0; i < k; ++i) z[i] -= Lt[(size_t)k * ns + i] * z[k];
      for (int i = 0; i < ns; ++i) x[sa + i] = z[i];
    }
  // residual with L_w assembled from the branch admittances
  std::vector<cd> r(b);
  for (int e = 0; e < m.b; ++e) {
    const int ru = ps.br_ru[e], rv = ps.br_rv[e];
    if (ru == rv) continue;
    const cd y = yinv[e];
    const cd xu = ru >= 0 ? x[ru] : 0.0, xv = rv >= 0 ? x[rv] : 0.0;
    if (ru >= 0) r[ru] -= y * (xu - xv);
    if (rv >= 0) r[rv] -= y * (xv - xu);
  }
  double nr = 0, nb = 0;
  for (int i = 0; i < nu; ++i) {
    nr += std::norm(r[i]);
    nb += std::norm(b[i]);
  }
  return std::sqrt(nr / nb);
}

}  // namespace pfft
