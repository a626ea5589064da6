// Near-field pair blocks of the pre-correction (Sec. IV-B step 4, Eq. Lb).
//
// For every unordered near pair (t, u), t <= u, the 3x3 block
//   s_i s_j / (4 A_t A_u) * ( D_ij - G_ij ),
// D the direct integral of (r - p_i).(r' - q_j) / |r - r'| over t x u (the
// inner integral over u in closed form, the outer one over t by a rule that
// depends on how close the two are) and G the same interaction as the grid
// sees it: t's and u's projection moments joined through the grid Green's
// function, G = sum_g sum_h m_t(g) H(a_t + g - a_u - h) m_u(h) over the two
// 4 x 4 x 4 stencils.  One thread computes one pair; the same pair function
// also runs in a host loop for the host-only model (inspection without a
// GPU).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "model.h"

namespace pfft {

namespace {

// Closed-form flat-triangle potentials of triangle Q at point r:
// V0 = int_Q 1/|r - r'| dr', V1 = int_Q (r' - r)/|r - r'| dr'
// (Wilton-Rao-Glisson / Graglia edge sums).
__host__ __device__ inline void tri_pot(const double r[3], const double Q[9], double &V0out, double V1[3]) {
  double e1[3], e2[3], nrm[3];
  for (int d = 0; d < 3; ++d) {
    e1[d] = Q[3 + d] - Q[d];
    e2[d] = Q[6 + d] - Q[d];
  }
  nrm[0] = e1[1] * e2[2] - e1[2] * e2[1];
  nrm[1] = e1[2] * e2[0] - e1[0] * e2[2];
  nrm[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double inv = 1.0 / sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
  for (int d = 0; d < 3; ++d) nrm[d] *= inv;
  const double w0 = (r[0] - Q[0]) * nrm[0] + (r[1] - Q[1]) * nrm[1] + (r[2] - Q[2]) * nrm[2];
  const double aw = fabs(w0);
  const double rho[3] = {r[0] - w0 * nrm[0], r[1] - w0 * nrm[1], r[2] - w0 * nrm[2]};
  double V0 = 0, Vr[3] = {0, 0, 0};
  for (int i = 0; i < 3; ++i) {
    const double *qa = Q + 3 * i, *qb = Q + 3 * (i == 2 ? 0 : i + 1);
    double L[3] = {qb[0] - qa[0], qb[1] - qa[1], qb[2] - qa[2]};
    const double len = sqrt(L[0] * L[0] + L[1] * L[1] + L[2] * L[2]);
    const double lu[3] = {L[0] / len, L[1] / len, L[2] / len};
    const double u[3] = {lu[1] * nrm[2] - lu[2] * nrm[1], lu[2] * nrm[0] - lu[0] * nrm[2],
                         lu[0] * nrm[1] - lu[1] * nrm[0]};
    const double ar[3] = {qa[0] - rho[0], qa[1] - rho[1], qa[2] - rho[2]};
    const double t0 = ar[0] * u[0] + ar[1] * u[1] + ar[2] * u[2];
    const double sm = ar[0] * lu[0] + ar[1] * lu[1] + ar[2] * lu[2], sp = sm + len;
    const double R02 = t0 * t0 + w0 * w0;
    const double Rm = sqrt(R02 + sm * sm), Rp = sqrt(R02 + sp * sp);
    double f = 0, beta = 0;
    if (R02 > 1e-28 * len * len) {
      const double Ap = sp >= 0 ? Rp + sp : R02 / (Rp - sp);
      const double Am = sm >= 0 ? Rm + sm : R02 / (Rm - sm);
      f = log(Ap / Am);
      beta = atan2(t0 * sp, R02 + aw * Rp) - atan2(t0 * sm, R02 + aw * Rm);
    }
    V0 += t0 * f - aw * beta;
    const double g = 0.5 * (R02 * f + sp * Rp - sm * Rm);
    for (int d = 0; d < 3; ++d) Vr[d] += u[d] * g;
  }
  V0out = V0;
  for (int d = 0; d < 3; ++d) V1[d] = Vr[d] - w0 * V0 * nrm[d];
}

struct NearGeom {
  const double *V;       // [nv][3]
  const int *T;          // [n][3]
  const double *area;    // [n]
  const int8_t *sgn;     // [n][3]
  const double *M0;      // [n][64]
  const double *M1;      // [n][64][3]
  const double *pl;      // [n][3][3] vertex - centroid
  const int *anchor;     // [n][3]
  const double *H;       // grid Green's function over offsets [-Dm, Dm]^3
  int Dm[3], S[3];
  const double *rule;    // [points][4]: barycentric point on t, weight (each rule sums to 1)
  int roff[5];           // class c takes points [roff[c], roff[c + 1])
};

// One pair: the scaled (direct - grid) block and the scaled direct block.
__host__ __device__ inline void pair_block(const NearGeom &g, int t, int u, int cls, double out[9],
                                           double dir[9]) {
  double P[9], Q[9];
  for (int v = 0; v < 3; ++v)
    for (int d = 0; d < 3; ++d) {
      P[3 * v + d] = g.V[3 * g.T[3 * t + v] + d];
      Q[3 * v + d] = g.V[3 * g.T[3 * u + v] + d];
    }
  double E[9];
  for (int k = 0; k < 9; ++k) E[k] = 0;
  const double At = g.area[t];
  for (int q = g.roff[cls]; q < g.roff[cls + 1]; ++q) {
    const double *L = g.rule + 4 * q;
    double r[3];
    for (int d = 0; d < 3; ++d) r[d] = L[0] * P[d] + L[1] * P[3 + d] + L[2] * P[6 + d];
    double V0, V1[3];
    tri_pot(r, Q, V0, V1);
    const double w = L[3] * At;
    for (int i = 0; i < 3; ++i) {
      const double a[3] = {r[0] - P[3 * i], r[1] - P[3 * i + 1], r[2] - P[3 * i + 2]};
      const double aV1 = a[0] * V1[0] + a[1] * V1[1] + a[2] * V1[2];
      for (int j = 0; j < 3; ++j) {
        const double ab = a[0] * (r[0] - Q[3 * j]) + a[1] * (r[1] - Q[3 * j + 1]) + a[2] * (r[2] - Q[3 * j + 2]);
        E[3 * i + j] += w * (aV1 + ab * V0);
      }
    }
  }
  if (u == t)
    for (int i = 0; i < 3; ++i)
      for (int j = i + 1; j < 3; ++j) E[3 * i + j] = E[3 * j + i] = 0.5 * (E[3 * i + j] + E[3 * j + i]);
  // the grid's interaction of the two stencils
  const double *M0t = g.M0 + 64 * (size_t)t, *M1t = g.M1 + 192 * (size_t)t;
  const double *M0u = g.M0 + 64 * (size_t)u, *M1u = g.M1 + 192 * (size_t)u;
  const int b0 = g.anchor[3 * t] - g.anchor[3 * u] + g.Dm[0];
  const int b1 = g.anchor[3 * t + 1] - g.anchor[3 * u + 1] + g.Dm[1];
  const int b2 = g.anchor[3 * t + 2] - g.anchor[3 * u + 2] + g.Dm[2];
  double X[4][4];
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 4; ++c) X[a][c] = 0;
  for (int gg = 0; gg < 64; ++gg) {
    const int gi = gg >> 4, gj = (gg >> 2) & 3, gk = gg & 3;
    double tmp[4] = {0, 0, 0, 0};
    for (int h = 0; h < 64; ++h) {
      const int hi = h >> 4, hj = (h >> 2) & 3, hk = h & 3;
      const double Hv = g.H[((size_t)(b0 + gi - hi) * g.S[1] + (b1 + gj - hj)) * g.S[2] + (b2 + gk - hk)];
      tmp[0] += Hv * M0u[h];
      tmp[1] += Hv * M1u[3 * h];
      tmp[2] += Hv * M1u[3 * h + 1];
      tmp[3] += Hv * M1u[3 * h + 2];
    }
    const double mt[4] = {M0t[gg], M1t[3 * gg], M1t[3 * gg + 1], M1t[3 * gg + 2]};
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 4; ++c) X[a][c] += mt[a] * tmp[c];
  }
  const double *plt = g.pl + 9 * (size_t)t, *plu = g.pl + 9 * (size_t)u;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double gr = 0;
      for (int c = 0; c < 3; ++c)
        gr += X[1 + c][1 + c] - plu[3 * j + c] * X[1 + c][0] - plt[3 * i + c] * X[0][1 + c] +
              plt[3 * i + c] * plu[3 * j + c] * X[0][0];
      const double sc = g.sgn[3 * t + i] * g.sgn[3 * u + j] / (4.0 * g.area[t] * g.area[u]);
      out[3 * i + j] = sc * (E[3 * i + j] - gr);
      dir[3 * i + j] = sc * E[3 * i + j];
    }
  if (u == t)
    for (int i = 0; i < 3; ++i)
      for (int j = i + 1; j < 3; ++j) out[3 * i + j] = out[3 * j + i] = 0.5 * (out[3 * i + j] + out[3 * j + i]);
}

struct PairRange {
  int64_t r0, r1;        // pairs [r0, r1) of the class-sorted list
  int64_t cb[3];         // first pair of classes 1, 2, 3
  int64_t ntouch;        // pairs [0, ntouch) also keep their direct block
};

__global__ void __launch_bounds__(256) k_near_blocks(NearGeom g, PairRange pr, const int *pt, const int *pu,
                                                    const int64_t *pidx, double *blk, double *dirb) {
  const int64_t r = pr.r0 + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= pr.r1) return;
  const int cls = (r >= pr.cb[0]) + (r >= pr.cb[1]) + (r >= pr.cb[2]);
  double out[9], dir[9];
  pair_block(g, pt[r], pu[r], cls, out, dir);
  double *o = blk + 9 * pidx[r];
  for (int k = 0; k < 9; ++k) o[k] = out[k];
  if (r < pr.ntouch)
    for (int k = 0; k < 9; ++k) dirb[9 * r + k] = dir[k];
}

// Gauss-Legendre nodes and weights on [0, 1] (Newton iteration on P_q).
void gauss01(int q, std::vector<double> &x, std::vector<double> &w) {
  x.resize(q);
  w.resize(q);
  for (int i = 0; i < q; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (q + 0.5)), dp = 1;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = z;
      for (int k = 2; k <= q; ++k) {
        const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (z * p1 - p0) / (z * z - 1);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = 0.5 * (1 - z);
    w[i] = 1.0 / ((1 - z * z) * dp * dp);
  }
}

// Class 0 (pairs that touch): t is cut into three pieces from its centroid;
// each piece maps (s, v) in [0,1]^2 to (1 - u)(edge point s) + u c with
// u = v^2 (graded toward the edge, where the outer integrand behaves like
// d log d) and s = sigma^2 / (sigma^2 + (1 - sigma)^2) (graded toward the
// vertices); Gauss-Legendre of order 16 in (sigma, v).
void graded_rule(std::vector<double> &R) {
  const int q = 16;
  std::vector<double> x, wx;
  gauss01(q, x, wx);
  for (int k = 0; k < 3; ++k)
    for (int a = 0; a < q; ++a) {
      const double sg = x[a], A = sg * sg, B = (1 - sg) * (1 - sg);
      const double s = A / (A + B), ds = 2 * sg * (1 - sg) / ((A + B) * (A + B));
      for (int b2 = 0; b2 < q; ++b2) {
        const double v = x[b2], u = v * v, du = 2 * v;
        double base[3] = {0, 0, 0};
        base[k] = 1 - s;
        base[(k + 1) % 3] = s;
        for (int d = 0; d < 3; ++d) R.push_back((1 - u) * base[d] + u / 3.0);
        R.push_back(2.0 / 3.0 * (1 - u) * wx[a] * ds * wx[b2] * du);
      }
    }
}

// Classes 1..3: the 7-point Dunavant rule (degree 5) on the 4^level
// congruent sub-triangles of t (midpoint subdivision), level 3, 2, 1.
void subdivided_rule(int level, std::vector<double> &R) {
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
  struct Tri { double b[3][3]; };
  std::vector<Tri> cur(1);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) cur[0].b[i][j] = (i == j);
  for (int lv = 0; lv < level; ++lv) {
    std::vector<Tri> nxt;
    for (const Tri &T : cur) {
      double m01[3], m12[3], m20[3];
      for (int d = 0; d < 3; ++d) {
        m01[d] = 0.5 * (T.b[0][d] + T.b[1][d]);
        m12[d] = 0.5 * (T.b[1][d] + T.b[2][d]);
        m20[d] = 0.5 * (T.b[2][d] + T.b[0][d]);
      }
      const double *sets[4][3] = {{T.b[0], m01, m20}, {m01, T.b[1], m12}, {m20, m12, T.b[2]}, {m01, m12, m20}};
      for (int s = 0; s < 4; ++s) {
        Tri c;
        for (int v = 0; v < 3; ++v)
          for (int d = 0; d < 3; ++d) c.b[v][d] = sets[s][v][d];
        nxt.push_back(c);
      }
    }
    cur.swap(nxt);
  }
  const double ws = 1.0 / (double)cur.size();
  for (const Tri &S : cur)
    for (int q = 0; q < 7; ++q) {
      for (int v = 0; v < 3; ++v)
        R.push_back(D7_L[q][0] * S.b[0][v] + D7_L[q][1] * S.b[1][v] + D7_L[q][2] * S.b[2][v]);
      R.push_back(D7_W[q] * ws);
    }
}

void dev_ok(hipError_t e, const char *what) {
  if (e != hipSuccess) throw SetupError{-4, std::string("near-field blocks: ") + what + ": " + hipGetErrorString(e)};
}

template <class X>
X *dev_upload(const X *h, size_t n, hipStream_t st, std::vector<void *> &owned) {
  void *p = nullptr;
  dev_ok(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(X)), "hipMalloc");
  owned.push_back(p);
  if (n) dev_ok(hipMemcpyAsync(p, h, n * sizeof(X), hipMemcpyHostToDevice, st), "upload");
  return (X *)p;
}

}  // namespace

void near_pair_blocks(const HostModel &m, const NearPairList &pl, const std::vector<double> &Htab, const int Dm[3],
                      const int S[3], bool device, void *stream, double *blk, double *dirb) {
  std::vector<double> rule;
  NearGeom g;
  g.roff[0] = 0;
  graded_rule(rule);
  for (int c = 1; c <= 3; ++c) {
    g.roff[c] = (int)(rule.size() / 4);
    subdivided_rule(4 - c, rule);
  }
  g.roff[4] = (int)(rule.size() / 4);
  for (int d = 0; d < 3; ++d) {
    g.Dm[d] = Dm[d];
    g.S[d] = S[d];
  }
  const int64_t np = (int64_t)pl.t.size();
  if (!device) {
    g.V = m.V.data();
    g.T = m.T.data();
    g.area = m.area.data();
    g.sgn = m.tri_sign.data();
    g.M0 = m.M0.data();
    g.M1 = m.M1.data();
    g.pl = m.pl.data();
    g.anchor = m.anchor.data();
    g.H = Htab.data();
    g.rule = rule.data();
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = 0; r < np; ++r) {
      const int cls = (r >= pl.cls_end[0]) + (r >= pl.cls_end[1]) + (r >= pl.cls_end[2]);
      double out[9], dir[9];
      pair_block(g, pl.t[r], pl.u[r], cls, out, dir);
      std::copy(out, out + 9, blk + 9 * pl.idx[r]);
      if (r < pl.cls_end[0]) std::copy(dir, dir + 9, dirb + 9 * r);
    }
    return;
  }
  hipStream_t st = (hipStream_t)stream;
  std::vector<void *> owned;
  auto release = [&]() {
    for (void *p : owned) (void)hipFree(p);
    owned.clear();
  };
  try {
    const size_t n = (size_t)m.n;
    g.V = dev_upload(m.V.data(), m.V.size(), st, owned);
    g.T = dev_upload(m.T.data(), 3 * n, st, owned);
    g.area = dev_upload(m.area.data(), n, st, owned);
    g.sgn = dev_upload(m.tri_sign.data(), 3 * n, st, owned);
    g.M0 = dev_upload(m.M0.data(), 64 * n, st, owned);
    g.M1 = dev_upload(m.M1.data(), 192 * n, st, owned);
    g.pl = dev_upload(m.pl.data(), 9 * n, st, owned);
    g.anchor = dev_upload(m.anchor.data(), 3 * n, st, owned);
    g.H = dev_upload(Htab.data(), Htab.size(), st, owned);
    g.rule = dev_upload(rule.data(), rule.size(), st, owned);
    const int *dt = dev_upload(pl.t.data(), (size_t)np, st, owned);
    const int *du = dev_upload(pl.u.data(), (size_t)np, st, owned);
    const int64_t *di = dev_upload(pl.idx.data(), (size_t)np, st, owned);
    double *dblk = nullptr, *ddir = nullptr;
    const int64_t nt = pl.cls_end[0];
    dev_ok(hipMalloc((void **)&dblk, std::max<size_t>(9 * (size_t)np, 1) * sizeof(double)), "hipMalloc blocks");
    owned.push_back(dblk);
    dev_ok(hipMalloc((void **)&ddir, std::max<size_t>(9 * (size_t)nt, 1) * sizeof(double)), "hipMalloc direct");
    owned.push_back(ddir);
    PairRange pr;
    for (int c = 0; c < 3; ++c) pr.cb[c] = pl.cls_end[c];
    pr.ntouch = nt;
    // launches of at most 2^22 pairs
    const int64_t chunk = (int64_t)1 << 22;
    for (int64_t r0 = 0; r0 < np; r0 += chunk) {
      pr.r0 = r0;
      pr.r1 = std::min(np, r0 + chunk);
      const unsigned nb = (unsigned)((pr.r1 - pr.r0 + 255) / 256);
      hipLaunchKernelGGL(k_near_blocks, dim3(nb), dim3(256), 0, st, g, pr, dt, du, di, dblk, ddir);
      dev_ok(hipGetLastError(), "launch");
    }
    dev_ok(hipMemcpyAsync(blk, dblk, 9 * (size_t)np * sizeof(double), hipMemcpyDeviceToHost, st), "download");
    if (nt) dev_ok(hipMemcpyAsync(dirb, ddir, 9 * (size_t)nt * sizeof(double), hipMemcpyDeviceToHost, st), "download");
    dev_ok(hipStreamSynchronize(st), "synchronize");
  } catch (...) {
    (void)hipStreamSynchronize(st);
    release();
    throw;
  }
  release();
}

}  // namespace pfft
