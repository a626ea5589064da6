/* Oracle helper (test infrastructure only): raw triangle-pair blocks of the
 * static kernel (first term of Eq. Zb, static Green's function of
 * Eq. StaticGF, constant factors outside),
 *
 *     M[i][j] = int_t int_t' (r - p_i).(r' - q_j) / |r - r'| dS' dS ,
 *
 * with p_i the vertices of the outer triangle t and q_j those of the inner
 * triangle t'.  Both integrals are numerical; no closed-form potential is
 * used anywhere:
 *
 *  - touching pairs (same triangle, common edge, common vertex): the
 *    Sauter-Schwab regularised cubature.  The four-dimensional domain is cut
 *    into 6 / 5 / 2 pieces, each mapped from the unit hypercube so that the
 *    Jacobian vanishes to the order of the 1/R singularity; the transformed
 *    integrand is smooth and a q^4 tensor Gauss-Legendre rule converges
 *    exponentially in q;
 *  - separated pairs: tensor products of collapsed (conical) Gauss rules on
 *    both triangles, the order chosen from the separation ratio; pairs closer
 *    than one radius are first split recursively (the larger triangle into
 *    its four midpoint children) until every piece pair is that far apart.
 *
 * Plain C, FP64, OpenMP over pairs.  The GPU library neither links nor calls
 * this file.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double tri_area(const double *T) {
  double e1[3], e2[3], c[3];
  for (int d = 0; d < 3; ++d) { e1[d] = T[3 + d] - T[d]; e2[d] = T[6 + d] - T[d]; }
  cross3(e1, e2, c);
  return 0.5 * sqrt(dot3(c, c));
}

/* Gauss-Legendre nodes and weights on [0, 1] (q <= 32): Newton's method on
 * the Legendre polynomial P_q from the Chebyshev-like first guesses
 * cos(pi (k + 3/4) / (q + 1/2)). */
static void gauss01(int q, double *x, double *w) {
  for (int k = 0; k < q; ++k) {
    double z = cos(M_PI * (k + 0.75) / (q + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int n = 2; n <= q; ++n) {
        double p2 = ((2.0 * n - 1.0) * z * p1 - (n - 1.0) * p0) / n;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int n = 2; n <= q; ++n) {
        double p2 = ((2.0 * n - 1.0) * z * p1 - (n - 1.0) * p0) / n;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (z * p1 - p0) / (z * z - 1.0);
    }
    x[k] = 0.5 * (1.0 - z);
    w[k] = 1.0 / ((1.0 - z * z) * dp * dp);   /* 2/((1-z^2) P'^2) on [-1,1], halved */
  }
}

/* reference triangle {0 <= x2 <= x1 <= 1}; chi(x) = a0 + x1 (a1 - a0) + x2 (a2 - a1) */
static void chi(const double *T, double x1, double x2, double *r) {
  for (int d = 0; d < 3; ++d) r[d] = T[d] + x1 * (T[3 + d] - T[d]) + x2 * (T[6 + d] - T[3 + d]);
}

/* Moments of one pair integral.  With local origins c (centroid of the
 * outer triangle) and c' (of the inner one), rt = r - c, rq = r' - c',
 * pt_i = p_i - c, qt_j = q_j - c', the block entry is
 *   sum w (rt - pt_i).(rq - qt_j) / R
 *     = s - a.qt_j - pt_i.b + (pt_i.qt_j) g
 * with g = sum w/R, a = sum w rt/R, b = sum w rq/R, s = sum w rt.rq/R. */
typedef struct {
  double g, a[3], b[3], s;
} moments;

static void add_point_pair(const double *r, const double *rp, const double *c, const double *cq, double wt,
                           moments *M) {
  const double D[3] = {r[0] - rp[0], r[1] - rp[1], r[2] - rp[2]};
  const double g = wt / sqrt(dot3(D, D));
  const double rt[3] = {r[0] - c[0], r[1] - c[1], r[2] - c[2]};
  const double rq[3] = {rp[0] - cq[0], rp[1] - cq[1], rp[2] - cq[2]};
  M->g += g;
  for (int d = 0; d < 3; ++d) {
    M->a[d] += g * rt[d];
    M->b[d] += g * rq[d];
  }
  M->s += g * dot3(rt, rq);
}

static void centroid(const double *T, double *c) {
  for (int d = 0; d < 3; ++d) c[d] = (T[d] + T[3 + d] + T[6 + d]) / 3.0;
}

/* block entries from the moments, scaled */
static void moments_to_block(const moments *M, const double *Pv, const double *Qv, const double *c,
                             const double *cq, double scale, double *out) {
  double pt[3][3], qt[3][3];
  for (int i = 0; i < 3; ++i)
    for (int d = 0; d < 3; ++d) {
      pt[i][d] = Pv[3 * i + d] - c[d];
      qt[i][d] = Qv[3 * i + d] - cq[d];
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      out[3 * i + j] = scale * (M->s - dot3(M->a, qt[j]) - dot3(pt[i], M->b) + dot3(pt[i], qt[j]) * M->g);
}

/* ---------------------------------------------------------------------------
 * touching pairs: Sauter-Schwab
 *
 * The caller orders the vertices so that the shared ones come first, in the
 * same order on both triangles: a common edge is then chi(s, 0) on both, a
 * common vertex chi(0, 0).  kind 3 = same triangle, 2 = common edge,
 * 1 = common vertex.  The integral over the reference pair
 * int_T^ int_T^ F(x, y) dy dx is the sum over the pieces of
 * int_[0,1]^4 J(xi, eta) F(x(xi, eta), y(xi, eta)), and the physical integral
 * carries the factor (2 A_t)(2 A_t').
 * ------------------------------------------------------------------------- */
static int ss_npieces(int kind) { return kind == 3 ? 6 : kind == 2 ? 5 : 2; }

/* piece p of the case: reference points x, y of both triangles and the
 * Jacobian J at (xi, e1, e2, e3) in the unit hypercube */
static void ss_piece(int kind, int p, double xi, double e1, double e2, double e3, double *x, double *y,
                     double *J) {
  if (kind == 3) {
    *J = xi * xi * xi * e1 * e1 * e2;
    switch (p >> 1) {
      case 0:
        x[0] = xi;                       x[1] = xi * (1 - e1 + e1 * e2);
        y[0] = xi * (1 - e1 * e2 * e3);  y[1] = xi * (1 - e1);
        break;
      case 1:
        x[0] = xi;                       x[1] = xi * e1 * (1 - e2 + e2 * e3);
        y[0] = xi * (1 - e1 * e2);       y[1] = xi * e1 * (1 - e2);
        break;
      default:
        x[0] = xi * (1 - e1 * e2 * e3);  x[1] = xi * e1 * (1 - e2 * e3);
        y[0] = xi;                       y[1] = xi * e1 * (1 - e2);
        break;
    }
    if (p & 1) {   /* the mirror piece: x and y exchanged */
      double t0 = x[0], t1 = x[1];
      x[0] = y[0]; x[1] = y[1]; y[0] = t0; y[1] = t1;
    }
    return;
  }
  if (kind == 2) {
    *J = xi * xi * xi * e1 * e1 * (p == 0 ? 1.0 : e2);
    switch (p) {
      case 0:
        x[0] = xi;                       x[1] = xi * e1 * e3;
        y[0] = xi * (1 - e1 * e2);       y[1] = xi * e1 * (1 - e2);
        break;
      case 1:
        x[0] = xi;                       x[1] = xi * e1;
        y[0] = xi * (1 - e1 * e2 * e3);  y[1] = xi * e1 * e2 * (1 - e3);
        break;
      case 2:
        x[0] = xi * (1 - e1 * e2);       x[1] = xi * e1 * (1 - e2);
        y[0] = xi;                       y[1] = xi * e1 * e2 * e3;
        break;
      case 3:
        x[0] = xi * (1 - e1 * e2 * e3);  x[1] = xi * e1 * e2 * (1 - e3);
        y[0] = xi;                       y[1] = xi * e1;
        break;
      default:
        x[0] = xi * (1 - e1 * e2 * e3);  x[1] = xi * e1 * (1 - e2 * e3);
        y[0] = xi;                       y[1] = xi * e1 * e2;
        break;
    }
    return;
  }
  *J = xi * xi * xi * e2;
  if (p == 0) {
    x[0] = xi;       x[1] = xi * e1;
    y[0] = xi * e2;  y[1] = xi * e2 * e3;
  } else {
    x[0] = xi * e2;  x[1] = xi * e2 * e3;
    y[0] = xi;       y[1] = xi * e1;
  }
}

/* Gauss rule on [0, 1] for a factor 1 / |a + t b|: the sinh substitution
 * t = t* + d sinh(u) about the point t* of [0, 1] nearest to the zero of the
 * linear function, d its distance there (in t units), turns the
 * near-singular factor into a smooth one (it matters for obtuse and thin
 * triangles, where a + t b passes close to zero). */
static void sinh_rule(const double *a, const double *b, int q, const double *gx, const double *gw, double *x,
                      double *w) {
  const double bb = dot3(b, b);
  double ts = bb > 0.0 ? -dot3(a, b) / bb : 0.5;
  if (ts < 0.0) ts = 0.0;
  if (ts > 1.0) ts = 1.0;
  double m[3] = {a[0] + ts * b[0], a[1] + ts * b[1], a[2] + ts * b[2]};
  double d = bb > 0.0 ? sqrt(dot3(m, m) / bb) : 1.0;
  if (d > 1.0) d = 1.0;
  if (d < 1e-6) d = 1e-6;
  const double u0 = asinh((0.0 - ts) / d), u1 = asinh((1.0 - ts) / d);
  for (int k = 0; k < q; ++k) {
    const double u = u0 + (u1 - u0) * gx[k];
    x[k] = ts + d * sinh(u);
    w[k] = gw[k] * (u1 - u0) * d * cosh(u);
  }
}

/* One touching pair.  In every piece the physical difference r - r' is a
 * power product of the variables times a "bracket" that depends on the
 * remaining ones and is linear in one of them, v_s: eta3 for the same
 * triangle (bracket of eta3 alone) and the common edge (bracket of eta2,
 * eta3), eta2 for the common vertex (bracket of eta1, eta2, eta3).  v_s
 * takes a sinh rule built, for each node of the bracket's other variables,
 * from the bracket's values at v_s = 0 and 1; the other variables take the
 * plain Gauss rule. */
static void ss_pair(int kind, const double *Tp, const double *Tq, int q, const double *gx, const double *gw,
                    const double *c, const double *cq, moments *acc) {
  int par[2], npar, scl[3], nscl, sv;
  if (kind == 3) { npar = 0; scl[0] = 0; scl[1] = 1; scl[2] = 2; nscl = 3; sv = 3; }
  else if (kind == 2) { npar = 1; par[0] = 2; scl[0] = 0; scl[1] = 1; nscl = 2; sv = 3; }
  else { npar = 2; par[0] = 1; par[1] = 3; scl[0] = 0; nscl = 1; sv = 2; }
  int npc = 1, nsc = 1;
  for (int i = 0; i < npar; ++i) npc *= q;
  for (int i = 0; i < nscl; ++i) nsc *= q;
  for (int p = 0; p < ss_npieces(kind); ++p) {
    for (int ip = 0; ip < npc; ++ip) {
      double v[4], wp = 1.0;
      for (int i = 0, r = ip; i < npar; ++i, r /= q) { v[par[i]] = gx[r % q]; wp *= gw[r % q]; }
      /* bracket at v_s = 0 and 1 with the power-product variables at 1 */
      double br[2][3];
      for (int e = 0; e < 2; ++e) {
        for (int i = 0; i < nscl; ++i) v[scl[i]] = 1.0;
        v[sv] = (double)e;
        double x[2], y[2], J, r[3], rp[3];
        ss_piece(kind, p, v[0], v[1], v[2], v[3], x, y, &J);
        chi(Tp, x[0], x[1], r);
        chi(Tq, y[0], y[1], rp);
        for (int d = 0; d < 3; ++d) br[e][d] = r[d] - rp[d];
      }
      double bvec[3] = {br[1][0] - br[0][0], br[1][1] - br[0][1], br[1][2] - br[0][2]};
      double xs[32], ws[32];
      sinh_rule(br[0], bvec, q, gx, gw, xs, ws);
      for (int is = 0; is < nsc; ++is) {
        double wsc = wp;
        for (int i = 0, r = is; i < nscl; ++i, r /= q) { v[scl[i]] = gx[r % q]; wsc *= gw[r % q]; }
        for (int k = 0; k < q; ++k) {
          v[sv] = xs[k];
          double x[2], y[2], J, r[3], rp[3];
          ss_piece(kind, p, v[0], v[1], v[2], v[3], x, y, &J);
          chi(Tp, x[0], x[1], r);
          chi(Tq, y[0], y[1], rp);
          add_point_pair(r, rp, c, cq, wsc * ws[k] * J, acc);
        }
      }
    }
  }
}

/* P, Q: m pairs of vertex rows (ordered as above); kind[m]; q Gauss points
 * per hypercube dimension (q <= 32). */
void oracle_blocks_touching(long m, const double *P, const double *Q, const int *kind, long q, double *out) {
  double gx[32], gw[32];
  if (q > 32) q = 32;
  gauss01((int)q, gx, gw);
#pragma omp parallel for schedule(dynamic, 16)
  for (long k = 0; k < m; ++k) {
    const double *Pk = P + 9 * k, *Qk = Q + 9 * k;
    const double scale = 4.0 * tri_area(Pk) * tri_area(Qk);
    double c[3], cq[3];
    centroid(Pk, c);
    centroid(Qk, cq);
    moments acc = {0};
    ss_pair(kind[k], Pk, Qk, (int)q, gx, gw, c, cq, &acc);
    moments_to_block(&acc, Pk, Qk, c, cq, scale, out + 9 * k);
  }
}

/* ---------------------------------------------------------------------------
 * separated pairs
 * ------------------------------------------------------------------------- */
#define NRULE 5
static const int RULE_Q[NRULE] = {3, 4, 5, 6, 8};
static double rule_l[NRULE][144][3], rule_w[NRULE][144];
static int rule_n[NRULE];
static int rules_ready = 0;

/* collapsed (conical) product rule with q x q points on the unit triangle,
 * barycentric points, weights summing to 1 */
static void make_rules(void) {
  for (int k = 0; k < NRULE; ++k) {
    const int q = RULE_Q[k];
    double x[32], w[32];
    gauss01(q, x, w);
    int n = 0;
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j) {
        const double l1 = x[i], l2 = x[j] * (1.0 - x[i]);
        rule_l[k][n][0] = 1.0 - l1 - l2;
        rule_l[k][n][1] = l1;
        rule_l[k][n][2] = l2;
        rule_w[k][n] = 2.0 * w[i] * w[j] * (1.0 - x[i]);
        ++n;
      }
    rule_n[k] = n;
  }
  rules_ready = 1;
}

static void centroid_radius(const double *T, double *c, double *rad) {
  centroid(T, c);
  double r = 0.0;
  for (int v = 0; v < 3; ++v) {
    double D[3] = {T[3 * v] - c[0], T[3 * v + 1] - c[1], T[3 * v + 2] - c[2]};
    double l = sqrt(dot3(D, D));
    if (l > r) r = l;
  }
  *rad = r;
}

static void child(const double *T, int k, double *C) {
  double m01[3], m12[3], m20[3];
  for (int d = 0; d < 3; ++d) {
    m01[d] = 0.5 * (T[d] + T[3 + d]);
    m12[d] = 0.5 * (T[3 + d] + T[6 + d]);
    m20[d] = 0.5 * (T[6 + d] + T[d]);
  }
  const double *v[3];
  if (k == 0) { v[0] = T; v[1] = m01; v[2] = m20; }
  else if (k == 1) { v[0] = m01; v[1] = T + 3; v[2] = m12; }
  else if (k == 2) { v[0] = m20; v[1] = m12; v[2] = T + 6; }
  else { v[0] = m01; v[1] = m12; v[2] = m20; }
  for (int i = 0; i < 3; ++i)
    for (int d = 0; d < 3; ++d) C[3 * i + d] = v[i][d];
}

/* Integrates over the piece pair (Dp, Dq) (sub-triangles of the outer and
 * inner triangles); c, cq are the local origins of the moments (centroids of
 * the whole triangles). */
static void separated(const double *Dp, const double *Dq, const double *c, const double *cq, int depth,
                      double split, moments *acc) {
  double mp[3], mq[3], rp, rq;
  centroid_radius(Dp, mp, &rp);
  centroid_radius(Dq, mq, &rq);
  double D[3] = {mp[0] - mq[0], mp[1] - mq[1], mp[2] - mq[2]};
  const double rmax = rp > rq ? rp : rq;
  const double eta = (sqrt(dot3(D, D)) - rp - rq) / rmax;
  if (eta < split && depth < 12) {
    double C[9];
    for (int k = 0; k < 4; ++k) {
      if (rp >= rq) {
        child(Dp, k, C);
        separated(C, Dq, c, cq, depth + 1, split, acc);
      } else {
        child(Dq, k, C);
        separated(Dp, C, c, cq, depth + 1, split, acc);
      }
    }
    return;
  }
  const int ri = split > 1.0 ? NRULE - 1 : eta >= 40.0 ? 0 : eta >= 12.0 ? 1 : eta >= 4.0 ? 2 : eta >= 2.0 ? 3 : 4;
  const double Ap = tri_area(Dp), Aq = tri_area(Dq);
  const int n = rule_n[ri];
  /* inner points: absolute (for r - r') and relative to cq (moments) */
  double qx[144], qy[144], qz[144], ux[144], uy[144], uz[144], qw[144];
  for (int b = 0; b < n; ++b) {
    const double *l = rule_l[ri][b];
    qx[b] = l[0] * Dq[0] + l[1] * Dq[3] + l[2] * Dq[6];
    qy[b] = l[0] * Dq[1] + l[1] * Dq[4] + l[2] * Dq[7];
    qz[b] = l[0] * Dq[2] + l[1] * Dq[5] + l[2] * Dq[8];
    ux[b] = qx[b] - cq[0];
    uy[b] = qy[b] - cq[1];
    uz[b] = qz[b] - cq[2];
    qw[b] = Aq * rule_w[ri][b];
  }
  for (int a = 0; a < n; ++a) {
    const double *l = rule_l[ri][a];
    const double rx = l[0] * Dp[0] + l[1] * Dp[3] + l[2] * Dp[6];
    const double ry = l[0] * Dp[1] + l[1] * Dp[4] + l[2] * Dp[7];
    const double rz = l[0] * Dp[2] + l[1] * Dp[5] + l[2] * Dp[8];
    const double tx = rx - c[0], ty = ry - c[1], tz = rz - c[2];
    double g = 0.0, bx = 0.0, by = 0.0, bz = 0.0, ss = 0.0;
    for (int b = 0; b < n; ++b) {
      const double dx = rx - qx[b], dy = ry - qy[b], dz = rz - qz[b];
      const double h = qw[b] / sqrt(dx * dx + dy * dy + dz * dz);
      g += h;
      bx += h * ux[b];
      by += h * uy[b];
      bz += h * uz[b];
      ss += h * (tx * ux[b] + ty * uy[b] + tz * uz[b]);
    }
    const double wa = Ap * rule_w[ri][a];
    acc->g += wa * g;
    acc->a[0] += wa * g * tx;
    acc->a[1] += wa * g * ty;
    acc->a[2] += wa * g * tz;
    acc->b[0] += wa * bx;
    acc->b[1] += wa * by;
    acc->b[2] += wa * bz;
    acc->s += wa * ss;
  }
}

/* P, Q: m pairs of vertex rows of triangles that share no vertex.  refine
 * = 1 asks for a much finer integration (pieces split until they are four
 * radii apart, the highest order everywhere), used to check the default. */
void oracle_blocks_separated(long m, const double *P, const double *Q, int refine, double *out) {
  if (!rules_ready) make_rules();
  const double split = refine ? 4.0 : 1.0;
#pragma omp parallel for schedule(dynamic, 64)
  for (long k = 0; k < m; ++k) {
    double c[3], cq[3];
    centroid(P + 9 * k, c);
    centroid(Q + 9 * k, cq);
    moments acc = {0};
    separated(P + 9 * k, Q + 9 * k, c, cq, 0, split, &acc);
    moments_to_block(&acc, P + 9 * k, Q + 9 * k, c, cq, 1.0, out + 9 * k);
  }
}

/* Gauss-Legendre rule on [0, 1] as computed here (for tests of the helper). */
void oracle_gauss01(long q, double *x, double *w) { gauss01((int)q, x, w); }
