/* Oracle helper (test infrastructure only): raw triangle-pair blocks of the
 * static kernel,
 *     M[i][j] = int_t int_t' (r - p_i).(r' - q_j) / |r - r'| dS' dS,
 * evaluated exactly as the numpy oracle does (closed-form inner integral over
 * t', caller-supplied outer rule on t; or a product rule on both triangles),
 * only faster.  Plain C, FP64, OpenMP over pairs.  Not used by the GPU
 * library.
 */
#include <math.h>
#include <string.h>

static void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* V0 = int_Q 1/R, V1 = int_Q (r' - r)/R for a flat triangle Q (3x3 rows). */
static void potentials(const double *r, const double *Q, double *V0out, double *V1) {
  double e1[3], e2[3], nrm[3];
  for (int d = 0; d < 3; ++d) { e1[d] = Q[3 + d] - Q[d]; e2[d] = Q[6 + d] - Q[d]; }
  cross3(e1, e2, nrm);
  double nn = sqrt(dot3(nrm, nrm));
  for (int d = 0; d < 3; ++d) nrm[d] /= nn;
  double rq[3] = {r[0] - Q[0], r[1] - Q[1], r[2] - Q[2]};
  double w0 = dot3(rq, nrm), aw = fabs(w0);
  double rho[3] = {r[0] - w0 * nrm[0], r[1] - w0 * nrm[1], r[2] - w0 * nrm[2]};
  double V0 = 0.0, Vr[3] = {0, 0, 0};
  for (int i = 0; i < 3; ++i) {
    const double *qa = Q + 3 * i, *qb = Q + 3 * ((i + 1) % 3);
    double L[3] = {qb[0] - qa[0], qb[1] - qa[1], qb[2] - qa[2]};
    double ln = sqrt(dot3(L, L));
    double l[3] = {L[0] / ln, L[1] / ln, L[2] / ln}, u[3];
    cross3(l, nrm, u);
    double ar[3] = {qa[0] - rho[0], qa[1] - rho[1], qa[2] - rho[2]};
    double t0 = dot3(ar, u), sm = dot3(ar, l), sp = sm + ln;
    double R02 = t0 * t0 + w0 * w0;
    double Rm = sqrt(R02 + sm * sm), Rp = sqrt(R02 + sp * sp);
    double f = 0.0, beta = 0.0;
    if (R02 > (1e-14 * ln) * (1e-14 * ln)) {
      double Ap = sp >= 0 ? Rp + sp : R02 / (Rp - sp);
      double Am = sm >= 0 ? Rm + sm : R02 / (Rm - sm);
      f = log(Ap) - log(Am);
      beta = atan2(t0 * sp, R02 + aw * Rp) - atan2(t0 * sm, R02 + aw * Rm);
    }
    V0 += t0 * f - aw * beta;
    double g = 0.5 * (R02 * f + sp * Rp - sm * Rm);
    for (int d = 0; d < 3; ++d) Vr[d] += u[d] * g;
  }
  *V0out = V0;
  for (int d = 0; d < 3; ++d) V1[d] = Vr[d] - w0 * V0 * nrm[d];
}

static double tri_area(const double *P) {
  double e1[3], e2[3], c[3];
  for (int d = 0; d < 3; ++d) { e1[d] = P[3 + d] - P[d]; e2[d] = P[6 + d] - P[d]; }
  cross3(e1, e2, c);
  return 0.5 * sqrt(dot3(c, c));
}

void oracle_blocks_analytic(long m, const double *P, const double *Q, long nq,
                            const double *lam, const double *w, double *out) {
#pragma omp parallel for schedule(dynamic, 64)
  for (long k = 0; k < m; ++k) {
    const double *Pk = P + 9 * k, *Qk = Q + 9 * k;
    double A = tri_area(Pk);
    double acc[9] = {0};
    for (long q = 0; q < nq; ++q) {
      double r[3];
      for (int d = 0; d < 3; ++d)
        r[d] = lam[3 * q] * Pk[d] + lam[3 * q + 1] * Pk[3 + d] + lam[3 * q + 2] * Pk[6 + d];
      double V0, V1[3];
      potentials(r, Qk, &V0, V1);
      double a[3][3], bq[3][3];
      for (int i = 0; i < 3; ++i)
        for (int d = 0; d < 3; ++d) { a[i][d] = r[d] - Pk[3 * i + d]; bq[i][d] = r[d] - Qk[3 * i + d]; }
      for (int i = 0; i < 3; ++i) {
        double aV1 = dot3(a[i], V1);
        for (int j = 0; j < 3; ++j) acc[3 * i + j] += w[q] * (aV1 + dot3(a[i], bq[j]) * V0);
      }
    }
    for (int i = 0; i < 9; ++i) out[9 * k + i] = A * acc[i];
  }
}

void oracle_blocks_product(long m, const double *P, const double *Q, long nq,
                           const double *lam, const double *w, double *out) {
#pragma omp parallel for schedule(static)
  for (long k = 0; k < m; ++k) {
    const double *Pk = P + 9 * k, *Qk = Q + 9 * k;
    double AP = tri_area(Pk), AQ = tri_area(Qk);
    double r[64][3], rp[64][3];
    long nn = nq > 64 ? 64 : nq;
    for (long q = 0; q < nn; ++q)
      for (int d = 0; d < 3; ++d) {
        r[q][d] = lam[3 * q] * Pk[d] + lam[3 * q + 1] * Pk[3 + d] + lam[3 * q + 2] * Pk[6 + d];
        rp[q][d] = lam[3 * q] * Qk[d] + lam[3 * q + 1] * Qk[3 + d] + lam[3 * q + 2] * Qk[6 + d];
      }
    double acc[9] = {0};
    for (long a = 0; a < nn; ++a) {
      for (long b = 0; b < nn; ++b) {
        double D[3] = {r[a][0] - rp[b][0], r[a][1] - rp[b][1], r[a][2] - rp[b][2]};
        double W = w[a] * w[b] / sqrt(dot3(D, D));
        for (int i = 0; i < 3; ++i) {
          double ai[3] = {r[a][0] - Pk[3 * i], r[a][1] - Pk[3 * i + 1], r[a][2] - Pk[3 * i + 2]};
          for (int j = 0; j < 3; ++j) {
            double bj[3] = {rp[b][0] - Qk[3 * j], rp[b][1] - Qk[3 * j + 1], rp[b][2] - Qk[3 * j + 2]};
            acc[3 * i + j] += W * dot3(ai, bj);
          }
        }
      }
    }
    for (int i = 0; i < 9; ++i) out[9 * k + i] = AP * AQ * acc[i];
  }
}
