// Flexible GMRES over all (frequency, port) right-hand sides at once
// (Sec. IV-A: GMRES on Eq. FinalME with the preconditioner of Eq. Precond),
// and the port solves / R-L extraction entry points (Sec. V).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <functional>
#include <map>
#include <set>

#include "engine.h"
#include "learned.h"
#include "precond.h"

using namespace pfft;

static void *pre_alloc(Precond *p, size_t bytes) {
  void *ptr = nullptr;
  hip_ok(hipMalloc(&ptr, bytes ? bytes : 16), "hipMalloc precond");
  p->allocs.push_back(ptr);
  return ptr;
}

template <typename V>
static V *pre_upload(Precond *p, const std::vector<V> &h) {
  V *d = (V *)pre_alloc(p, h.size() * sizeof(V));
  if (!h.empty()) hip_ok(hipMemcpy(d, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice), "upload precond");
  return d;
}

static void precond_free(Precond *p) {
  if (!p) return;
  for (void *q : p->allocs) hipFree(q);
  if (p->d_env) hipFree(p->d_env);
  if (p->d_diag) hipFree(p->d_diag);
  if (p->d_yinv) hipFree(p->d_yinv);
  if (p->d_work) hipFree(p->d_work);
  if (p->d_fidx) hipFree(p->d_fidx);
  if (p->d_tmp) hipFree(p->d_tmp);
  if (p->d_colenv) hipFree(p->d_colenv);
  if (p->d_full) hipFree(p->d_full);
  if (p->d_om) hipFree(p->d_om);
  if (p->d_status) hipFree(p->d_status);
  if (p->d_l11) hipFree(p->d_l11);
  if (p->d_l11t) hipFree(p->d_l11t);
  if (p->d_l21) hipFree(p->d_l21);
  if (p->d_uvec) hipFree(p->d_uvec);
  delete p;
}

int precond_uses_nd(const pfft_ctx *c) { return c->pre && c->pre->built ? (c->pre->ps.nd ? 1 : 0) : -1; }

void pfft_ctx_free(pfft_ctx *c) {
  precond_free(c->pre);
  learned_free(c);
  for (auto &w : c->ws)
    for (void *p : w.allocs) hipFree(p);
  for (int i = 0; i < pfft_ctx::kLanes; ++i) {
    if (c->lane[i]) hipStreamDestroy(c->lane[i]);
    if (c->ev_join[i]) hipEventDestroy(c->ev_join[i]);
  }
  if (c->ev_fork) hipEventDestroy(c->ev_fork);
  for (void *p : c->allocs) hipFree(p);
  delete c;
}

// Builds the structure once, factors every distinct frequency of omega[0..R)
// and uploads the per-RHS factor index.
Precond *pfft::precond_prepare(pfft_ctx *c, int R, const double *omega, hipStream_t st) {
  if (c->pre && c->pre->built && c->pre->nd_mode != c->plans.nd) {
    // the ordering plan changed: rebuild structure and factors
    hip_ok(hipStreamSynchronize(st), "precond rebuild sync");
    precond_free(c->pre);
    c->pre = nullptr;
  }
  if (!c->pre) c->pre = new Precond();
  Precond *P = c->pre;
  const HostModel &m = c->m;
  if (!P->built) {
    P->nd_mode = c->plans.nd;
    build_precond_struct(m, P->ps, P->nd_mode);
    if (std::max(P->ps.W, P->ps.Wc) + 8 >= 4096)
      throw SetupError{PFFT_EINVAL, "preconditioner envelope wider than 4087"};
    PrecondDev &d = P->dev;
    const PrecondStruct &ps = P->ps;
    d.nu = ps.nu;
    d.ncomp = ps.ncomp;
    d.W = ps.W;
    d.Wc = ps.Wc;
    d.pr = ps.pr;
    d.pc = ps.pc;
    d.clast = pre_upload(P, ps.clast);
    d.col_off = pre_upload(P, ps.col_off);
    d.nnz_col = (int64_t)ps.nu * ps.pc;
    d.b = m.b;
    d.l = m.l;
    d.p = m.p;
    d.comp_off = pre_upload(P, ps.comp_off);
    d.comp_mid = pre_upload(P, ps.comp_mid);
    d.nnz_full = ps.env_off[ps.nu];
    d.first = pre_upload(P, ps.first);
    d.env_off = pre_upload(P, ps.env_off);
    d.nnz_env = (int64_t)ps.nu * ps.pr;
    d.br_ru = pre_upload(P, ps.br_ru);
    d.br_rv = pre_upload(P, ps.br_rv);
    d.br_link = pre_upload(P, ps.br_link);
    d.br_offu = pre_upload(P, ps.br_offu);
    d.br_offv = pre_upload(P, ps.br_offv);
    d.inc_off = pre_upload(P, ps.inc_off);
    d.inc_br = pre_upload(P, ps.inc_br);
    d.inc_sg = pre_upload(P, ps.inc_sg);
    d.src_off = pre_upload(P, ps.src_off);
    d.src_br = pre_upload(P, ps.src_br);
    d.src_sg = pre_upload(P, ps.src_sg);
    d.link_kind = pre_upload(P, ps.link_kind);
    d.port_loop = pre_upload(P, ps.port_loop);
    // diagonals for the device factorization
    std::vector<double> gd(m.b, 0.0);
    for (int e = 0; e < m.b; ++e)
      for (int q = 0; q < 5; ++q)
        if (m.gram_col[5 * e + q] == e) gd[e] += m.gram_val[5 * e + q];
    P->d_gdiag = pre_upload(P, gd);
    P->d_kdiag = pre_upload(P, m.kdiag);
    d.nd = ps.nd ? 1 : 0;
    if (ps.nd) {
      d.nsn = ps.nsn;
      d.nlvl = (int)ps.lvl_off.size() - 1;
      d.max_front = ps.max_front;
      d.sn_start = pre_upload(P, ps.sn_start);
      d.st_ids = pre_upload(P, ps.st_ids);
      d.st_pos = pre_upload(P, ps.st_pos);
      d.ch_off = pre_upload(P, ps.ch_off);
      d.ch_ids = pre_upload(P, ps.ch_ids);
      d.lvl_off = pre_upload(P, ps.lvl_off);
      d.lvl_sn = pre_upload(P, ps.lvl_sn);
      d.st_off = pre_upload(P, ps.st_off);
      d.l11_off = pre_upload(P, ps.l11_off);
      d.l21_off = pre_upload(P, ps.l21_off);
      d.nl11 = ps.l11_off[ps.nsn];
      d.nl21 = ps.l21_off[ps.nsn];
      d.nst_tot = ps.st_off[ps.nsn];
      d.lvl_off_host = P->ps.lvl_off.data();
      d.lvl_front_host = P->ps.lvl_front.data();
    }
    P->built = true;
  }
  // distinct frequencies of this batch
  std::vector<double> om(omega, omega + R);
  std::vector<double> uniq = om;
  std::sort(uniq.begin(), uniq.end());
  uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
  if (uniq != P->omegas || P->factor_plan != c->plans.factor) {
    const int nf = (int)uniq.size();
    const size_t ne = (size_t)P->ps.nu * P->ps.pr, nc = (size_t)P->ps.nu * P->ps.pc;
    const size_t nfull = P->ps.env_off[P->ps.nu];
    if (nf > P->cap_f) {
      hip_ok(hipStreamSynchronize(st), "precond realloc sync");
      if (P->d_env) hipFree(P->d_env);
      if (P->d_diag) hipFree(P->d_diag);
      if (P->d_yinv) hipFree(P->d_yinv);
      if (P->d_colenv) hipFree(P->d_colenv);
      if (P->d_full) hipFree(P->d_full);
      if (P->d_om) hipFree(P->d_om);
      if (P->d_status) hipFree(P->d_status);
      P->d_env = P->d_diag = P->d_yinv = P->d_colenv = P->d_full = nullptr;
      P->d_om = nullptr;
      P->d_status = nullptr;
      P->cap_f = 0;
      hip_ok(hipMalloc(&P->d_full, std::max<size_t>(16, nfull * nf * sizeof(double2))), "hipMalloc full");
      hip_ok(hipMalloc(&P->d_env, std::max<size_t>(16, ne * nf * sizeof(double2))), "hipMalloc env");
      hip_ok(hipMalloc(&P->d_colenv, std::max<size_t>(16, nc * nf * sizeof(double2))), "hipMalloc colenv");
      hip_ok(hipMalloc(&P->d_diag, std::max<size_t>(16, (size_t)P->ps.nu * nf * sizeof(double2))), "hipMalloc diag");
      hip_ok(hipMalloc(&P->d_yinv, (size_t)m.b * nf * sizeof(double2)), "hipMalloc yinv");
      hip_ok(hipMalloc(&P->d_om, (size_t)nf * sizeof(double)), "hipMalloc omegas");
      hip_ok(hipMalloc(&P->d_status, (size_t)nf * (P->ps.ncomp + 1) * sizeof(int)), "hipMalloc status");
      P->cap_f = nf;
    }
    if (P->ps.nd) {
      // supernodal factors on the host (each factorization is parallel inside)
      const PrecondStruct &ps = P->ps;
      const size_t n11 = ps.l11_off[ps.nsn], n21 = ps.l21_off[ps.nsn];
      std::vector<std::complex<double>> a11(nf * n11), a11t(nf * n11), a21(nf * n21),
          dg((size_t)nf * ps.nu), yi((size_t)nf * m.b);
      for (int f = 0; f < nf; ++f) {
        std::vector<std::complex<double>> e1, e2, e3, d1, y1;
        if (!factor_precond_nd(m, ps, uniq[f], c->sigma, c->mu_r, e1, e2, e3, d1, y1))
          throw SetupError{PFFT_EFACTOR, "zero pivot in the nodal factorization"};
        std::copy(e1.begin(), e1.end(), a11.begin() + f * n11);
        std::copy(e2.begin(), e2.end(), a11t.begin() + f * n11);
        std::copy(e3.begin(), e3.end(), a21.begin() + f * n21);
        std::copy(d1.begin(), d1.end(), dg.begin() + (size_t)f * ps.nu);
        std::copy(y1.begin(), y1.end(), yi.begin() + (size_t)f * m.b);
      }
      hip_ok(hipStreamSynchronize(st), "precond sync");
      P->omegas.clear();
      if (P->d_l11) hipFree(P->d_l11);
      if (P->d_l11t) hipFree(P->d_l11t);
      if (P->d_l21) hipFree(P->d_l21);
      P->d_l11 = P->d_l11t = P->d_l21 = nullptr;
      hip_ok(hipMalloc(&P->d_l11, std::max<size_t>(16, nf * n11 * sizeof(double2))), "hipMalloc nd l11");
      hip_ok(hipMalloc(&P->d_l11t, std::max<size_t>(16, nf * n11 * sizeof(double2))), "hipMalloc nd l11t");
      hip_ok(hipMalloc(&P->d_l21, std::max<size_t>(16, nf * n21 * sizeof(double2))), "hipMalloc nd l21");
      if (n11) {
        hip_ok(hipMemcpy(P->d_l11, a11.data(), nf * n11 * sizeof(double2), hipMemcpyHostToDevice), "l11");
        hip_ok(hipMemcpy(P->d_l11t, a11t.data(), nf * n11 * sizeof(double2), hipMemcpyHostToDevice), "l11t");
      }
      if (n21) hip_ok(hipMemcpy(P->d_l21, a21.data(), nf * n21 * sizeof(double2), hipMemcpyHostToDevice), "l21");
      if (ps.nu)
        hip_ok(hipMemcpy(P->d_diag, dg.data(), (size_t)ps.nu * nf * sizeof(double2), hipMemcpyHostToDevice), "diag");
      hip_ok(hipMemcpy(P->d_yinv, yi.data(), (size_t)m.b * nf * sizeof(double2), hipMemcpyHostToDevice), "yinv");
      P->dev.l11 = P->d_l11;
      P->dev.l11t = P->d_l11t;
      P->dev.l21 = P->d_l21;
    } else if (c->plans.factor == 0 && factor_device_ok(P->ps)) {
      // device factorization, ordered after earlier work on st that reads the old factors
      hip_ok(hipMemcpyAsync(P->d_om, uniq.data(), nf * sizeof(double), hipMemcpyHostToDevice, st), "omegas");
      FactorArgs fa;
      fa.nu = P->ps.nu;
      fa.b = m.b;
      fa.W = std::max(P->ps.W, 1);
      fa.Wc = std::max(P->ps.Wc, 1);
      fa.pr = P->ps.pr;
      fa.pc = P->ps.pc;
      fa.ncomp = P->ps.ncomp;
      fa.nf = nf;
      fa.comp_off = P->dev.comp_off;
      fa.comp_mid = P->dev.comp_mid;
      fa.first = P->dev.first;
      fa.inc_off = P->dev.inc_off;
      fa.inc_br = P->dev.inc_br;
      fa.br_ru = P->dev.br_ru;
      fa.br_rv = P->dev.br_rv;
      fa.env_off = P->dev.env_off;
      fa.nnz_full = (int64_t)nfull;
      fa.gdiag = P->d_gdiag;
      fa.kdiag = P->d_kdiag;
      fa.omega = P->d_om;
      fa.sigma = c->sigma;
      fa.mu_r = c->mu_r;
      fa.env = P->d_env;
      fa.colenv = P->d_colenv;
      fa.full = P->d_full;
      fa.diag = P->d_diag;
      fa.yinv = P->d_yinv;
      fa.status = P->d_status;
      factor_precond_device(fa, st);
      std::vector<int> stat((size_t)nf * (P->ps.ncomp + 1));
      hip_ok(hipMemcpyAsync(stat.data(), P->d_status, stat.size() * sizeof(int), hipMemcpyDeviceToHost, st),
             "factor status");
      hip_ok(hipStreamSynchronize(st), "factor sync");
      P->omegas.clear();   // no valid factors until the check passes
      for (int v : stat)
        if (v) throw SetupError{PFFT_EFACTOR, "zero pivot in the nodal factorization"};
    } else {
      std::vector<std::complex<double>> env(nf * ne), dg((size_t)nf * P->ps.nu), yi((size_t)nf * m.b),
          ce((size_t)nf * nc), fe((size_t)nf * nfull);
      int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
      for (int f = 0; f < nf; ++f) {
        std::vector<std::complex<double>> e1, d1, y1, c1, f1;
        if (!factor_precond(m, P->ps, uniq[f], c->sigma, c->mu_r, e1, d1, y1, c1, f1)) {
          ++bad;
          continue;
        }
        std::copy(e1.begin(), e1.end(), env.begin() + (size_t)f * ne);
        std::copy(d1.begin(), d1.end(), dg.begin() + (size_t)f * P->ps.nu);
        std::copy(y1.begin(), y1.end(), yi.begin() + (size_t)f * m.b);
        std::copy(c1.begin(), c1.end(), ce.begin() + (size_t)f * nc);
        std::copy(f1.begin(), f1.end(), fe.begin() + (size_t)f * nfull);
      }
      if (bad) throw SetupError{PFFT_EFACTOR, "zero pivot in the nodal factorization"};
      // 64-entry layouts: the unit self entry of the register-window solve
      // in the last (padding) slot of every row, as the device assembly
      // writes it
      for (int f = 0; f < nf; ++f)
        for (int i = 0; i < P->ps.nu; ++i) {
          if (P->ps.pr == 64) env[(size_t)f * ne + (size_t)i * 64 + 63] = 1.0;
          if (P->ps.pc == 64) ce[(size_t)f * nc + (size_t)i * 64 + 63] = 1.0;
        }
      hip_ok(hipStreamSynchronize(st), "precond sync");
      P->omegas.clear();
      if (ne) hip_ok(hipMemcpy(P->d_env, env.data(), ne * nf * sizeof(double2), hipMemcpyHostToDevice), "env");
      if (P->ps.nu)
        hip_ok(hipMemcpy(P->d_diag, dg.data(), (size_t)P->ps.nu * nf * sizeof(double2), hipMemcpyHostToDevice),
               "diag");
      hip_ok(hipMemcpy(P->d_yinv, yi.data(), (size_t)m.b * nf * sizeof(double2), hipMemcpyHostToDevice), "yinv");
      if (nc) hip_ok(hipMemcpy(P->d_colenv, ce.data(), nc * nf * sizeof(double2), hipMemcpyHostToDevice), "colenv");
      if (nfull) hip_ok(hipMemcpy(P->d_full, fe.data(), nfull * nf * sizeof(double2), hipMemcpyHostToDevice), "full");
    }
    P->factor_plan = c->plans.factor;
    P->omegas = uniq;
    P->fidx_host.clear();
    P->dev.env = P->d_env;
    P->dev.diag = P->d_diag;
    P->dev.yinv = P->d_yinv;
    P->dev.colenv = P->d_colenv;
    P->dev.full = P->d_full;
    P->dev.nf = nf;
  }
  if (R > P->cap_R) {
    hip_ok(hipStreamSynchronize(st), "precond realloc sync");
    if (P->d_work) hipFree(P->d_work);
    if (P->d_fidx) hipFree(P->d_fidx);
    if (P->d_tmp) hipFree(P->d_tmp);
    hip_ok(hipMalloc(&P->d_work, std::max<size_t>(16, (size_t)R * P->ps.nu * sizeof(double2))), "hipMalloc work");
    hip_ok(hipMalloc(&P->d_fidx, (size_t)R * sizeof(int)), "hipMalloc fidx");
    hip_ok(hipMalloc(&P->d_tmp, (size_t)R * m.l * sizeof(double2)), "hipMalloc tmp");
    if (P->ps.nd) {
      if (P->d_uvec) hipFree(P->d_uvec);
      P->d_uvec = nullptr;
      hip_ok(hipMalloc(&P->d_uvec, std::max<size_t>(16, (size_t)R * P->ps.st_off[P->ps.nsn] * sizeof(double2))),
             "hipMalloc nd updates");
      P->dev.uvec = P->d_uvec;
    }
    P->cap_R = R;
    P->fidx_host.clear();
  }
  P->dev.ldl_plan = c->plans.ldl;
  std::vector<int> fidx(R);
  for (int r = 0; r < R; ++r)
    fidx[r] = (int)(std::lower_bound(P->omegas.begin(), P->omegas.end(), om[r]) - P->omegas.begin());
  if (fidx != P->fidx_host) {
    hip_ok(hipMemcpyAsync(P->d_fidx, fidx.data(), R * sizeof(int), hipMemcpyHostToDevice, st), "fidx");
    hip_ok(hipStreamSynchronize(st), "fidx sync");
    P->fidx_host = fidx;
  }
  return P;
}

// P^-1 y for right-hand sides [0, R), split over the stream lanes
static void precond_split(pfft_ctx *c, Precond *P, int R, const double2 *y, double2 *z, hipStream_t st) {
  const size_t l = c->m.l, nu = P->ps.nu;
  c->run_split(R, st, [&](int r0, int rn, hipStream_t s2, Workspace &) {
    precond_apply(P->dev, P->d_fidx + r0, y + r0 * l, z + r0 * l, P->d_work + r0 * nu, rn, s2);
  });
}

pfft_status pfft_internal_precond_matvec(pfft_ctx *c, int R, const double *omega, int flags, const double2 *x,
                                         double2 *y, hipStream_t st) {
  Precond *P = precond_prepare(c, R, omega, st);
  const size_t l = c->m.l, nu = P->ps.nu;
  if (flags & PFFT_LEARNED_ONLY) {
    c->timer.begin(ST_PRECOND, st);
    if (!learned_apply(c, R, omega, x, y, nullptr, st)) precond_apply(P->dev, P->d_fidx, x, y, P->d_work, R, st);
    c->timer.end(st);
  } else if (flags & PFFT_PRECOND_ONLY) {
    c->timer.begin(ST_PRECOND, st);
    precond_split(c, P, R, x, y, st);
    c->timer.end(st);
  } else {
    // Z_l x into the preconditioner scratch, then P^-1, per stream lane
    const int mf = flags & (PFFT_FAR_ONLY | PFFT_NEAR_ONLY);
    c->run_split(R, st, [&](int r0, int rn, hipStream_t s2, Workspace &w) {
      c->matvec_range(w, rn, omega + r0, 1, mf, x + r0 * l, P->d_tmp + r0 * l, s2);
      c->timer.begin(ST_PRECOND, s2);
      precond_apply(P->dev, P->d_fidx + r0, P->d_tmp + r0 * l, y + r0 * l, P->d_work + r0 * nu, rn, s2);
      c->timer.end(s2);
    });
  }
  hip_ok(hipGetLastError(), "precond launch");
  return PFFT_OK;
}

// ---------------------------------------------------------------------------
// batched FGMRES kernels
// ---------------------------------------------------------------------------
// h[r][j] = <V[r][j], w[r]> (conjugate-linear in V) for j < k
__global__ void k_mdot(const double2 *V, const double2 *w, double2 *h, int l, int ldV, int k, int hstride,
                       const uint8_t *active) {
  int j = blockIdx.x, r = blockIdx.y;
  if (active && !active[r]) return;
  const double2 *v = V + ((size_t)r * ldV + j) * l;
  const double2 *ww = w + (size_t)r * l;
  double sx = 0, sy = 0;
  for (int i = threadIdx.x; i < l; i += blockDim.x) {
    double2 a = v[i], b = ww[i];
    sx += a.x * b.x + a.y * b.y;
    sy += a.x * b.y - a.y * b.x;
  }
  __shared__ double shx[256], shy[256];
  shx[threadIdx.x] = sx;
  shy[threadIdx.x] = sy;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) { shx[threadIdx.x] += shx[threadIdx.x + s]; shy[threadIdx.x] += shy[threadIdx.x + s]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) h[(size_t)r * hstride + j] = make_double2(shx[0], shy[0]);
}

// w[r] -= sum_{j<k} h[r][j] V[r][j];  acc[r][j] += h[r][j] (optional)
__global__ void k_maxpy(const double2 *V, double2 *w, const double2 *h, int l, int ldV, int k, int hstride,
                        const uint8_t *active) {
  int r = blockIdx.y;
  if (active && !active[r]) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= l) return;
  double2 acc = w[(size_t)r * l + i];
  for (int j = 0; j < k; ++j) {
    double2 a = V[((size_t)r * ldV + j) * l + i], c = h[(size_t)r * hstride + j];
    acc.x -= c.x * a.x - c.y * a.y;
    acc.y -= c.x * a.y + c.y * a.x;
  }
  w[(size_t)r * l + i] = acc;
}

// dst[r] = src[r] * s[r]   (s real, 1/norm; 0 when the norm vanished)
__global__ void k_scale(const double2 *src, double2 *dst, const double2 *nrm2, int l, int dst_ld, int src_ld) {
  int r = blockIdx.y;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= l) return;
  double n = sqrt(fmax(nrm2[r].x, 0.0));
  double s = n > 0 ? 1.0 / n : 0.0;
  double2 v = src[(size_t)r * src_ld + i];
  dst[(size_t)r * dst_ld + i] = make_double2(v.x * s, v.y * s);
}

// Column k of H: h (first pass) + h2 (second pass), H[k+1][k] = norm;
// previous rotations, new rotation, residual estimate |g[k+1]|.
__global__ void k_givens(double2 *H, const double2 *h1, const double2 *h2, const double2 *nrm2, double2 *cs,
                         double2 *sn, double2 *g, double *resid, int k, int m, int R, double2 *Hraw) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double2 *Hc = H + (size_t)r * (m + 1) * m;   // H[i][k] at Hc[i * m + k]
  for (int i = 0; i <= k; ++i) {
    double2 a = h1[(size_t)r * (m + 1) + i], b = h2[(size_t)r * (m + 1) + i];
    Hc[i * m + k] = make_double2(a.x + b.x, a.y + b.y);
  }
  double nn = sqrt(fmax(nrm2[r].x, 0.0));
  Hc[(k + 1) * m + k] = make_double2(nn, 0.0);
  if (Hraw) {   // unrotated column k (Arnoldi relation Z_l z_k = sum_i H[i][k] v_i)
    double2 *Hr = Hraw + (size_t)r * (m + 1) * m;
    for (int i = 0; i <= k + 1; ++i) Hr[i * m + k] = Hc[i * m + k];
  }
  double2 *c = cs + (size_t)r * (m + 1), *s = sn + (size_t)r * (m + 1), *gg = g + (size_t)r * (m + 1);
  for (int i = 0; i < k; ++i) {
    double2 x = Hc[i * m + k], y = Hc[(i + 1) * m + k];
    double2 ci = c[i], si = s[i];
    // (x, y) -> (conj(c) x + conj(s) y, -s x + c y)
    double2 t = make_double2(ci.x * x.x + ci.y * x.y + si.x * y.x + si.y * y.y,
                             ci.x * x.y - ci.y * x.x + si.x * y.y - si.y * y.x);
    double2 u = make_double2(-(si.x * x.x - si.y * x.y) + (ci.x * y.x - ci.y * y.y),
                             -(si.x * x.y + si.y * x.x) + (ci.x * y.y + ci.y * y.x));
    Hc[i * m + k] = t;
    Hc[(i + 1) * m + k] = u;
  }
  double2 a = Hc[k * m + k], b = Hc[(k + 1) * m + k];
  double den = sqrt(a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y);
  double2 ck = den > 0 ? make_double2(a.x / den, a.y / den) : make_double2(1, 0);
  double2 sk = den > 0 ? make_double2(b.x / den, b.y / den) : make_double2(0, 0);
  c[k] = ck;
  s[k] = sk;
  Hc[k * m + k] = make_double2(den, 0.0);
  Hc[(k + 1) * m + k] = make_double2(0.0, 0.0);
  double2 gk = gg[k];
  gg[k + 1] = make_double2(-(sk.x * gk.x - sk.y * gk.y), -(sk.x * gk.y + sk.y * gk.x));
  gg[k] = make_double2(ck.x * gk.x + ck.y * gk.y, ck.x * gk.y - ck.y * gk.x);
  resid[r] = sqrt(gg[k + 1].x * gg[k + 1].x + gg[k + 1].y * gg[k + 1].y);
}

// y = H[0:kr,0:kr]^-1 g[0:kr] (upper triangular), kr per RHS
__global__ void k_backsolve(const double2 *H, const double2 *g, double2 *y, const int *kr, int m, int R) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const double2 *Hc = H + (size_t)r * (m + 1) * m;
  const double2 *gg = g + (size_t)r * (m + 1);
  double2 *yy = y + (size_t)r * (m + 1);
  int K = kr[r];
  for (int i = K - 1; i >= 0; --i) {
    double2 acc = gg[i];
    for (int j = i + 1; j < K; ++j) {
      double2 h = Hc[i * m + j], v = yy[j];
      acc.x -= h.x * v.x - h.y * v.y;
      acc.y -= h.x * v.y + h.y * v.x;
    }
    double2 d = Hc[i * m + i];
    double den = d.x * d.x + d.y * d.y;
    yy[i] = den > 0 ? make_double2((acc.x * d.x + acc.y * d.y) / den, (acc.y * d.x - acc.x * d.y) / den)
                    : make_double2(0, 0);
  }
}

// x[r] += sum_{j<kr} y[r][j] Z[r][j]
__global__ void k_xupdate(double2 *x, const double2 *Z, const double2 *y, const int *kr, int l, int m) {
  int r = blockIdx.y;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= l) return;
  double2 acc = x[(size_t)r * l + i];
  for (int j = 0; j < kr[r]; ++j) {
    double2 zz = Z[((size_t)r * m + j) * l + i], c = y[(size_t)r * (m + 1) + j];
    acc.x += c.x * zz.x - c.y * zz.y;
    acc.y += c.x * zz.y + c.y * zz.x;
  }
  x[(size_t)r * l + i] = acc;
}

__global__ void k_residual(const double2 *b, const double2 *Ax, double2 *r, int n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)n) return;
  r[i] = make_double2(b[i].x - Ax[i].x, b[i].y - Ax[i].y);
}

__global__ void k_init_g(double2 *g, const double2 *nrm2, int m, int R) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  for (int i = 0; i <= m; ++i) g[(size_t)r * (m + 1) + i] = make_double2(0, 0);
  g[(size_t)r * (m + 1)] = make_double2(sqrt(fmax(nrm2[r].x, 0.0)), 0.0);
}

// ---------------------------------------------------------------------------
// FGMRES driver
// ---------------------------------------------------------------------------
struct Fgmres {
  int R, l, m;
  double2 *V, *Z, *H, *cs, *sn, *g, *h1, *h2, *nrm, *yv, *x, *w, *b, *Ax;
  double2 *Hraw = nullptr;   // optional unrotated Hessenberg [R][m+1][m]
  double *resid;
  int *kr;
  std::vector<void *> al;
  void *alloc(size_t bytes) {
    void *p = nullptr;
    hip_ok(hipMalloc(&p, bytes ? bytes : 16), "hipMalloc gmres");
    al.push_back(p);
    return p;
  }
  Fgmres(int R_, int l_, int m_) : R(R_), l(l_), m(m_) {
    size_t vec = (size_t)R * l * sizeof(double2);
    V = (double2 *)alloc(vec * (m + 1));
    Z = (double2 *)alloc(vec * m);
    H = (double2 *)alloc((size_t)R * (m + 1) * m * sizeof(double2));
    cs = (double2 *)alloc((size_t)R * (m + 1) * sizeof(double2));
    sn = (double2 *)alloc((size_t)R * (m + 1) * sizeof(double2));
    g = (double2 *)alloc((size_t)R * (m + 1) * sizeof(double2));
    h1 = (double2 *)alloc((size_t)R * (m + 1) * sizeof(double2));
    h2 = (double2 *)alloc((size_t)R * (m + 1) * sizeof(double2));
    yv = (double2 *)alloc((size_t)R * (m + 1) * sizeof(double2));
    nrm = (double2 *)alloc((size_t)R * sizeof(double2));
    x = (double2 *)alloc(vec);
    w = (double2 *)alloc(vec);
    b = (double2 *)alloc(vec);
    Ax = (double2 *)alloc(vec);
    resid = (double *)alloc((size_t)R * sizeof(double));
    kr = (int *)alloc((size_t)R * sizeof(int));
  }
  ~Fgmres() {
    for (void *p : al) hipFree(p);
  }
};

// Solves Z_l(omega_r) x_r = b_r for all r; b is already in F.b.  precond: 0,
// 1 (P), 2 (P + learned).  Returns per-RHS iterations and true residuals.
// left: GMRES on P^-1 Z_l x = P^-1 b (precond 0 or 1): the basis vectors are
// the update directions (Z holds copies of V), every Arnoldi step is a product
// followed by P^-1, and the residual that is estimated, tested and reported
// is the preconditioned one, relative to |P^-1 b|.
// rec (optional) receives, for the first cycle, each RHS's Krylov length and
// residual estimates |g_{k+1}| after every step.
struct FirstCycle {
  std::vector<int> k;
  std::vector<std::vector<double>> res;
  std::vector<double> bnorm;
};
static void fgmres(pfft_ctx *c, Fgmres &F, const double *omega, double tol, int maxit, int precond,
                   std::vector<int> &iters, std::vector<double> &relres, hipStream_t st,
                   FirstCycle *rec = nullptr, bool left = false) {
  const int R = F.R, l = F.l, m = F.m;
  const dim3 gl((l + 255) / 256, R);
  if (precond != 1) left = false;   // without P both forms are plain GMRES
  Precond *P = precond ? precond_prepare(c, R, omega, st) : nullptr;
  hip_ok(hipMemsetAsync(F.x, 0, (size_t)R * l * sizeof(double2), st), "x0");
  iters.assign(R, 0);
  relres.assign(R, 1.0);
  std::vector<double> bnorm(R), res(R);
  std::vector<uint8_t> done(R, 0);
  std::vector<int> kconv(R, 0);
  // learned correction judged against the plain preconditioner's convergence
  // factor per step: a right-hand side whose residual estimate falls more
  // slowly over two steps is switched back to plain P for the rest of the solve
  std::vector<uint8_t> use_l(R, precond == 2 ? 1 : 0);
  const double judge = precond == 2 ? learned_judge_factor(c) : 0.0;
  std::vector<std::vector<double>> seq(R);
  // The preconditioner apply (F.w -> F.Ax) and the product (F.Ax -> F.w) use
  // fixed buffers in every iteration: after one eager iteration (which sets
  // up workspaces and uploads the per-RHS coefficients) they are captured as
  // HIP graphs on a private stream and replayed on st.
  hipStream_t cs = nullptr;
  hipGraphExec_t g_pre = nullptr, g_mv = nullptr;
  bool want_graphs = c->plans.graphs && !c->timer.on && c->chunk_for(R) >= R;
  // right: w -> P^-1 -> Ax -> Z_l -> w;  left: w -> Z_l -> Ax -> P^-1 -> w
  auto run_pre = [&](hipStream_t s2) {
    if (left)
      precond_split(c, P, R, F.Ax, F.w, s2);
    else
      precond_split(c, P, R, F.w, F.Ax, s2);
  };
  auto run_mv = [&](hipStream_t s2) {
    if (left)
      c->matvec(R, omega, 1, 0, F.w, F.Ax, s2);
    else
      c->matvec(R, omega, 1, 0, F.Ax, F.w, s2);
  };
  const size_t vbytes = (size_t)R * l * sizeof(double2);
  // left: P^-1 applied to a residual in w (through Ax, back into w)
  auto left_precond_w = [&]() {
    if (!precond) return;
    hip_ok(hipMemcpyAsync(F.Ax, F.w, vbytes, hipMemcpyDeviceToDevice, st), "left residual");
    if (g_pre)
      hip_ok(hipGraphLaunch(g_pre, st), "graph launch");
    else
      run_pre(st);
  };
  auto capture = [&](auto &&fn, hipGraphExec_t &exec) {
    hipGraph_t gr = nullptr;
    hip_ok(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
    try {
      fn(cs);
    } catch (...) {
      hipStreamEndCapture(cs, &gr);
      if (gr) hipGraphDestroy(gr);
      throw;
    }
    hip_ok(hipStreamEndCapture(cs, &gr), "end capture");
    const hipError_t e = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
    hipGraphDestroy(gr);
    hip_ok(e, "graph instantiate");
  };
  auto release_graphs = [&]() {
    if (g_pre) hipGraphExecDestroy(g_pre);
    if (g_mv) hipGraphExecDestroy(g_mv);
    if (cs) hipStreamDestroy(cs);
    g_pre = g_mv = nullptr;
    cs = nullptr;
  };
  // residual r0 = b (x0 = 0) in w; left: P^-1 b
  hip_ok(hipMemcpyAsync(F.w, F.b, vbytes, hipMemcpyDeviceToDevice, st), "r0");
  if (left) left_precond_w();
  // |b| (left: |P^-1 b|)
  k_mdot<<<dim3(1, R), 256, 0, st>>>(F.w, F.w, F.nrm, l, 1, 1, 1, nullptr);
  {
    std::vector<double2> n2(R);
    hip_ok(hipMemcpyAsync(n2.data(), F.nrm, R * sizeof(double2), hipMemcpyDeviceToHost, st), "bnorm");
    hip_ok(hipStreamSynchronize(st), "bnorm sync");
    for (int r = 0; r < R; ++r) bnorm[r] = std::sqrt(std::max(n2[r].x, 0.0));
  }
  int total = 0;
  if (rec) {
    rec->k.assign(R, 0);
    rec->res.assign(R, {});
    rec->bnorm = bnorm;
  }
  bool all_done = false;
  bool first = true;
  while (total < maxit && !all_done) {
    std::vector<uint8_t> done_before = done;
    std::vector<int> kthis(R, 0);   // Krylov length at convergence in this cycle
    k_mdot<<<dim3(1, R), 256, 0, st>>>(F.w, F.w, F.nrm, l, 1, 1, 1, nullptr);
    k_init_g<<<(R + 63) / 64, 64, 0, st>>>(F.g, F.nrm, m, R);
    k_scale<<<gl, 256, 0, st>>>(F.w, F.V, F.nrm, l, (m + 1) * l, l);
    int k = 0;
    for (; k < m && total + k < maxit; ++k) {
      // z_k = M(v_k): gather v_k of every RHS into w (contiguous), apply, store in Z
      hip_ok(hipMemcpy2DAsync(F.w, l * sizeof(double2), F.V + (size_t)k * l, (m + 1) * l * sizeof(double2),
                              l * sizeof(double2), R, hipMemcpyDeviceToDevice, st),
             "gather v");
      double2 *zk = F.Ax;  // contiguous [R][l]
      if (left) {
        zk = F.w;          // the update direction is v_k itself
      } else if (precond == 2 && learned_apply(c, R, omega, F.w, zk, use_l.data(), st)) {
      } else if (precond) {
        if (g_pre)
          hip_ok(hipGraphLaunch(g_pre, st), "graph launch");
        else
          run_pre(st);
      } else {
        hip_ok(hipMemcpyAsync(zk, F.w, (size_t)R * l * sizeof(double2), hipMemcpyDeviceToDevice, st), "noprec");
      }
      hip_ok(hipMemcpy2DAsync(F.Z + (size_t)k * l, m * l * sizeof(double2), zk, l * sizeof(double2),
                              l * sizeof(double2), R, hipMemcpyDeviceToDevice, st),
             "store z");
      // w = Z_l z_k  (left: w = P^-1 Z_l v_k)
      if (g_mv)
        hip_ok(hipGraphLaunch(g_mv, st), "graph launch");
      else
        run_mv(st);
      if (left && precond) {
        if (g_pre)
          hip_ok(hipGraphLaunch(g_pre, st), "graph launch");
        else
          run_pre(st);
      }
      if (want_graphs && !g_mv) {
        want_graphs = false;
        try {
          hip_ok(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
          hip_ok(hipStreamSynchronize(st), "pre-capture sync");
          capture(run_mv, g_mv);
          if (precond == 1) capture(run_pre, g_pre);
        } catch (const DeviceError &) {
          (void)hipGetLastError();   // graphs are an optimisation: stay eager
          release_graphs();
        }
      }
      // classical Gram-Schmidt, twice
      k_mdot<<<dim3(k + 1, R), 256, 0, st>>>(F.V, F.w, F.h1, l, m + 1, k + 1, m + 1, nullptr);
      k_maxpy<<<gl, 256, 0, st>>>(F.V, F.w, F.h1, l, m + 1, k + 1, m + 1, nullptr);
      k_mdot<<<dim3(k + 1, R), 256, 0, st>>>(F.V, F.w, F.h2, l, m + 1, k + 1, m + 1, nullptr);
      k_maxpy<<<gl, 256, 0, st>>>(F.V, F.w, F.h2, l, m + 1, k + 1, m + 1, nullptr);
      k_mdot<<<dim3(1, R), 256, 0, st>>>(F.w, F.w, F.nrm, l, 1, 1, 1, nullptr);
      k_scale<<<gl, 256, 0, st>>>(F.w, F.V + (size_t)(k + 1) * l, F.nrm, l, (m + 1) * l, l);
      k_givens<<<(R + 63) / 64, 64, 0, st>>>(F.H, F.h1, F.h2, F.nrm, F.cs, F.sn, F.g, F.resid, k, m, R,
                                             F.Hraw);
      hip_ok(hipMemcpyAsync(res.data(), F.resid, R * sizeof(double), hipMemcpyDeviceToHost, st), "resid");
      hip_ok(hipStreamSynchronize(st), "resid sync");
      if (rec && first)
        for (int r = 0; r < R; ++r)
          if (!done[r]) rec->res[r].push_back(res[r]);
      for (int r = 0; r < R; ++r) {
        if (done[r]) continue;
        if (k == 0) seq[r].clear();
        seq[r].push_back(res[r]);
        const size_t n = seq[r].size();
        if (use_l[r] && judge > 0 && n >= 3 && !(std::sqrt(seq[r][n - 1] / seq[r][n - 3]) <= judge)) {
          use_l[r] = 0;
          learned_judged_off(c, 1);
        }
      }
      bool all = true;
      for (int r = 0; r < R; ++r) {
        // the Arnoldi estimate aims below tol; the true residual decides at
        // the end of the cycle
        if (!done[r] && res[r] <= 0.9 * tol * bnorm[r]) {
          done[r] = 1;
          kthis[r] = k + 1;
          iters[r] = total + k + 1;
        }
        all = all && done[r];
      }
      if (all) {
        ++k;
        break;
      }
    }
    // x += Z y: converged in this cycle -> its own length, converged before ->
    // unchanged, otherwise the full cycle
    std::vector<int> kr(R);
    for (int r = 0; r < R; ++r) kr[r] = done_before[r] ? 0 : (kthis[r] > 0 ? kthis[r] : k);
    if (rec && first) rec->k = kr;
    first = false;
    hip_ok(hipMemcpyAsync(F.kr, kr.data(), R * sizeof(int), hipMemcpyHostToDevice, st), "kr");
    k_backsolve<<<(R + 63) / 64, 64, 0, st>>>(F.H, F.g, F.yv, F.kr, m, R);
    k_xupdate<<<gl, 256, 0, st>>>(F.x, F.Z, F.yv, F.kr, l, m);
    total += k;
    // true residual: restart vector, convergence test and the reported residual
    c->matvec(R, omega, 1, 0, F.x, F.Ax, st);
    k_residual<<<(unsigned)(((size_t)R * l + 255) / 256), 256, 0, st>>>(F.b, F.Ax, F.w, R * l);
    if (left) left_precond_w();
    k_mdot<<<dim3(1, R), 256, 0, st>>>(F.w, F.w, F.nrm, l, 1, 1, 1, nullptr);
    {
      std::vector<double2> t2(R);
      hip_ok(hipMemcpyAsync(t2.data(), F.nrm, R * sizeof(double2), hipMemcpyDeviceToHost, st), "true norm");
      hip_ok(hipStreamSynchronize(st), "true norm sync");
      // a right-hand side whose estimate converged but whose true residual
      // (FP32 grid rounding) is above tol continues from its true residual
      for (int r = 0; r < R; ++r)
        if (done[r] && std::sqrt(std::max(t2[r].x, 0.0)) > tol * bnorm[r]) done[r] = 0;
    }
    all_done = std::all_of(done.begin(), done.end(), [](uint8_t v) { return v != 0; });
  }
  // final true residuals
  k_mdot<<<dim3(1, R), 256, 0, st>>>(F.w, F.w, F.nrm, l, 1, 1, 1, nullptr);
  std::vector<double2> n2(R);
  hip_ok(hipMemcpyAsync(n2.data(), F.nrm, R * sizeof(double2), hipMemcpyDeviceToHost, st), "final norm");
  hip_ok(hipStreamSynchronize(st), "final sync");
  release_graphs();
  for (int r = 0; r < R; ++r) {
    relres[r] = std::sqrt(std::max(n2[r].x, 0.0)) / (bnorm[r] > 0 ? bnorm[r] : 1.0);
    if (!done[r]) iters[r] = total;
  }
}

// right-hand sides of the port solves (Sec. V): 1 V on the driven port's
// source loop, frequency-major
static void port_rhs(const pfft_ctx *c, int nfreq, const double *freq_hz, std::vector<double> &omega,
                     std::vector<double2> &bh) {
  const int p = c->m.p, l = c->m.l, R = nfreq * p;
  omega.assign(R, 0.0);
  bh.assign((size_t)R * l, make_double2(0, 0));
  for (int f = 0; f < nfreq; ++f)
    for (int k = 0; k < p; ++k) {
      int r = f * p + k;
      omega[r] = 2.0 * M_PI * freq_hz[f];
      bh[(size_t)r * l + c->m.port_loop[k]] = make_double2(1.0, 0.0);
    }
}

void pfft::solve_ports_krylov(pfft_ctx *c, int nfreq, const double *freq_hz, double tol, int maxit,
                              const KrylovFn &done, hipStream_t st) {
  const int R = nfreq * c->m.p, l = c->m.l, m = maxit;
  Fgmres F(R, l, m);
  F.Hraw = (double2 *)F.alloc((size_t)R * (m + 1) * m * sizeof(double2));
  std::vector<double> omega;
  std::vector<double2> bh;
  port_rhs(c, nfreq, freq_hz, omega, bh);
  hip_ok(hipMemcpyAsync(F.b, bh.data(), bh.size() * sizeof(double2), hipMemcpyHostToDevice, st), "b");
  std::vector<int> iters;
  std::vector<double> relres;
  FirstCycle rec;
  fgmres(c, F, omega.data(), tol, maxit, 1, iters, relres, st, &rec);
  KrylovView kv;
  kv.R = R;
  kv.l = l;
  kv.m = m;
  kv.V = F.V;
  kv.Z = F.Z;
  kv.Hraw = F.Hraw;
  kv.x = F.x;
  kv.omega = omega.data();
  kv.k = rec.k;
  kv.res = rec.res;
  kv.bnorm = rec.bnorm;
  kv.relres = relres;
  done(kv);
  hip_ok(hipStreamSynchronize(st), "krylov sync");
}

static pfft_status solve_ports_any(const char *name, bool left, pfft_ctx *c, int32_t nfreq,
                                   const double *freq_hz, double tol, int32_t maxit, int32_t restart,
                                   int32_t precond, void *Y_out, int32_t *iters_out, double *relres_out,
                                   void *hip_stream, void *Il_dev = nullptr) {
  const std::string who = std::string(name) + ": ";
  if (!c || nfreq <= 0 || !freq_hz || !Y_out || !(tol > 0) || maxit <= 0 || restart <= 0 || precond < 0 ||
      precond > (left ? 1 : 2)) {
    set_error(who + "bad argument");
    return PFFT_EINVAL;
  }
  if (c->m.p == 0) {
    set_error(who + "the problem has no ports");
    return PFFT_EINVAL;
  }
  for (int f = 0; f < nfreq; ++f)
    if (!(freq_hz[f] > 0)) {
      set_error(who + "frequencies must be positive");
      return PFFT_EINVAL;
    }
  try {
    hip_ok(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t st = (hipStream_t)hip_stream;
    const int p = c->m.p, l = c->m.l, R = nfreq * p;
    const int m = std::min(restart, maxit);
    Fgmres F(R, l, m);
    std::vector<double> omega;
    std::vector<double2> bh;
    port_rhs(c, nfreq, freq_hz, omega, bh);
    hip_ok(hipMemcpyAsync(F.b, bh.data(), bh.size() * sizeof(double2), hipMemcpyHostToDevice, st), "b");
    std::vector<int> iters;
    std::vector<double> relres;
    fgmres(c, F, omega.data(), tol, maxit, precond, iters, relres, st, nullptr, left);
    std::vector<double2> xh((size_t)R * l);
    if (Il_dev)
      hip_ok(hipMemcpyAsync(Il_dev, F.x, xh.size() * sizeof(double2), hipMemcpyDeviceToDevice, st), "loop currents");
    hip_ok(hipMemcpyAsync(xh.data(), F.x, xh.size() * sizeof(double2), hipMemcpyDeviceToHost, st), "x");
    hip_ok(hipStreamSynchronize(st), "x sync");
    double2 *Y = (double2 *)Y_out;
    bool ok = true;
    for (int f = 0; f < nfreq; ++f)
      for (int k = 0; k < p; ++k) {
        int r = f * p + k;
        for (int j = 0; j < p; ++j) Y[((size_t)f * p + j) * p + k] = xh[(size_t)r * l + c->m.port_loop[j]];
        if (iters_out) iters_out[f * p + k] = iters[r];
        if (relres_out) relres_out[f * p + k] = relres[r];
        ok = ok && relres[r] <= tol * 1.0001 + 1e-15;
      }
    if (!ok) {
      set_error(who + "some right-hand sides did not reach the tolerance");
      return PFFT_ENOCONV;
    }
    return PFFT_OK;
  } catch (const DeviceError &e) {
    set_error(who + e.msg);
    return (pfft_status)e.code;
  } catch (const SetupError &e) {
    set_error(who + e.msg);
    return (pfft_status)e.code;
  }
}

extern "C" {

pfft_status solve_ports(pfft_ctx *c, int32_t nfreq, const double *freq_hz, double tol, int32_t maxit,
                        int32_t restart, int32_t precond, void *Y_out, int32_t *iters_out, double *relres_out,
                        void *hip_stream) {
  return solve_ports_any("solve_ports", false, c, nfreq, freq_hz, tol, maxit, restart, precond, Y_out, iters_out,
                         relres_out, hip_stream);
}

pfft_status solve_ports_loops(pfft_ctx *c, int32_t nfreq, const double *freq_hz, double tol, int32_t maxit,
                              int32_t restart, int32_t precond, void *Y_out, int32_t *iters_out, double *relres_out,
                              void *Il_dev, void *hip_stream) {
  if (!Il_dev) {
    set_error("solve_ports_loops: null loop-current buffer");
    return PFFT_EINVAL;
  }
  return solve_ports_any("solve_ports_loops", false, c, nfreq, freq_hz, tol, maxit, restart, precond, Y_out,
                         iters_out, relres_out, hip_stream, Il_dev);
}

pfft_status solve_ports_lgmres(pfft_ctx *c, int32_t nfreq, const double *freq_hz, double tol, int32_t maxit,
                               int32_t restart, int32_t precond, void *Y_out, int32_t *iters_out,
                               double *relres_out, void *hip_stream) {
  return solve_ports_any("solve_ports_lgmres", true, c, nfreq, freq_hz, tol, maxit, restart, precond, Y_out,
                         iters_out, relres_out, hip_stream);
}

}  // extern "C"
