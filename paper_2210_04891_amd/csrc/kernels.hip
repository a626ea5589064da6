// Device kernels of the pFFT loop-space matrix-vector product for gfx950.
//
// Every product is a gather (no atomics), so results are bitwise
// reproducible run to run.  Complex numbers are float2/double2 (re, im).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace pfft {

#define HIP_CHECK_LAUNCH() (void)hipGetLastError()

template <typename T>
__device__ __forceinline__ V2<T> cmk(T a, T b) {
  V2<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ V2<T> cadd(V2<T> a, V2<T> b) { return cmk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ V2<T> csub(V2<T> a, V2<T> b) { return cmk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ V2<T> cmul(V2<T> a, V2<T> b) {
  return cmk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ V2<T> cscale(V2<T> a, T s) { return cmk<T>(a.x * s, a.y * s); }

static inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

// ===========================================================================
// batched prefix sums (complex128), three phases, deterministic
// ===========================================================================
constexpr int SCAN_T = 256, SCAN_E = 4, SCAN_B = SCAN_T * SCAN_E;

size_t scan_partials_size(int len, int R) { return (size_t)cdiv(len, SCAN_B) * R; }

__global__ void k_scan_block_sums(const double2 *in, double2 *part, int len, int ld, int nblk) {
  int r = blockIdx.y, blk = blockIdx.x;
  const double2 *row = in + (size_t)r * ld;
  double sx = 0, sy = 0;
  int base = blk * SCAN_B + threadIdx.x * SCAN_E;
  for (int k = 0; k < SCAN_E; ++k)
    if (base + k < len) { sx += row[base + k].x; sy += row[base + k].y; }
  __shared__ double shx[SCAN_T], shy[SCAN_T];
  shx[threadIdx.x] = sx;
  shy[threadIdx.x] = sy;
  __syncthreads();
  for (int s = SCAN_T / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) { shx[threadIdx.x] += shx[threadIdx.x + s]; shy[threadIdx.x] += shy[threadIdx.x + s]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)r * nblk + blk] = make_double2(shx[0], shy[0]);
}

// exclusive scan of block sums, one workgroup per row
__global__ void k_scan_partials(double2 *part, int nblk) {
  int r = blockIdx.x;
  double2 *row = part + (size_t)r * nblk;
  __shared__ double shx[SCAN_T], shy[SCAN_T];
  double cx = 0, cy = 0;
  for (int c0 = 0; c0 < nblk; c0 += SCAN_T) {
    int i = c0 + threadIdx.x;
    double vx = i < nblk ? row[i].x : 0, vy = i < nblk ? row[i].y : 0;
    shx[threadIdx.x] = vx;
    shy[threadIdx.x] = vy;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
      double ax = threadIdx.x >= off ? shx[threadIdx.x - off] : 0;
      double ay = threadIdx.x >= off ? shy[threadIdx.x - off] : 0;
      __syncthreads();
      shx[threadIdx.x] += ax;
      shy[threadIdx.x] += ay;
      __syncthreads();
    }
    double incx = shx[threadIdx.x], incy = shy[threadIdx.x];
    if (i < nblk) row[i] = make_double2(cx + incx - vx, cy + incy - vy);
    double tx = shx[SCAN_T - 1], ty = shy[SCAN_T - 1];
    __syncthreads();
    cx += tx;
    cy += ty;
  }
}

__global__ void k_scan_final(const double2 *in, double2 *out, const double2 *part, int len, int ld,
                             int nblk, int inclusive) {
  int r = blockIdx.y, blk = blockIdx.x;
  const double2 *row = in + (size_t)r * ld;
  double2 *orow = out + (size_t)r * ld;
  int base = blk * SCAN_B + threadIdx.x * SCAN_E;
  double vx[SCAN_E], vy[SCAN_E];
  double sx = 0, sy = 0;
  for (int k = 0; k < SCAN_E; ++k) {
    bool ok = base + k < len;
    vx[k] = ok ? row[base + k].x : 0;
    vy[k] = ok ? row[base + k].y : 0;
    sx += vx[k];
    sy += vy[k];
  }
  __shared__ double shx[SCAN_T], shy[SCAN_T];
  shx[threadIdx.x] = sx;
  shy[threadIdx.x] = sy;
  __syncthreads();
  for (int off = 1; off < SCAN_T; off <<= 1) {
    double ax = threadIdx.x >= off ? shx[threadIdx.x - off] : 0;
    double ay = threadIdx.x >= off ? shy[threadIdx.x - off] : 0;
    __syncthreads();
    shx[threadIdx.x] += ax;
    shy[threadIdx.x] += ay;
    __syncthreads();
  }
  double2 p = part[(size_t)r * nblk + blk];
  double cx = p.x + shx[threadIdx.x] - sx, cy = p.y + shy[threadIdx.x] - sy;
  for (int k = 0; k < SCAN_E; ++k) {
    if (inclusive) { cx += vx[k]; cy += vy[k]; }
    if (base + k < len) orow[base + k] = make_double2(cx, cy);
    if (!inclusive) { cx += vx[k]; cy += vy[k]; }
  }
}

void scan_rows(const double2 *in, double2 *out, int len, int ld, int R, bool inclusive,
               double2 *partials, hipStream_t st) {
  if (len <= 0 || R <= 0) return;
  int nblk = (int)cdiv(len, SCAN_B);
  k_scan_block_sums<<<dim3(nblk, R), SCAN_T, 0, st>>>(in, partials, len, ld, nblk);
  k_scan_partials<<<R, SCAN_T, 0, st>>>(partials, nblk);
  k_scan_final<<<dim3(nblk, R), SCAN_T, 0, st>>>(in, out, partials, len, ld, nblk, inclusive ? 1 : 0);
}

// ===========================================================================
// A^T: loop currents -> branch currents (Eq. CurT) by a subtree-sum scan
// ===========================================================================
// scan[r][k] (k < nn, preorder position) = sum of +-x over links ending at the
// node; scan[r][nn] = 0.
__global__ void k_inject(LoopMaps mp, const double2 *x, double2 *scan) {
  int r = blockIdx.y;
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > mp.nn) return;
  double sx = 0, sy = 0;
  if (k < mp.nn) {
    const double2 *xr = x + (size_t)r * mp.l;
    for (int q = mp.inj_off[k]; q < mp.inj_off[k + 1]; ++q) {
      double2 v = xr[mp.inj_link[q]];
      double sg = mp.inj_sgn[q];
      sx += sg * v.x;
      sy += sg * v.y;
    }
  }
  scan[(size_t)r * (mp.nn + 1) + k] = make_double2(sx, sy);
}

// after the exclusive scan: twig current = +-(P[hi] - P[lo]), link current = x;
// output alpha is RHS-contiguous: alpha[e][r]
__global__ void k_branch_out(LoopMaps mp, const double2 *x, const double2 *pfx, double2 *alpha, int R) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)mp.b * R) return;
  int e = (int)(idx / R), r = (int)(idx - (long)e * R);
  int a = mp.br_a[e];
  double2 v;
  if (a >= 0) {
    v = x[(size_t)r * mp.l + a];
  } else {
    const double2 *p = pfx + (size_t)r * (mp.nn + 1);
    double2 hi = p[mp.br_hi[e]], lo = p[mp.br_lo[e]];
    double sg = mp.br_sg[e];
    v = make_double2(sg * (hi.x - lo.x), sg * (hi.y - lo.y));
  }
  alpha[idx] = v;
}

void loop_to_branch(const LoopMaps &mp, const double2 *x, double2 *alpha, double2 *scan,
                    double2 *partials, int R, hipStream_t st) {
  k_inject<<<dim3(cdiv(mp.nn + 1, 256), R), 256, 0, st>>>(mp, x, scan);
  scan_rows(scan, scan, mp.nn + 1, mp.nn + 1, R, false, partials, st);
  k_branch_out<<<cdiv((long)mp.b * R, 256), 256, 0, st>>>(mp, x, scan, alpha, R);
}

// ===========================================================================
// A: branch voltages -> loop voltages (Eq. VolT) by a potential scan
// ===========================================================================
__device__ __forceinline__ double2 twig_drop(const LoopMaps &mp, const double2 *yb, int R, int pos) {
  int e = mp.pos_branch[pos];
  if (e < 0) return make_double2(0, 0);
  double2 v = yb[(size_t)e * R];
  double sg = mp.pos_sign[pos];
  return make_double2(sg * v.x, sg * v.y);
}

__global__ void k_drop_diff(LoopMaps mp, const double2 *yb, double2 *scan, int R) {
  int r = blockIdx.y;
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= mp.nn) return;
  const double2 *y = yb + r;   // yb[e][r]
  double2 d = twig_drop(mp, y, R, k);
  for (int q = mp.end_off[k]; q < mp.end_off[k + 1]; ++q) {
    double2 z = twig_drop(mp, y, R, mp.end_pos[q]);
    d.x -= z.x;
    d.y -= z.y;
  }
  scan[(size_t)r * (mp.nn + 1) + k] = d;
}

__global__ void k_link_out(LoopMaps mp, const double2 *yb, const double2 *D, double2 *yl, int R) {
  int r = blockIdx.y;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= mp.l) return;
  int e = mp.link_branch[i];
  double2 v = e < mp.b ? yb[(size_t)e * R + r] : make_double2(0, 0);
  int up = mp.link_upos[i], vp = mp.link_vpos[i];
  if (up >= 0) {
    const double2 *Dr = D + (size_t)r * (mp.nn + 1);
    v.x += Dr[vp].x - Dr[up].x;
    v.y += Dr[vp].y - Dr[up].y;
  }
  yl[(size_t)r * mp.l + i] = v;
}

void branch_to_loop(const LoopMaps &mp, const double2 *yb, double2 *yl, double2 *scan,
                    double2 *partials, int R, hipStream_t st) {
  k_drop_diff<<<dim3(cdiv(mp.nn, 256), R), 256, 0, st>>>(mp, yb, scan, R);
  scan_rows(scan, scan, mp.nn, mp.nn + 1, R, true, partials, st);
  k_link_out<<<dim3(cdiv(mp.l, 256), R), 256, 0, st>>>(mp, yb, scan, yl, R);
}

// ===========================================================================
// per-triangle current moments: J = (c0, d) / (2A), c0 = sum s a, d = sum s a (p - c)
// ===========================================================================
template <typename T>
__global__ void k_tri_current(GridMaps g, const double2 *alpha, V2<T> *J, int R) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)g.n * R) return;
  int t = (int)(idx / R), r = (int)(idx - (long)t * R);
  double c0x = 0, c0y = 0, dx[3] = {0, 0, 0}, dy[3] = {0, 0, 0};
  for (int i = 0; i < 3; ++i) {
    double2 v = alpha[(size_t)g.tri_edge[3 * t + i] * R + r];
    double s = g.tri_sign[3 * t + i];
    c0x += s * v.x;
    c0y += s * v.y;
    for (int c = 0; c < 3; ++c) {
      double p = g.pl[9 * t + 3 * i + c];
      dx[c] += s * v.x * p;
      dy[c] += s * v.y * p;
    }
  }
  double f = g.inv2A[t];
  V2<T> *o = J + ((size_t)r * g.n + t) * 4;
  o[0] = cmk<T>((T)(c0x * f), (T)(c0y * f));
  for (int c = 0; c < 3; ++c) o[1 + c] = cmk<T>((T)(dx[c] * f), (T)(dy[c] * f));
}

template <typename T>
void tri_currents(const GridMaps &g, const double2 *alpha, V2<T> *J, int R, hipStream_t st) {
  k_tri_current<T><<<cdiv((long)g.n * R, 256), 256, 0, st>>>(g, alpha, J, R);
}

// ===========================================================================
// projection (Eq. Projection): node-major gather, Q_c[g] = sum J0 M1_c - J_c M0
// ===========================================================================
template <typename T>
__global__ void k_project(GridMaps g, const V2<T> *J, V2<T> *Q) {
  int r = blockIdx.y;
  int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= g.N) return;
  const V2<T> *Jr = J + (size_t)r * g.n * 4;
  const T *w = (const T *)g.pg_w;
  V2<T> q0 = cmk<T>(0, 0), q1 = q0, q2 = q0;
  for (int k = g.pg_off[node]; k < g.pg_off[node + 1]; ++k) {
    int t = g.pg_tri[k];
    T m0 = w[4 * (size_t)k], m1x = w[4 * (size_t)k + 1], m1y = w[4 * (size_t)k + 2], m1z = w[4 * (size_t)k + 3];
    const V2<T> *jt = Jr + 4 * (size_t)t;
    V2<T> j0 = jt[0], jx = jt[1], jy = jt[2], jz = jt[3];
    q0.x += j0.x * m1x - jx.x * m0;
    q0.y += j0.y * m1x - jx.y * m0;
    q1.x += j0.x * m1y - jy.x * m0;
    q1.y += j0.y * m1y - jy.y * m0;
    q2.x += j0.x * m1z - jz.x * m0;
    q2.y += j0.y * m1z - jz.y * m0;
  }
  V2<T> *Qr = Q + (size_t)r * 3 * g.N;
  Qr[node] = q0;
  Qr[g.N + node] = q1;
  Qr[2 * (size_t)g.N + node] = q2;
}

template <typename T>
void project(const GridMaps &g, const V2<T> *J, V2<T> *Q, int R, hipStream_t st) {
  k_project<T><<<dim3(cdiv(g.N, 256), R), 256, 0, st>>>(g, J, Q);
}

// ===========================================================================
// LDS-staged radix-2 FFT along one axis of a [A][L][C] tensor
// ===========================================================================
// A workgroup transforms CW consecutive lines (line = a * C + c).  Input
// holds n_in points per line (zero padding up to Lf), output keeps the first
// n_out points.  mul != nullptr: forward FFT, multiply by the folded real
// spectrum, inverse FFT (the fused last-axis convolution).
struct FftArgs {
  int A, C, n_in, n_out, Lf, logL, CW;
  int sign;         // -1 forward, +1 inverse
  float scale;      // applied on output
  // fused multiply: spectrum index (kx, ky) from the line index
  int fused, two_nx, two_ny, nx, ny, nz;
};

__device__ __forceinline__ unsigned brev(unsigned k, int logL) { return __brev(k) >> (32 - logL); }

template <typename T>
__device__ void lds_fft(V2<T> *sm, const V2<T> *tw, int CW, int Lf, int logL, int sign) {
  int half_tot = Lf >> 1;
  for (int s = 1; s <= logL; ++s) {
    int len = 1 << s, half = len >> 1;
    int tstride = Lf >> s;
    for (int idx = threadIdx.x; idx < CW * half_tot; idx += blockDim.x) {
      int cw = idx / half_tot, j = idx - cw * half_tot;
      int grp = j >> (s - 1), pos = j & (half - 1);
      int i0 = cw * Lf + grp * len + pos, i1 = i0 + half;
      V2<T> w = tw[pos * tstride];
      if (sign > 0) w.y = -w.y;
      V2<T> u = sm[i0], v = cmul<T>(sm[i1], w);
      sm[i0] = cadd<T>(u, v);
      sm[i1] = csub<T>(u, v);
    }
    __syncthreads();
  }
}

template <typename T>
__global__ void k_fft_axis(FftArgs a, const V2<T> *in, V2<T> *out, const T *ghat) {
  extern __shared__ unsigned char smraw[];
  V2<T> *tw = (V2<T> *)smraw;               // Lf/2 twiddles exp(-2 pi i k / Lf)
  V2<T> *sm = tw + (a.Lf >> 1);              // CW x Lf
  long *ibase = (long *)(sm + (size_t)a.CW * a.Lf);   // per line: input base
  long *obase = ibase + a.CW;                          // per line: output base
  int *grow = (int *)(obase + a.CW);                   // per line: spectrum row (fused)
  const int Lf = a.Lf, CW = a.CW;
  const long nlines = (long)a.A * a.C;
  const long line0 = (long)blockIdx.x * CW;
  for (int k = threadIdx.x; k < (Lf >> 1); k += blockDim.x) {
    T sn, cs;
    if (sizeof(T) == 4) {
      float sf, cf;
      sincospif(2.0f * (float)k / (float)Lf, &sf, &cf);
      sn = sf;
      cs = cf;
    } else {
      double sd, cd;
      sincospi(2.0 * (double)k / (double)Lf, &sd, &cd);
      sn = (T)sd;
      cs = (T)cd;
    }
    tw[k] = cmk<T>(cs, -sn);
  }
  for (int cw = threadIdx.x; cw < CW; cw += blockDim.x) {
    long line = line0 + cw;
    if (line >= nlines) {
      ibase[cw] = -1;
      continue;
    }
    long aa = line / a.C, cc = line - aa * a.C;
    ibase[cw] = aa * a.n_in * a.C + cc;
    obase[cw] = aa * a.n_out * a.C + cc;
    if (a.fused) {
      long ky = line % a.two_ny, kx = (line / a.two_ny) % a.two_nx;
      int fx = kx <= a.nx ? (int)kx : a.two_nx - (int)kx;
      int fy = ky <= a.ny ? (int)ky : a.two_ny - (int)ky;
      grow[cw] = (fx * (a.ny + 1) + fy) * (a.nz + 1);
    }
  }
  for (int k = threadIdx.x; k < CW * Lf; k += blockDim.x) sm[k] = cmk<T>(0, 0);
  __syncthreads();
  // load (bit-reversed placement)
  const int nin = a.n_in;
  if (a.C == 1) {
    for (int idx = threadIdx.x; idx < CW * nin; idx += blockDim.x) {
      int cw = idx / nin, k = idx - cw * nin;
      long b0 = ibase[cw];
      if (b0 < 0) continue;
      sm[cw * Lf + brev(k, a.logL)] = in[b0 + k];
    }
  } else {
    for (int idx = threadIdx.x; idx < CW * nin; idx += blockDim.x) {
      int k = idx / CW, cw = idx - k * CW;
      long b0 = ibase[cw];
      if (b0 < 0) continue;
      sm[cw * Lf + brev(k, a.logL)] = in[b0 + (long)k * a.C];
    }
  }
  __syncthreads();
  lds_fft<T>(sm, tw, CW, Lf, a.logL, a.sign);
  if (a.fused) {
    // multiply by the real, even spectrum and transform back
    for (int idx = threadIdx.x; idx < CW * Lf; idx += blockDim.x) {
      int cw = idx / Lf, k = idx - cw * Lf;
      if (ibase[cw] < 0) continue;
      int fz = k <= a.nz ? k : Lf - k;
      sm[idx] = cscale<T>(sm[idx], ghat[grow[cw] + fz]);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < CW * Lf; idx += blockDim.x) {
      int cw = idx / Lf, k = idx - cw * Lf;
      int kb = brev(k, a.logL);
      if (k < kb) {
        V2<T> t0 = sm[cw * Lf + k];
        sm[cw * Lf + k] = sm[cw * Lf + kb];
        sm[cw * Lf + kb] = t0;
      }
    }
    __syncthreads();
    lds_fft<T>(sm, tw, CW, Lf, a.logL, +1);
  }
  // store
  const T sc = (T)a.scale;
  const int nout = a.n_out;
  if (a.C == 1) {
    for (int idx = threadIdx.x; idx < CW * nout; idx += blockDim.x) {
      int cw = idx / nout, k = idx - cw * nout;
      long b0 = obase[cw];
      if (ibase[cw] < 0) continue;
      out[b0 + k] = cscale<T>(sm[cw * Lf + k], sc);
    }
  } else {
    for (int idx = threadIdx.x; idx < CW * nout; idx += blockDim.x) {
      int k = idx / CW, cw = idx - k * CW;
      if (ibase[cw] < 0) continue;
      out[obase[cw] + (long)k * a.C] = cscale<T>(sm[cw * Lf + k], sc);
    }
  }
}

static int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

template <typename T>
static void fft_axis(const V2<T> *in, V2<T> *out, long A, long C, int n_in, int n_out, int Lf,
                     int sign, float scale, const T *ghat, const int *dims, hipStream_t st) {
  FftArgs a{};
  a.A = (int)A;
  a.C = (int)C;
  a.n_in = n_in;
  a.n_out = n_out;
  a.Lf = Lf;
  a.logL = ilog2(Lf);
  int per_line = Lf * (int)sizeof(V2<T>);
  int cw = (65536 - (Lf / 2) * (int)sizeof(V2<T>)) / (per_line + 20);
  if (cw < 1) cw = 1;
  if (cw > 64) cw = 64;
  if (C > 1 && cw > C) cw = (int)C;
  a.CW = cw;
  a.sign = sign;
  a.scale = scale;
  a.fused = ghat != nullptr;
  if (dims) {
    a.nx = dims[0];
    a.ny = dims[1];
    a.nz = dims[2];
    a.two_nx = 2 * dims[0];
    a.two_ny = 2 * dims[1];
  }
  long lines = A * C;
  size_t shm = (size_t)(Lf / 2) * sizeof(V2<T>) + (size_t)cw * Lf * sizeof(V2<T>) +
               (size_t)cw * (2 * sizeof(long) + sizeof(int));
  k_fft_axis<T><<<cdiv(lines, cw), 256, shm, st>>>(a, in, out, ghat);
}

template <typename T>
void convolve(const GridMaps &g, V2<T> *Q, V2<T> *T1, V2<T> *T2, int R, hipStream_t st, PassHook *hook) {
  const int Nx = g.dims[0], Ny = g.dims[1], Nz = g.dims[2];
  long ch = 3L * R;
  // X forward: [ch][Nx][Ny*Nz] -> [ch][2Nx][Ny*Nz]
  if (hook) hook->pass(0, st);
  fft_axis<T>(Q, T1, ch, (long)Ny * Nz, Nx, 2 * Nx, 2 * Nx, -1, 1.0f, nullptr, nullptr, st);
  // Y forward: [ch*2Nx][Ny][Nz] -> [ch*2Nx][2Ny][Nz]
  if (hook) hook->pass(1, st);
  fft_axis<T>(T1, T2, ch * 2 * Nx, Nz, Ny, 2 * Ny, 2 * Ny, -1, 1.0f, nullptr, nullptr, st);
  // Z forward, multiply, inverse, crop: [ch*2Nx*2Ny][Nz] in place
  if (hook) hook->pass(2, st);
  fft_axis<T>(T2, T2, ch * 4L * Nx * Ny, 1, Nz, Nz, 2 * Nz, -1, 1.0f / (2.0f * Nz),
              (const T *)g.ghat, g.dims, st);
  // Y inverse, crop: [ch*2Nx][2Ny][Nz] -> [ch*2Nx][Ny][Nz]
  if (hook) hook->pass(3, st);
  fft_axis<T>(T2, T1, ch * 2 * Nx, Nz, 2 * Ny, Ny, 2 * Ny, +1, 1.0f / (2.0f * Ny), nullptr, nullptr, st);
  // X inverse, crop: [ch][2Nx][Ny*Nz] -> [ch][Nx][Ny*Nz]
  if (hook) hook->pass(4, st);
  fft_axis<T>(T1, Q, ch, (long)Ny * Nz, 2 * Nx, Nx, 2 * Nx, +1, 1.0f / (2.0f * Nx), nullptr, nullptr, st);
  if (hook) hook->done(st);
}

void fft3_full_fp64(double2 *data, const int d2[3], hipStream_t st) {
  long X = d2[0], Y = d2[1], Z = d2[2];
  fft_axis<double>(data, data, X * Y, 1, (int)Z, (int)Z, (int)Z, -1, 1.0f, nullptr, nullptr, st);
  fft_axis<double>(data, data, X, Z, (int)Y, (int)Y, (int)Y, -1, 1.0f, nullptr, nullptr, st);
  fft_axis<double>(data, data, 1, Y * Z, (int)X, (int)X, (int)X, -1, 1.0f, nullptr, nullptr, st);
}

template <typename T>
__global__ void k_fold(const double2 *full, T *ghat, int nx, int ny, int nz) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long tot = (long)(nx + 1) * (ny + 1) * (nz + 1);
  if (idx >= tot) return;
  int kz = idx % (nz + 1);
  int ky = (idx / (nz + 1)) % (ny + 1);
  int kx = idx / ((long)(nz + 1) * (ny + 1));
  ghat[idx] = (T)full[((long)kx * 2 * ny + ky) * 2 * nz + kz].x;
}

template <typename T>
void fold_spectrum(const double2 *full, T *ghat, const int dims[3], hipStream_t st) {
  long tot = (long)(dims[0] + 1) * (dims[1] + 1) * (dims[2] + 1);
  k_fold<T><<<cdiv(tot, 256), 256, 0, st>>>(full, ghat, dims[0], dims[1], dims[2]);
}

// ===========================================================================
// interpolation (Eq. interpolation, I = B^T), triangle phase:
// U = (sum_c sum_g M1_c phi_c, sum_g M0 phi_x, ... phi_y, ... phi_z)
// ===========================================================================
template <typename T>
__global__ void k_interp_tri(GridMaps g, const V2<T> *phi, double2 *U) {
  int r = blockIdx.y;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.n) return;
  const int Ny = g.dims[1], Nz = g.dims[2];
  const V2<T> *P = phi + (size_t)r * 3 * g.N;
  const T *w = (const T *)g.tri_w + (size_t)t * 256;
  int ax = g.anchor[3 * t], ay = g.anchor[3 * t + 1], az = g.anchor[3 * t + 2];
  double s1x = 0, s1y = 0, ux[3] = {0, 0, 0}, uy[3] = {0, 0, 0};
  for (int k = 0; k < 64; ++k) {
    int i = k >> 4, j = (k >> 2) & 3, l = k & 3;
    long node = ((long)(ax + i) * Ny + (ay + j)) * Nz + (az + l);
    double m0 = w[4 * k];
    for (int c = 0; c < 3; ++c) {
      V2<T> v = P[(size_t)c * g.N + node];
      double m1 = w[4 * k + 1 + c];
      s1x += m1 * v.x;
      s1y += m1 * v.y;
      ux[c] += m0 * v.x;
      uy[c] += m0 * v.y;
    }
  }
  double2 *o = U + ((size_t)t * gridDim.y + r) * 4;   // U[t][r][4]
  o[0] = make_double2(s1x, s1y);
  for (int c = 0; c < 3; ++c) o[1 + c] = make_double2(ux[c], uy[c]);
}

template <typename T>
void interp_tri(const GridMaps &g, const V2<T> *phi, double2 *U, int R, hipStream_t st) {
  k_interp_tri<T><<<dim3(cdiv(g.n, 128), R), 128, 0, st>>>(g, phi, U);
}

// ===========================================================================
// edge phase: far field from the two triangles, near-field CSR, Gram, combine
// ===========================================================================
// One thread per (edge, RHS), RHS fastest: the near-field row's values and
// columns are shared by the RHS lanes and each gathered column alpha[col][.]
// is one contiguous segment, so every load of the sparse product coalesces.
__global__ void k_combine(CombineMaps c, const double2 *alpha, const double2 *U, const double2 *zs,
                          const double2 *jw, double2 *y, int R, int mode) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)c.b * R) return;
  int e = (int)(idx / R), r = (int)(idx - (long)e * R);
  double kx = 0, ky = 0;
  if (mode & 1) {
    for (int side = 0; side < 2; ++side) {
      int t = c.efar_t[2 * e + side];
      double s = c.efar_s[2 * e + side];
      const double *p = c.efar_pl + 6 * (size_t)e + 3 * side;
      const double2 *u = U + ((size_t)t * R + r) * 4;
      double vx = u[0].x - (p[0] * u[1].x + p[1] * u[2].x + p[2] * u[3].x);
      double vy = u[0].y - (p[0] * u[1].y + p[1] * u[2].y + p[2] * u[3].y);
      kx += s * vx;
      ky += s * vy;
    }
  }
  if (mode & 2) {
    const int64_t q1 = c.nf_rowptr[e + 1];
    for (int64_t q = c.nf_rowptr[e]; q < q1; ++q) {
      double v = c.nf_val[q];
      double2 x = alpha[(size_t)c.nf_col[q] * R + r];
      kx += v * x.x;
      ky += v * x.y;
    }
  }
  double2 out;
  if (mode & 4) {
    double gx = 0, gy = 0;
    for (int q = 0; q < 5; ++q) {
      double v = c.gram_val[5 * e + q];
      double2 x = alpha[(size_t)c.gram_col[5 * e + q] * R + r];
      gx += v * x.x;
      gy += v * x.y;
    }
    double2 z = zs[r], j = jw[r];
    out.x = z.x * gx - z.y * gy + j.x * kx - j.y * ky;
    out.y = z.x * gy + z.y * gx + j.x * ky + j.y * kx;
  } else {
    out = make_double2(kx, ky);
  }
  y[idx] = out;
}

void combine(const CombineMaps &c, const double2 *alpha, const double2 *U, const double2 *zs,
             const double2 *jw, double2 *y, int R, int mode, hipStream_t st) {
  k_combine<<<cdiv((long)c.b * R, 256), 256, 0, st>>>(c, alpha, U, zs, jw, y, R, mode);
}

// out[c][r] = in[r][c] for a rows x cols complex128 matrix, 32 x 32 LDS tiles
__global__ void k_transpose(const double2 *in, double2 *out, int rows, int cols) {
  __shared__ double2 tile[32][33];
  int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    int r = r0 + k, c = c0 + threadIdx.x;
    if (r < rows && c < cols) tile[k][threadIdx.x] = in[(size_t)r * cols + c];
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    int c = c0 + k, r = r0 + threadIdx.x;
    if (r < rows && c < cols) out[(size_t)c * rows + r] = tile[threadIdx.x][k];
  }
}

void transpose(const double2 *in, double2 *out, int rows, int cols, hipStream_t st) {
  k_transpose<<<dim3(cdiv(cols, 32), cdiv(rows, 32)), dim3(32, 8), 0, st>>>(in, out, rows, cols);
}

// explicit instantiations
template void tri_currents<float>(const GridMaps &, const double2 *, V2<float> *, int, hipStream_t);
template void tri_currents<double>(const GridMaps &, const double2 *, V2<double> *, int, hipStream_t);
template void project<float>(const GridMaps &, const V2<float> *, V2<float> *, int, hipStream_t);
template void project<double>(const GridMaps &, const V2<double> *, V2<double> *, int, hipStream_t);
template void convolve<float>(const GridMaps &, V2<float> *, V2<float> *, V2<float> *, int, hipStream_t, PassHook *);
template void convolve<double>(const GridMaps &, V2<double> *, V2<double> *, V2<double> *, int, hipStream_t, PassHook *);
template void interp_tri<float>(const GridMaps &, const V2<float> *, double2 *, int, hipStream_t);
template void interp_tri<double>(const GridMaps &, const V2<double> *, double2 *, int, hipStream_t);
template void fold_spectrum<float>(const double2 *, float *, const int *, hipStream_t);
template void fold_spectrum<double>(const double2 *, double *, const int *, hipStream_t);

}  // namespace pfft
