// Learned correction of the preconditioner inside flexible GMRES.
//
// A per-loop multilayer perceptron (F = 16 inputs, two ReLU layers of width
// H, 2 outputs) refines M(v) = P^-1 v.  Its matrix products run on the gfx950
// matrix cores (v_mfma_f32_32x32x8_bf16: bf16 operands, FP32 accumulation);
// biases, ReLU, the loss and Adam are FP32 vector code.  Training pairs come
// from the solver: after each restart of a plain-P solve, the true residual
// r_j and the error e_j = x* - x_j (Z_l e_j = r_j).  Features, targets and
// the update rule are documented with the entry points in pfft.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <random>
#include <vector>

#include "engine.h"
#include "learned.h"
#include "precond.h"

namespace pfft {

namespace {

constexpr int F_IN = 16;
constexpr int F_OUT = 2;
constexpr uint32_t MAGIC = 0x504D4C50u;  // "PMLP"
constexpr double DELTA_CAP2 = 16.0;      // fallback when sum |y|^2 > 16 l

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__host__ __device__ inline uint16_t to_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);                                           // nearest, ties to even
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float from_bf16(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

// ---------------------------------------------------------------------------
// C[m][n] = epilogue( sum_k A(m,k) B(k,n) ), A(m,k) = A[m sam + k sak],
// B(k,n) = B[k sbk + n sbn].  An operand is bf16, or FP32 split on load into
// bf16 hi + lo (x = hi + lo to ~2^-16 relative; the products hi*hi, lo*hi,
// hi*lo are accumulated, so FP32 activations keep ~FP32 accuracy).
// Epilogue: + bias[n]; ReLU; zero where mask[m][n] (FP32, same layout as C)
// is not positive; store FP32 and/or bf16.
// ---------------------------------------------------------------------------
struct Gemm {
  int M, N, K;
  const void *A;
  long long sam, sak;
  int a32;
  const void *B;
  long long sbk, sbn;
  int b32;
  const float *bias;
  const float *mask;
  int relu;
  float *Cf;
  uint16_t *Cb;
  long long ldc;
};

template <bool F32>
__device__ inline void load_split(const void *p, long long o, bool ok, short &hi, short &lo) {
  if (F32) {
    const float x = ok ? ((const float *)p)[o] : 0.f;
    const uint16_t h = to_bf16(x);
    hi = (short)h;
    lo = (short)to_bf16(x - from_bf16(h));
  } else {
    hi = ok ? (short)((const uint16_t *)p)[o] : (short)0;
    lo = 0;
  }
}

// One wave per 32x32 tile of C; the NW waves of a block share the 32 rows of
// A (n tiles blockIdx.y*NW .. +NW-1).  Operand layout of the 32x32x8 bf16
// MFMA: lane l holds A[l%32][4(l/32) + t] and B[4(l/32) + t][l%32], t = 0..3;
// accumulator v of lane l is C[8(v/4) + 4(l/32) + v%4][l%32].
template <int NW, bool A32, bool B32>
__global__ __launch_bounds__(64 * NW) void k_gemm(Gemm g) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.x * 32, n0 = (blockIdx.y * NW + w) * 32;
  if (n0 >= g.N) return;
  const int r = lane & 31, kq = (lane >> 5) * 4;
  const int am = m0 + r, bn = n0 + r;
  const bool aok = am < g.M, bok = bn < g.N;
  const long long abase = aok ? (long long)am * g.sam : 0, bbase = bok ? (long long)bn * g.sbn : 0;
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  for (int k0 = 0; k0 < g.K; k0 += 8) {
    bf16x4 ah, al, bh, bl;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = k0 + kq + t;
      const bool kok = k < g.K;
      short h, lo;
      load_split<A32>(g.A, abase + (long long)k * g.sak, aok && kok, h, lo);
      ah[t] = h;
      al[t] = lo;
      load_split<B32>(g.B, bbase + (long long)k * g.sbk, bok && kok, h, lo);
      bh[t] = h;
      bl[t] = lo;
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah, bh, acc, 0, 0, 0);
    if (A32) acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(al, bh, acc, 0, 0, 0);
    if (B32) acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah, bl, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int row = m0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    if (row < g.M && bok) {
      float x = acc[v];
      if (g.bias) x += g.bias[bn];
      if (g.relu && x <= 0.f) x = 0.f;   // NaN passes through
      const long long o = (long long)row * g.ldc + bn;
      if (g.mask && !(g.mask[o] > 0.f)) x = 0.f;
      if (g.Cf) g.Cf[o] = x;
      if (g.Cb) g.Cb[o] = to_bf16(x);
    }
  }
}

template <bool A32, bool B32>
void gemm_nw(const Gemm &g, int nw, dim3 grid, hipStream_t st) {
  switch (nw) {
    case 8: k_gemm<8, A32, B32><<<grid, 512, 0, st>>>(g); break;
    case 4: k_gemm<4, A32, B32><<<grid, 256, 0, st>>>(g); break;
    case 2: k_gemm<2, A32, B32><<<grid, 128, 0, st>>>(g); break;
    default: k_gemm<1, A32, B32><<<grid, 64, 0, st>>>(g); break;
  }
}

void gemm(const Gemm &g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return;
  const int nt = (g.N + 31) / 32, mt = (g.M + 31) / 32;
  const int nw = nt >= 8 ? 8 : nt >= 4 ? 4 : nt >= 2 ? 2 : 1;
  const dim3 grid(mt, (nt + nw - 1) / nw);
  if (g.a32 && g.b32) gemm_nw<true, true>(g, nw, grid, st);
  else if (g.a32) gemm_nw<true, false>(g, nw, grid, st);
  else if (g.b32) gemm_nw<false, true>(g, nw, grid, st);
  else gemm_nw<false, false>(g, nw, grid, st);
}

// ---------------------------------------------------------------------------
// loss, reductions, optimiser
// ---------------------------------------------------------------------------
template <typename Tv>
__device__ inline Tv block_sum256(Tv v, Tv *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

// dy = 2 w wscale (y - t); per-block partial loss
__global__ __launch_bounds__(256) void k_loss(const float *Y, const float *T, const float *w, double wscale, int B,
                                              float *dyf, double *part) {
  __shared__ double sh[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  double l = 0;
  if (i < B) {
    const double ww = (double)w[i] * wscale;
    const double d0 = (double)Y[2 * i] - T[2 * i], d1 = (double)Y[2 * i + 1] - T[2 * i + 1];
    l = ww * (d0 * d0 + d1 * d1);
    const float g0 = (float)(2.0 * ww * d0), g1 = (float)(2.0 * ww * d1);
    dyf[2 * i] = g0;
    dyf[2 * i + 1] = g1;
  }
  const double s = block_sum256(l, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[slot] = sum of n partials (fixed order)
__global__ void k_sum_final(const double *part, int n, double *out, int slot) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double s = 0;
    for (int i = 0; i < n; ++i) s += part[i];
    out[slot] = s;
  }
}

// column sums of X [M][ld] over rows: partials [gridDim.y][N], then final
__global__ __launch_bounds__(256) void k_colsum_part(const float *X, int M, int N, int ld, float *part) {
  __shared__ float sh[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
  float s = 0.f;
  if (c < N)
    for (int r = blockIdx.y * 4 + g; r < M; r += 4 * gridDim.y) s += X[(long long)r * ld + c];
  sh[g][threadIdx.x & 63] = s;
  __syncthreads();
  if (g == 0 && c < N) {
    const int t = threadIdx.x & 63;
    part[(long long)blockIdx.y * N + c] = (sh[0][t] + sh[1][t]) + (sh[2][t] + sh[3][t]);
  }
}

__global__ void k_colsum_final(const float *part, int S, int N, float *out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  double s = 0;
  for (int z = 0; z < S; ++z) s += part[(long long)z * N + c];
  out[c] = (float)s;
}

constexpr int COLSUM_SPLIT = 64;

void colsum(const float *X, int M, int N, int ld, float *part, float *out, hipStream_t st) {
  k_colsum_part<<<dim3((N + 63) / 64, COLSUM_SPLIT), 256, 0, st>>>(X, M, N, ld, part);
  k_colsum_final<<<(N + 255) / 256, 256, 0, st>>>(part, COLSUM_SPLIT, N, out);
}

// Adam (Kingma & Ba): p -= lr mhat / (sqrt(vhat) + eps); refresh the bf16
// copy of the first nb entries (the weight matrices)
__global__ void k_adam(float *p, float *m, float *v, const float *g, int n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2, uint16_t *pb, int nb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  p[i] = pi;
  if (i < nb) pb[i] = to_bf16(pi);
}

// ---------------------------------------------------------------------------
// features, correction, collection
// ---------------------------------------------------------------------------
// per RHS: |v|^2, |z|^2
__global__ __launch_bounds__(256) void k_norms(const double2 *v, const double2 *z, int l, double *out) {
  __shared__ double sh[256];
  const int r = blockIdx.x;
  double a = 0, b = 0;
  for (int i = threadIdx.x; i < l; i += 256) {
    const double2 x = v[(size_t)r * l + i], y = z[(size_t)r * l + i];
    a += x.x * x.x + x.y * x.y;
    b += y.x * y.x + y.y * y.y;
  }
  a = block_sum256(a, sh);
  __syncthreads();
  b = block_sum256(b, sh);
  if (threadIdx.x == 0) {
    out[2 * r] = a;
    out[2 * r + 1] = b;
  }
}

struct FeatArgs {
  const double2 *v, *z;     // [R][l]
  const double *nrm;        // [R][2]
  const int *fidx;          // [R] factor index
  const double2 *yinv;      // [nf][b] 1/D_e
  const int *link_kind;     // [l] mesh branch or -(port+1)
  const uint8_t *self_loop; // [l]
  const float *logf;        // [R]
  const int *n1_off, *n1;   // ring-1 link neighbours of each loop (CSR over loops)
  const int *n2_off, *n2;   // ring-2 link neighbours
  int l, b, R;
  uint16_t *X;              // [R*l][16]
};

// mean of (v sv, z sz) over the loops nb[off[i] .. off[i+1]) of RHS r
__device__ inline void ring_mean(const FeatArgs &a, const int *off, const int *nb, int i, size_t base, double sv,
                                 double sz, float out[4]) {
  const int k0 = off[i], k1 = off[i + 1];
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  for (int k = k0; k < k1; ++k) {
    const double2 vj = a.v[base + nb[k]], zj = a.z[base + nb[k]];
    s0 += vj.x;
    s1 += vj.y;
    s2 += zj.x;
    s3 += zj.y;
  }
  const double w = k1 > k0 ? 1.0 / (k1 - k0) : 0.0;
  out[0] = (float)(s0 * w * sv);
  out[1] = (float)(s1 * w * sv);
  out[2] = (float)(s2 * w * sz);
  out[3] = (float)(s3 * w * sz);
}

__global__ __launch_bounds__(256) void k_features(FeatArgs a) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long long)a.R * a.l) return;
  const int r = (int)(idx / a.l), i = (int)(idx - (long long)r * a.l);
  const size_t base = (size_t)r * a.l;
  const double nv = a.nrm[2 * r], nz = a.nrm[2 * r + 1];
  const double sv = nv > 0 ? sqrt(a.l / nv) : 0.0, sz = nz > 0 ? sqrt(a.l / nz) : 0.0;
  const double2 vv = a.v[idx], zz = a.z[idx];
  const int e = a.link_kind[i];
  float f7 = 0.f;
  if (e >= 0) {
    const double2 y = a.yinv[(size_t)a.fidx[r] * a.b + e];
    const double ay = sqrt(y.x * y.x + y.y * y.y);
    f7 = ay > 0 ? (float)(y.x / ay) : 0.f;   // Re D / |D| = Re(1/D) / |1/D|
  }
  float f[F_IN] = {(float)(vv.x * sv), (float)(vv.y * sv), (float)(zz.x * sz), (float)(zz.y * sz),
                   a.logf[r], e < 0 ? 1.f : 0.f, a.self_loop[i] ? 1.f : 0.f, f7};
  ring_mean(a, a.n1_off, a.n1, i, base, sv, sz, f + 8);
  ring_mean(a, a.n2_off, a.n2, i, base, sv, sz, f + 12);
  uint4 pk[2];
  for (int h = 0; h < 2; ++h) {
    const float *g = f + 8 * h;
    pk[h].x = (uint32_t)to_bf16(g[0]) | ((uint32_t)to_bf16(g[1]) << 16);
    pk[h].y = (uint32_t)to_bf16(g[2]) | ((uint32_t)to_bf16(g[3]) << 16);
    pk[h].z = (uint32_t)to_bf16(g[4]) | ((uint32_t)to_bf16(g[5]) << 16);
    pk[h].w = (uint32_t)to_bf16(g[6]) | ((uint32_t)to_bf16(g[7]) << 16);
  }
  reinterpret_cast<uint4 *>(a.X)[2 * idx] = pk[0];
  reinterpret_cast<uint4 *>(a.X)[2 * idx + 1] = pk[1];
}

// ok[r] = every y of RHS r finite and sum |y|^2 <= cap2
__global__ __launch_bounds__(256) void k_check(const float *Y, int l, double cap2, uint8_t *ok) {
  __shared__ double sh[256];
  const int r = blockIdx.x;
  double s = 0;
  for (int i = threadIdx.x; i < l; i += 256) {
    const float y0 = Y[2 * ((size_t)r * l + i)], y1 = Y[2 * ((size_t)r * l + i) + 1];
    s += (double)y0 * y0 + (double)y1 * y1;   // NaN / inf propagate into s
  }
  s = block_sum256(s, sh);
  if (threadIdx.x == 0) ok[r] = (s <= cap2) ? 1 : 0;
}

// z += (y0 + j y1) |z| / sqrt(l) where ok and enabled
__global__ __launch_bounds__(256) void k_correct(double2 *z, const float *Y, const double *nrm, const uint8_t *ok,
                                                 const uint8_t *en, int l, int R) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long long)R * l) return;
  const int r = (int)(idx / l);
  const double nz = nrm[2 * r + 1];
  if (!ok[r] || !en[r] || !(nz > 0)) return;
  const double sc = sqrt(nz / l);
  double2 zz = z[idx];
  zz.x += (double)Y[2 * idx] * sc;
  zz.y += (double)Y[2 * idx + 1] * sc;
  z[idx] = zz;
}

__global__ void k_stats(const uint8_t *ok, const uint8_t *en, int R, long long *stats) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    long long n = 0, bad = 0;
    for (int r = 0; r < R; ++r) {
      n += en[r] ? 1 : 0;
      bad += (en[r] && !ok[r]) ? 1 : 0;
    }
    stats[0] += n;
    stats[1] += bad;
  }
}

// per RHS: |r|^2, |z|^2, <z, e> (conjugate-linear in z)
__global__ __launch_bounds__(256) void k_dots(const double2 *rv, const double2 *z, const double2 *e, int l,
                                              double *out) {
  __shared__ double sh[256];
  const int r = blockIdx.x;
  double a = 0, b = 0, cr = 0, ci = 0;
  for (int i = threadIdx.x; i < l; i += 256) {
    const size_t o = (size_t)r * l + i;
    const double2 x = rv[o], y = z[o], q = e[o];
    a += x.x * x.x + x.y * x.y;
    b += y.x * y.x + y.y * y.y;
    cr += y.x * q.x + y.y * q.y;
    ci += y.x * q.y - y.y * q.x;
  }
  a = block_sum256(a, sh);
  __syncthreads();
  b = block_sum256(b, sh);
  __syncthreads();
  cr = block_sum256(cr, sh);
  __syncthreads();
  ci = block_sum256(ci, sh);
  if (threadIdx.x == 0) {
    out[4 * r] = a;
    out[4 * r + 1] = b;
    out[4 * r + 2] = cr;
    out[4 * r + 3] = ci;
  }
}

// E[r][i] = x[r][i] * s[r]
__global__ void k_scale_rows(const double2 *x, const double *s, int l, double2 *E) {
  const int r = blockIdx.y, i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= l) return;
  const double2 v = x[(size_t)r * l + i];
  E[(size_t)r * l + i] = make_double2(v.x * s[r], v.y * s[r]);
}

// Backward Arnoldi recursion for the exact errors e_j = Z_l^-1 v_j:
// E[k+1][r] = (Z[r][k] - sum_{i<=k} H[r][i][k] E[i][r]) / H[r][k+1][k];
// E [K][R][l], Z [R][m][l], H [R][m+1][m]
__global__ void k_krylov_error(const double2 *Z, const double2 *H, double2 *E, int l, int m, int k, int R) {
  const int r = blockIdx.y, i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= l) return;
  const int RR = gridDim.y;
  const double2 *Hc = H + (size_t)r * (m + 1) * m;
  double2 acc = Z[((size_t)r * m + k) * l + i];
  for (int j = 0; j <= k; ++j) {
    const double2 h = Hc[j * m + k], e = E[((size_t)j * RR + r) * l + i];
    acc.x -= h.x * e.x - h.y * e.y;
    acc.y -= h.x * e.y + h.y * e.x;
  }
  const double2 d = Hc[(k + 1) * m + k];
  const double den = d.x * d.x + d.y * d.y;
  const double2 q = den > 0 ? make_double2((acc.x * d.x + acc.y * d.y) / den, (acc.y * d.x - acc.x * d.y) / den)
                            : make_double2(0.0, 0.0);
  E[((size_t)(k + 1) * RR + r) * l + i] = q;
  (void)R;
}

// T[r*l+i] = (g_r e_i - z_i) s_r  (FP32 pair); coef [R][3] = Re g, Im g, s
__global__ void k_targets(const double2 *z, const double2 *e, const double *coef, int l, int R, float *T) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)R * l) return;
  const int r = (int)(idx / l);
  const double gr = coef[3 * r], gi = coef[3 * r + 1], s = coef[3 * r + 2];
  const double2 q = e[idx], zz = z[idx];
  T[2 * idx] = (float)((gr * q.x - gi * q.y - zz.x) * s);
  T[2 * idx + 1] = (float)((gr * q.y + gi * q.x - zz.y) * s);
}

// per RHS sum |t|^2 (of the FP32 targets)
__global__ __launch_bounds__(256) void k_tnorm(const float *T, int l, double *out) {
  __shared__ double sh[256];
  const int r = blockIdx.x;
  double s = 0;
  for (int i = threadIdx.x; i < l; i += 256) {
    const double a = T[2 * ((size_t)r * l + i)], b = T[2 * ((size_t)r * l + i) + 1];
    s += a * a + b * b;
  }
  s = block_sum256(s, sh);
  if (threadIdx.x == 0) out[r] = s;
}

// per-block partial of sum_i |y_i - t_i|^2 / (G den[group_i]) over a chunk
__global__ __launch_bounds__(256) void k_set_loss(const float *Y, const float *T, const int *gs, const double *den,
                                                  int G, int n, double *part) {
  __shared__ double sh[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  double l = 0;
  if (i < n) {
    const double d0 = (double)Y[2 * i] - T[2 * i], d1 = (double)Y[2 * i + 1] - T[2 * i + 1];
    l = (d0 * d0 + d1 * d1) / ((double)G * den[gs[i]]);
  }
  const double s = block_sum256(l, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_fill_int(int *p, long long n, int v) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__device__ inline unsigned long long splitmix64(unsigned long long z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// minibatch row i of step s: uniform draw from the training set; weight
// 1 / (G den[group])
__global__ void k_gather(const uint16_t *Xs, const float *Ts, const int *gs, const double *den, int G, long long rows,
                         unsigned long long seed, long long step, int B, int F, uint16_t *X, float *T, float *w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const unsigned long long h = splitmix64(splitmix64(seed) ^ (unsigned long long)(step * B + i));
  const long long j = (long long)(h % (unsigned long long)rows);
  for (int f = 0; f < F; ++f) X[(long long)i * F + f] = Xs[j * F + f];
  T[2 * i] = Ts[2 * j];
  T[2 * i + 1] = Ts[2 * j + 1];
  w[i] = (float)(1.0 / ((double)G * den[gs[j]]));
}

// ---------------------------------------------------------------------------
// network parameters and buffers
// ---------------------------------------------------------------------------
struct Shape {
  int F = F_IN, H = 256, O = F_OUT;
  long long nw() const { return (long long)H * F + (long long)H * H + (long long)O * H; }
  long long np() const { return nw() + 2LL * H + O; }
  long long blob_bytes() const { return 16 + 4 * ((nw() + 1) / 2) + 4 * (2LL * H + O); }
};

bool parse_header(const void *blob, long long nbytes, Shape &s) {
  if (!blob || nbytes < 16) return false;
  int32_t h[4];
  memcpy(h, blob, 16);
  if ((uint32_t)h[0] != MAGIC || h[1] <= 0 || h[2] <= 0 || h[3] <= 0 || h[1] > 4096 || h[2] > 4096 || h[3] > 64)
    return false;
  s.F = h[1];
  s.H = h[2];
  s.O = h[3];
  return s.blob_bytes() == nbytes;
}

// device parameters: FP32 masters P = [W1 W2 W3 b1 b2 b3], bf16 weights Wb
struct Net {
  Shape s;
  float *P = nullptr, *G = nullptr, *Mm = nullptr, *Vv = nullptr;
  uint16_t *Wb = nullptr;
  long long adam_t = 0;
  const uint16_t *W1() const { return Wb; }
  const uint16_t *W2() const { return Wb + (long long)s.H * s.F; }
  const uint16_t *W3() const { return Wb + (long long)s.H * s.F + (long long)s.H * s.H; }
  const float *b1() const { return P + s.nw(); }
  const float *b2() const { return P + s.nw() + s.H; }
  const float *b3() const { return P + s.nw() + 2LL * s.H; }
};

void net_free(Net &n) {
  for (void *p : {(void *)n.P, (void *)n.G, (void *)n.Mm, (void *)n.Vv, (void *)n.Wb})
    if (p) hipFree(p);
  n = Net();
}

void dev_alloc(void **p, size_t bytes, const char *what) {
  hip_ok(hipMalloc(p, bytes ? bytes : 16), what);
}

// host blob -> device net (allocates)
void net_from_blob(Net &n, const Shape &s, const void *blob, hipStream_t st) {
  net_free(n);
  n.s = s;
  const long long np = s.np(), nw = s.nw();
  dev_alloc((void **)&n.P, np * 4, "mlp params");
  dev_alloc((void **)&n.G, np * 4, "mlp grads");
  dev_alloc((void **)&n.Mm, np * 4, "mlp adam m");
  dev_alloc((void **)&n.Vv, np * 4, "mlp adam v");
  dev_alloc((void **)&n.Wb, nw * 2, "mlp bf16 weights");
  const uint8_t *b = (const uint8_t *)blob;
  std::vector<uint16_t> wb(nw);
  memcpy(wb.data(), b + 16, nw * 2);
  std::vector<float> p(np);
  for (long long i = 0; i < nw; ++i) p[i] = from_bf16(wb[i]);
  memcpy(p.data() + nw, b + 16 + 4 * ((nw + 1) / 2), (np - nw) * 4);
  hip_ok(hipMemcpyAsync(n.Wb, wb.data(), nw * 2, hipMemcpyHostToDevice, st), "upload weights");
  hip_ok(hipMemcpyAsync(n.P, p.data(), np * 4, hipMemcpyHostToDevice, st), "upload params");
  hip_ok(hipMemsetAsync(n.Mm, 0, np * 4, st), "adam m");
  hip_ok(hipMemsetAsync(n.Vv, 0, np * 4, st), "adam v");
  hip_ok(hipStreamSynchronize(st), "net upload");
  n.adam_t = 0;
}

std::vector<uint8_t> net_to_blob(const Net &n, hipStream_t st) {
  const Shape &s = n.s;
  const long long np = s.np(), nw = s.nw();
  std::vector<uint8_t> out(s.blob_bytes(), 0);
  int32_t h[4] = {(int32_t)MAGIC, s.F, s.H, s.O};
  memcpy(out.data(), h, 16);
  std::vector<uint16_t> wb(nw);
  std::vector<float> p(np);
  hip_ok(hipMemcpyAsync(wb.data(), n.Wb, nw * 2, hipMemcpyDeviceToHost, st), "download weights");
  hip_ok(hipMemcpyAsync(p.data(), n.P, np * 4, hipMemcpyDeviceToHost, st), "download params");
  hip_ok(hipStreamSynchronize(st), "net download");
  memcpy(out.data() + 16, wb.data(), nw * 2);
  memcpy(out.data() + 16 + 4 * ((nw + 1) / 2), p.data() + nw, (np - nw) * 4);
  return out;
}

// seeded He initialisation; the output layer starts small (correction ~ 0)
std::vector<uint8_t> init_blob(int H, unsigned long long seed) {
  Shape s;
  s.H = H;
  std::vector<uint8_t> out(s.blob_bytes(), 0);
  int32_t h[4] = {(int32_t)MAGIC, s.F, s.H, s.O};
  memcpy(out.data(), h, 16);
  std::mt19937_64 gen(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<uint16_t> wb(s.nw());
  long long k = 0;
  for (long long i = 0; i < (long long)H * s.F; ++i) wb[k++] = to_bf16((float)(nd(gen) * std::sqrt(2.0 / s.F)));
  for (long long i = 0; i < (long long)H * H; ++i) wb[k++] = to_bf16((float)(nd(gen) * std::sqrt(2.0 / H)));
  for (long long i = 0; i < (long long)s.O * H; ++i) wb[k++] = to_bf16((float)(nd(gen) * 0.1 / std::sqrt((double)H)));
  memcpy(out.data() + 16, wb.data(), wb.size() * 2);
  return out;   // biases stay zero
}

// activations of `rows` rows: bf16 for inference, FP32 for training
struct Acts {
  long long cap = 0;
  int H = 0;
  bool f32 = false;
  void *H1 = nullptr, *H2 = nullptr;
  float *Y = nullptr;
  void ensure(long long rows, int h, bool train) {
    if (rows <= cap && h == H && train == f32) return;
    release();
    const size_t es = train ? 4 : 2;
    dev_alloc(&H1, (size_t)rows * h * es, "mlp h1");
    dev_alloc(&H2, (size_t)rows * h * es, "mlp h2");
    dev_alloc((void **)&Y, (size_t)rows * F_OUT * 4, "mlp y");
    cap = rows;
    H = h;
    f32 = train;
  }
  void release() {
    for (void *p : {H1, H2, (void *)Y})
      if (p) hipFree(p);
    H1 = H2 = nullptr;
    Y = nullptr;
    cap = 0;
  }
};

void forward(const Net &n, long long rows, const uint16_t *X, Acts &a, hipStream_t st, float *Y = nullptr) {
  const Shape &s = n.s;
  const int M = (int)rows, t = a.f32 ? 1 : 0;
  float *h1f = t ? (float *)a.H1 : nullptr, *h2f = t ? (float *)a.H2 : nullptr;
  uint16_t *h1b = t ? nullptr : (uint16_t *)a.H1, *h2b = t ? nullptr : (uint16_t *)a.H2;
  gemm({M, s.H, s.F, X, s.F, 1, 0, n.W1(), 1, s.F, 0, n.b1(), nullptr, 1, h1f, h1b, s.H}, st);
  gemm({M, s.H, s.H, a.H1, s.H, 1, t, n.W2(), 1, s.H, 0, n.b2(), nullptr, 1, h2f, h2b, s.H}, st);
  gemm({M, s.O, s.H, a.H2, s.H, 1, t, n.W3(), 1, s.H, 0, n.b3(), nullptr, 0, Y ? Y : a.Y, nullptr, s.O}, st);
}

// inference over many rows in chunks of at most INFER_CHUNK (the hidden
// activations of a chunk: 2 x INFER_CHUNK x H bf16), outputs into Y[rows][2]
constexpr long long INFER_CHUNK = 1LL << 22;
void forward_chunked(const Net &n, long long rows, const uint16_t *X, Acts &a, float *Y, hipStream_t st) {
  a.ensure(std::min(rows, INFER_CHUNK), n.s.H, false);
  for (long long r0 = 0; r0 < rows; r0 += INFER_CHUNK) {
    const long long m = std::min(INFER_CHUNK, rows - r0);
    forward(n, m, X + r0 * n.s.F, a, st, Y + 2 * r0);
  }
}

// backward buffers for B rows (FP32)
struct Grads {
  long long cap = 0;
  int H = 0;
  float *dy = nullptr, *dH2 = nullptr, *dH1 = nullptr, *cpart = nullptr;
  double *lpart = nullptr;
  void ensure(long long rows, int h) {
    if (rows <= cap && h == H) return;
    release();
    dev_alloc((void **)&dy, (size_t)rows * F_OUT * 4, "dy");
    dev_alloc((void **)&dH2, (size_t)rows * h * 4, "dh2");
    dev_alloc((void **)&dH1, (size_t)rows * h * 4, "dh1");
    dev_alloc((void **)&cpart, (size_t)COLSUM_SPLIT * std::max(h, F_OUT) * 4, "colsum partials");
    dev_alloc((void **)&lpart, (size_t)((rows + 255) / 256) * 8, "loss partials");
    cap = rows;
    H = h;
  }
  void release() {
    for (void *p : {(void *)dy, (void *)dH2, (void *)dH1, (void *)cpart, (void *)lpart})
      if (p) hipFree(p);
    *this = Grads();
  }
};

// loss (into lossv[slot]) and gradients (into n.G) of rows X, targets T,
// weights w * wscale; a holds the FP32 activations of forward(X)
void backward(Net &n, int B, const uint16_t *X, const float *T, const float *w, double wscale, Acts &a, Grads &g,
              double *lossv, int slot, hipStream_t st) {
  const Shape &s = n.s;
  const int H = s.H, F = s.F, O = s.O;
  float *gW1 = n.G, *gW2 = n.G + (long long)H * F, *gW3 = gW2 + (long long)H * H;
  float *gb1 = n.G + s.nw(), *gb2 = gb1 + H, *gb3 = gb2 + H;
  const float *H1 = (const float *)a.H1, *H2 = (const float *)a.H2;
  const int nb = (B + 255) / 256;
  k_loss<<<nb, 256, 0, st>>>(a.Y, T, w, wscale, B, g.dy, g.lpart);
  k_sum_final<<<1, 1, 0, st>>>(g.lpart, nb, lossv, slot);
  // output layer: gW3 = dy^T H2, gb3 = sum dy, dH2 = (dy W3) * [H2 > 0]
  gemm({O, H, B, g.dy, 1, O, 1, H2, H, 1, 1, nullptr, nullptr, 0, gW3, nullptr, H}, st);
  colsum(g.dy, B, O, O, g.cpart, gb3, st);
  gemm({B, H, O, g.dy, O, 1, 1, n.W3(), H, 1, 0, nullptr, H2, 0, g.dH2, nullptr, H}, st);
  // second hidden layer: gW2 = dH2^T H1, gb2, dH1 = (dH2 W2) * [H1 > 0]
  gemm({H, H, B, g.dH2, 1, H, 1, H1, H, 1, 1, nullptr, nullptr, 0, gW2, nullptr, H}, st);
  colsum(g.dH2, B, H, H, g.cpart, gb2, st);
  gemm({B, H, H, g.dH2, H, 1, 1, n.W2(), H, 1, 0, nullptr, H1, 0, g.dH1, nullptr, H}, st);
  // first hidden layer: gW1 = dH1^T X, gb1
  gemm({H, F, B, g.dH1, 1, H, 1, X, F, 1, 0, nullptr, nullptr, 0, gW1, nullptr, F}, st);
  colsum(g.dH1, B, H, H, g.cpart, gb1, st);
}

}  // namespace

// ---------------------------------------------------------------------------
// per-context state
// ---------------------------------------------------------------------------
struct Learned {
  Net net;
  bool have = false;
  long long *stats = nullptr;   // [2] device: applications, numeric fallbacks
  long long judged_off = 0;     // right-hand sides switched back to plain P
  double judge = 0.0;           // plain per-step reduction factor x 1.1 (0: unknown)
  uint8_t *en = nullptr;        // [cap_R] device enable mask
  std::vector<uint8_t> en_host;
  uint8_t *self_loop = nullptr; // [l]
  int *n1_off = nullptr, *n1 = nullptr, *n2_off = nullptr, *n2 = nullptr;  // link-neighbour rings
  // inference (hidden activations per chunk of rows; outputs of all rows)
  Acts act;
  float *Yall = nullptr;
  long long cap_y = 0;
  long long cap_rows = 0;
  uint16_t *X = nullptr;
  int cap_R = 0;
  double *nrm = nullptr;
  uint8_t *ok = nullptr;
  float *logf = nullptr;
  std::vector<double> logf_omega;
  // training set
  long long rows = 0, cap_set = 0;
  uint16_t *Xs = nullptr;
  float *Ts = nullptr;
  int *gs = nullptr;
  std::vector<double> den;
  // training minibatch
  Acts bact;
  Grads grads;
  long long cap_B = 0;
  uint16_t *Xb = nullptr;
  float *Tb = nullptr, *wb = nullptr;
  double *d_loss = nullptr;
  long long cap_loss = 0;
};

namespace {

Learned *learned_of(pfft_ctx *c, hipStream_t st) {
  if (c->learned) return c->learned;
  Learned *L = new Learned();
  c->learned = L;
  const HostModel &m = c->m;
  std::vector<uint8_t> sl(m.l, 0);
  for (int i = 0; i < m.l; ++i) {
    const int e = m.links[i];
    sl[i] = (e < m.b && m.bu[e] == m.bv[e]) ? 1 : 0;
  }
  dev_alloc((void **)&L->self_loop, m.l, "self loops");
  hip_ok(hipMemcpyAsync(L->self_loop, sl.data(), m.l, hipMemcpyHostToDevice, st), "self loops");
  // link neighbours of loop i (loop i = the cycle of link branch links[i]):
  // ring 1, the other links at the two end nodes of its link; ring 2, the
  // links at the nodes one branch away from those ends (not in ring 1)
  {
    const int nn = m.nn, nbr = (int)m.bu.size();
    std::vector<int> ln_off(nn + 1, 0), ln, adj_off(nn + 1, 0), adj;
    for (int i = 0; i < m.l; ++i) {
      const int e = m.links[i];
      ln_off[m.bu[e] + 1]++;
      if (m.bv[e] != m.bu[e]) ln_off[m.bv[e] + 1]++;
    }
    for (int k = 0; k < nn; ++k) ln_off[k + 1] += ln_off[k];
    ln.resize(ln_off[nn]);
    {
      std::vector<int> fill(ln_off.begin(), ln_off.end() - 1);
      for (int i = 0; i < m.l; ++i) {
        const int e = m.links[i];
        ln[fill[m.bu[e]]++] = i;
        if (m.bv[e] != m.bu[e]) ln[fill[m.bv[e]]++] = i;
      }
    }
    for (int e = 0; e < nbr; ++e)
      if (m.bu[e] != m.bv[e]) {
        adj_off[m.bu[e] + 1]++;
        adj_off[m.bv[e] + 1]++;
      }
    for (int k = 0; k < nn; ++k) adj_off[k + 1] += adj_off[k];
    adj.resize(adj_off[nn]);
    {
      std::vector<int> fill(adj_off.begin(), adj_off.end() - 1);
      for (int e = 0; e < nbr; ++e)
        if (m.bu[e] != m.bv[e]) {
          adj[fill[m.bu[e]]++] = m.bv[e];
          adj[fill[m.bv[e]]++] = m.bu[e];
        }
    }
    std::vector<int> o1(m.l + 1, 0), o2(m.l + 1, 0), r1, r2;
    std::vector<std::vector<int>> s1(m.l), s2(m.l);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int i = 0; i < m.l; ++i) {
      const int e = m.links[i];
      const int ends[2] = {m.bu[e], m.bv[e]};
      auto &a1 = s1[i];
      auto &a2 = s2[i];
      for (int x : ends)
        for (int k = ln_off[x]; k < ln_off[x + 1]; ++k)
          if (ln[k] != i) a1.push_back(ln[k]);
      std::sort(a1.begin(), a1.end());
      a1.erase(std::unique(a1.begin(), a1.end()), a1.end());
      for (int x : ends)
        for (int q = adj_off[x]; q < adj_off[x + 1]; ++q) {
          const int y = adj[q];
          for (int k = ln_off[y]; k < ln_off[y + 1]; ++k)
            if (ln[k] != i && !std::binary_search(a1.begin(), a1.end(), ln[k])) a2.push_back(ln[k]);
        }
      std::sort(a2.begin(), a2.end());
      a2.erase(std::unique(a2.begin(), a2.end()), a2.end());
    }
    for (int i = 0; i < m.l; ++i) {
      o1[i + 1] = o1[i] + (int)s1[i].size();
      o2[i + 1] = o2[i] + (int)s2[i].size();
    }
    r1.reserve(o1[m.l]);
    r2.reserve(o2[m.l]);
    for (int i = 0; i < m.l; ++i) {
      r1.insert(r1.end(), s1[i].begin(), s1[i].end());
      r2.insert(r2.end(), s2[i].begin(), s2[i].end());
    }
    auto up = [&](int **d, const std::vector<int> &h, const char *what) {
      dev_alloc((void **)d, std::max<size_t>(h.size(), 1) * sizeof(int), what);
      if (!h.empty()) hip_ok(hipMemcpyAsync(*d, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice, st), what);
    };
    up(&L->n1_off, o1, "ring 1");
    up(&L->n1, r1, "ring 1");
    up(&L->n2_off, o2, "ring 2");
    up(&L->n2, r2, "ring 2");
    hip_ok(hipStreamSynchronize(st), "rings");
  }
  dev_alloc((void **)&L->stats, 2 * sizeof(long long), "learned stats");
  hip_ok(hipMemsetAsync(L->stats, 0, 2 * sizeof(long long), st), "learned stats");
  hip_ok(hipStreamSynchronize(st), "learned init");
  return L;
}

void ensure_infer(Learned *L, int R, int l) {
  const long long rows = (long long)R * l;
  if (rows > L->cap_rows) {
    if (L->X) hipFree(L->X);
    dev_alloc((void **)&L->X, (size_t)rows * F_IN * 2, "features");
    L->cap_rows = rows;
  }
  if (R > L->cap_R) {
    for (void *p : {(void *)L->nrm, (void *)L->ok, (void *)L->logf, (void *)L->en})
      if (p) hipFree(p);
    dev_alloc((void **)&L->en, (size_t)R, "enable");
    L->en_host.clear();
    dev_alloc((void **)&L->nrm, (size_t)R * 2 * 8, "norms");
    dev_alloc((void **)&L->ok, (size_t)R, "ok");
    dev_alloc((void **)&L->logf, (size_t)R * 4, "log f");
    L->cap_R = R;
    L->logf_omega.clear();
  }
}

void set_logf(Learned *L, int R, const double *omega, hipStream_t st) {
  std::vector<double> om(omega, omega + R);
  if (om == L->logf_omega) return;
  std::vector<float> lf(R);
  for (int r = 0; r < R; ++r) lf[r] = (float)((std::log10(omega[r] / (2.0 * M_PI)) - 8.0) / 2.0);
  hip_ok(hipMemcpyAsync(L->logf, lf.data(), R * 4, hipMemcpyHostToDevice, st), "log f");
  hip_ok(hipStreamSynchronize(st), "log f sync");
  L->logf_omega = om;
}

// features of v (with z = P^-1 v already computed) into L->X; norms into L->nrm
void features(pfft_ctx *c, Learned *L, Precond *P, int R, const double *omega, const double2 *v, const double2 *z,
              hipStream_t st) {
  const int l = c->m.l;
  ensure_infer(L, R, l);
  set_logf(L, R, omega, st);
  k_norms<<<R, 256, 0, st>>>(v, z, l, L->nrm);
  FeatArgs a{v, z, L->nrm, P->d_fidx, P->dev.yinv, P->dev.link_kind, L->self_loop, L->logf,
             L->n1_off, L->n1, L->n2_off, L->n2, l, c->m.b, R, L->X};
  const long long n = (long long)R * l;
  k_features<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(a);
}

void grow_set(Learned *L, long long need) {
  if (need <= L->cap_set) return;
  long long cap = std::max(need, 2 * L->cap_set);
  uint16_t *X;
  float *T;
  int *g;
  dev_alloc((void **)&X, (size_t)cap * F_IN * 2, "training features");
  dev_alloc((void **)&T, (size_t)cap * 2 * 4, "training targets");
  dev_alloc((void **)&g, (size_t)cap * 4, "training groups");
  if (L->rows) {
    hip_ok(hipMemcpy(X, L->Xs, (size_t)L->rows * F_IN * 2, hipMemcpyDeviceToDevice), "grow X");
    hip_ok(hipMemcpy(T, L->Ts, (size_t)L->rows * 2 * 4, hipMemcpyDeviceToDevice), "grow T");
    hip_ok(hipMemcpy(g, L->gs, (size_t)L->rows * 4, hipMemcpyDeviceToDevice), "grow g");
  }
  for (void *p : {(void *)L->Xs, (void *)L->Ts, (void *)L->gs})
    if (p) hipFree(p);
  L->Xs = X;
  L->Ts = T;
  L->gs = g;
  L->cap_set = cap;
}

void clear_set(Learned *L) {
  for (void *p : {(void *)L->Xs, (void *)L->Ts, (void *)L->gs})
    if (p) hipFree(p);
  L->Xs = nullptr;
  L->Ts = nullptr;
  L->gs = nullptr;
  L->rows = L->cap_set = 0;
  L->den.clear();
}

pfft_status fail(const char *where, const std::string &msg, int code) {
  set_error(std::string(where) + ": " + msg);
  return (pfft_status)code;
}

}  // namespace

double learned_judge_factor(pfft_ctx *c) { return c->learned ? c->learned->judge : 0.0; }

void learned_set_judge(pfft_ctx *c, double factor) { learned_of(c, nullptr)->judge = factor; }

void learned_judged_off(pfft_ctx *c, int n) {
  if (c->learned) c->learned->judged_off += n;
}

bool learned_apply(pfft_ctx *c, int R, const double *omega, const double2 *v, double2 *z, const uint8_t *enable,
                   hipStream_t st) {
  Learned *L = c->learned;
  if (!L || !L->have) return false;
  std::vector<uint8_t> en(R, 1);
  if (enable) en.assign(enable, enable + R);
  if (std::none_of(en.begin(), en.end(), [](uint8_t e) { return e != 0; })) return false;
  Precond *P = precond_prepare(c, R, omega, st);
  precond_apply(P->dev, P->d_fidx, v, z, P->d_work, R, st);
  const int l = c->m.l;
  features(c, L, P, R, omega, v, z, st);
  if (en != L->en_host) {
    hip_ok(hipMemcpyAsync(L->en, en.data(), R, hipMemcpyHostToDevice, st), "enable mask");
    hip_ok(hipStreamSynchronize(st), "enable sync");
    L->en_host = en;
  }
  const long long rows = (long long)R * l;
  if (rows > L->cap_y) {
    if (L->Yall) hipFree(L->Yall);
    dev_alloc((void **)&L->Yall, (size_t)rows * F_OUT * 4, "mlp outputs");
    L->cap_y = rows;
  }
  forward_chunked(L->net, rows, L->X, L->act, L->Yall, st);
  k_check<<<R, 256, 0, st>>>(L->Yall, l, DELTA_CAP2 * l, L->ok);
  k_correct<<<(unsigned)((rows + 255) / 256), 256, 0, st>>>(z, L->Yall, L->nrm, L->ok, L->en, l, R);
  k_stats<<<1, 1, 0, st>>>(L->ok, L->en, R, L->stats);
  hip_ok(hipGetLastError(), "learned apply");
  return true;
}

void learned_free(pfft_ctx *c) {
  Learned *L = c->learned;
  if (!L) return;
  net_free(L->net);
  L->act.release();
  L->bact.release();
  L->grads.release();
  clear_set(L);
  for (void *p : {(void *)L->n1_off, (void *)L->n1, (void *)L->n2_off, (void *)L->n2, (void *)L->Yall})
    if (p) hipFree(p);
  for (void *p : {(void *)L->stats, (void *)L->en, (void *)L->self_loop, (void *)L->X, (void *)L->nrm, (void *)L->ok,
                  (void *)L->logf, (void *)L->Xb, (void *)L->Tb, (void *)L->wb, (void *)L->d_loss})
    if (p) hipFree(p);
  delete L;
  c->learned = nullptr;
}

}  // namespace pfft

using namespace pfft;

extern "C" {

pfft_status pfft_precond_load(pfft_ctx *c, const void *blob, int64_t nbytes) {
  Shape s;
  if (!c || !parse_header(blob, nbytes, s)) return fail("pfft_precond_load", "malformed weight blob", PFFT_EINVAL);
  if (s.F != F_IN || s.O != F_OUT)
    return fail("pfft_precond_load", "the correction network needs F = 16 inputs and O = 2 outputs", PFFT_EINVAL);
  try {
    hip_ok(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t st = nullptr;
    Learned *L = learned_of(c, st);
    net_from_blob(L->net, s, blob, st);
    hip_ok(hipMemset(L->stats, 0, 2 * sizeof(long long)), "stats");
    L->judged_off = 0;
    L->have = true;
    return PFFT_OK;
  } catch (const DeviceError &e) {
    return fail("pfft_precond_load", e.msg, e.code);
  }
}

pfft_status pfft_precond_save(pfft_ctx *c, void *buf, int64_t cap_bytes, int64_t *nbytes) {
  if (!c || !nbytes) return fail("pfft_precond_save", "bad argument", PFFT_EINVAL);
  if (!c->learned || !c->learned->have) return fail("pfft_precond_save", "no network", PFFT_EINVAL);
  try {
    hip_ok(hipSetDevice(c->device), "hipSetDevice");
    std::vector<uint8_t> b = net_to_blob(c->learned->net, nullptr);
    *nbytes = (int64_t)b.size();
    if (buf && cap_bytes >= (int64_t)b.size()) memcpy(buf, b.data(), b.size());
    return PFFT_OK;
  } catch (const DeviceError &e) {
    return fail("pfft_precond_save", e.msg, e.code);
  }
}

pfft_status pfft_learned_collect(pfft_ctx *c, int32_t nfreq, const double *freq_hz, double tol, int32_t maxit,
                                 int64_t *rows_out, void *hip_stream) {
  if (!c || nfreq <= 0 || !freq_hz || !(tol > 0) || maxit <= 0)
    return fail("pfft_learned_collect", "bad argument", PFFT_EINVAL);
  if (c->m.p == 0) return fail("pfft_learned_collect", "the problem has no ports", PFFT_EINVAL);
  for (int f = 0; f < nfreq; ++f)
    if (!(freq_hz[f] > 0)) return fail("pfft_learned_collect", "frequencies must be positive", PFFT_EINVAL);
  double2 *E = nullptr, *vk = nullptr, *zk = nullptr, *hk = nullptr;
  double *dots = nullptr, *coef = nullptr, *tn = nullptr;
  float *Tt = nullptr;
  auto cleanup = [&]() {
    for (void *p : {(void *)E, (void *)vk, (void *)zk, (void *)hk, (void *)dots, (void *)coef, (void *)tn,
                    (void *)Tt})
      if (p) hipFree(p);
  };
  try {
    hip_ok(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t st = (hipStream_t)hip_stream;
    Learned *L = learned_of(c, st);
    KrylovFn done = [&](const KrylovView &kv) {
      const int R = kv.R, l = kv.l, m = kv.m;
      const size_t vec = (size_t)R * l * sizeof(double2);
      int K = 0;
      for (int r = 0; r < R; ++r) K = std::max(K, kv.k[r]);
      if (K == 0) return;
      {  // plain per-step residual reduction factor (median over the RHS)
        std::vector<double> q;
        for (int r = 0; r < R; ++r)
          if (kv.k[r] > 0 && kv.relres[r] > 0) q.push_back(std::pow(kv.relres[r], 1.0 / kv.k[r]));
        if (!q.empty()) {
          std::nth_element(q.begin(), q.begin() + q.size() / 2, q.end());
          L->judge = std::min(1.1 * q[q.size() / 2], 0.999);
        }
      }
      Precond *P = precond_prepare(c, R, kv.omega, st);
      dev_alloc((void **)&E, vec * K, "collect errors");
      dev_alloc((void **)&vk, vec, "collect v");
      dev_alloc((void **)&zk, vec, "collect z");
      dev_alloc((void **)&hk, (size_t)R * (K + 1) * sizeof(double2), "collect h");
      dev_alloc((void **)&dots, (size_t)R * 4 * 8, "collect dots");
      dev_alloc((void **)&coef, (size_t)R * 3 * 8, "collect coef");
      dev_alloc((void **)&tn, (size_t)R * 8, "collect tnorm");
      dev_alloc((void **)&Tt, (size_t)R * l * 2 * 4, "collect targets");
      const long long n = (long long)R * l;
      const unsigned nb = (unsigned)((n + 255) / 256);
      // e_0 = Z_l^-1 v_0 = x / |b|
      std::vector<double> inv_b(R);
      for (int r = 0; r < R; ++r) inv_b[r] = kv.bnorm[r] > 0 ? 1.0 / kv.bnorm[r] : 0.0;
      hip_ok(hipMemcpyAsync(coef, inv_b.data(), R * 8, hipMemcpyHostToDevice, st), "inv b");
      k_scale_rows<<<dim3((l + 255) / 256, R), 256, 0, st>>>(kv.x, coef, l, E);
      // e_{k+1} = (z_k - sum_{i<=k} H[i][k] e_i) / H[k+1][k]
      for (int k = 0; k + 1 < K; ++k)
        k_krylov_error<<<dim3((l + 255) / 256, R), 256, 0, st>>>(kv.Z, kv.Hraw, E, l, m, k, R);
      std::vector<double> hd(4 * R), hc(3 * R), ht(R);
      for (int k = 0; k < K; ++k) {
        // pairs kept while the estimated error of e_k stays below 1e-3:
        // |r_k| >= 1e3 |r_final|
        std::vector<int> keep;
        for (int r = 0; r < R; ++r) {
          if (k >= kv.k[r]) continue;
          const double rk = k == 0 ? kv.bnorm[r] : kv.res[r][k - 1];
          if (rk >= 1e3 * kv.relres[r] * kv.bnorm[r]) keep.push_back(r);
        }
        if (keep.empty()) continue;
        // contiguous v_k, z_k of every RHS
        hip_ok(hipMemcpy2DAsync(vk, l * sizeof(double2), kv.V + (size_t)k * l, (size_t)(m + 1) * l * sizeof(double2),
                                l * sizeof(double2), R, hipMemcpyDeviceToDevice, st),
               "gather v");
        hip_ok(hipMemcpy2DAsync(zk, l * sizeof(double2), kv.Z + (size_t)k * l, (size_t)m * l * sizeof(double2),
                                l * sizeof(double2), R, hipMemcpyDeviceToDevice, st),
               "gather z");
        const double2 *ek = E + (size_t)k * R * l;
        k_dots<<<R, 256, 0, st>>>(vk, zk, ek, l, dots);
        hip_ok(hipMemcpyAsync(hd.data(), dots, 4 * R * 8, hipMemcpyDeviceToHost, st), "dots");
        hip_ok(hipStreamSynchronize(st), "dots sync");
        std::vector<int> keep2;
        for (int r = 0; r < R; ++r) hc[3 * r] = hc[3 * r + 1] = hc[3 * r + 2] = 0.0;
        for (int r : keep) {
          const double nz = hd[4 * r + 1];
          const std::complex<double> ze(hd[4 * r + 2], hd[4 * r + 3]);
          if (!(nz > 0) || !(std::abs(ze) > 0)) continue;
          const std::complex<double> g = nz / ze;
          hc[3 * r] = g.real();
          hc[3 * r + 1] = g.imag();
          hc[3 * r + 2] = std::sqrt(l / nz);
          keep2.push_back(r);
        }
        if (keep2.empty()) continue;
        hip_ok(hipMemcpyAsync(coef, hc.data(), 3 * R * 8, hipMemcpyHostToDevice, st), "coef");
        k_targets<<<nb, 256, 0, st>>>(zk, ek, coef, l, R, Tt);
        k_tnorm<<<R, 256, 0, st>>>(Tt, l, tn);
        features(c, L, P, R, kv.omega, vk, zk, st);
        hip_ok(hipMemcpyAsync(ht.data(), tn, R * 8, hipMemcpyDeviceToHost, st), "tnorm");
        hip_ok(hipStreamSynchronize(st), "tnorm sync");
        grow_set(L, L->rows + (long long)keep2.size() * l);
        for (int r : keep2) {
          if (!(ht[r] > 0)) continue;
          const long long o = L->rows;
          hip_ok(hipMemcpyAsync(L->Xs + o * F_IN, L->X + (size_t)r * l * F_IN, (size_t)l * F_IN * 2,
                                hipMemcpyDeviceToDevice, st),
                 "append X");
          hip_ok(hipMemcpyAsync(L->Ts + o * 2, Tt + (size_t)r * l * 2, (size_t)l * 2 * 4, hipMemcpyDeviceToDevice, st),
                 "append T");
          k_fill_int<<<(l + 255) / 256, 256, 0, st>>>(L->gs + o, l, (int)L->den.size());
          L->den.push_back(ht[r]);
          L->rows += l;
        }
        hip_ok(hipStreamSynchronize(st), "append sync");
      }
    };
    solve_ports_krylov(c, nfreq, freq_hz, tol, maxit, done, st);
    cleanup();
    if (rows_out) *rows_out = c->learned->rows;
    return PFFT_OK;
  } catch (const DeviceError &ex) {
    cleanup();
    return fail("pfft_learned_collect", ex.msg, ex.code);
  } catch (const SetupError &ex) {
    cleanup();
    return fail("pfft_learned_collect", ex.msg, ex.code);
  }
}

pfft_status pfft_learned_train(pfft_ctx *c, int32_t steps, int32_t batch, int32_t hidden, double lr, uint64_t seed,
                               float *loss_out, void *hip_stream) {
  if (!c || steps < 0 || batch <= 0 || !(lr > 0) || hidden <= 0 || hidden > 4096)
    return fail("pfft_learned_train", "bad argument", PFFT_EINVAL);
  Learned *L = c->learned;
  if (!L || L->rows == 0) return fail("pfft_learned_train", "the training set is empty", PFFT_EINVAL);
  try {
    hip_ok(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t st = (hipStream_t)hip_stream;
    if (!L->have) {
      std::vector<uint8_t> b = init_blob(hidden, seed);
      Shape s;
      parse_header(b.data(), (long long)b.size(), s);
      net_from_blob(L->net, s, b.data(), st);
      hip_ok(hipMemset(L->stats, 0, 2 * sizeof(long long)), "stats");
      L->judged_off = 0;
      L->have = true;
    }
    Net &n = L->net;
    const int H = n.s.H;
    if (batch > L->cap_B) {
      for (void *p : {(void *)L->Xb, (void *)L->Tb, (void *)L->wb})
        if (p) hipFree(p);
      dev_alloc((void **)&L->Xb, (size_t)batch * F_IN * 2, "batch X");
      dev_alloc((void **)&L->Tb, (size_t)batch * 2 * 4, "batch T");
      dev_alloc((void **)&L->wb, (size_t)batch * 4, "batch w");
      L->cap_B = batch;
    }
    L->bact.ensure(batch, H, true);
    L->grads.ensure(batch, H);
    if (steps > L->cap_loss) {
      if (L->d_loss) hipFree(L->d_loss);
      dev_alloc((void **)&L->d_loss, (size_t)steps * 8, "loss history");
      L->cap_loss = steps;
    }
    const int G = (int)L->den.size();
    double *d_den;
    dev_alloc((void **)&d_den, (size_t)G * 8, "group norms");
    hip_ok(hipMemcpyAsync(d_den, L->den.data(), (size_t)G * 8, hipMemcpyHostToDevice, st), "group norms");
    const double wscale = (double)L->rows / batch;
    const long long np = n.s.np();
    for (int s = 0; s < steps; ++s) {
      k_gather<<<(batch + 255) / 256, 256, 0, st>>>(L->Xs, L->Ts, L->gs, d_den, G, L->rows, seed, n.adam_t, batch,
                                                     F_IN, L->Xb, L->Tb, L->wb);
      forward(n, batch, L->Xb, L->bact, st);
      backward(n, batch, L->Xb, L->Tb, L->wb, wscale, L->bact, L->grads, L->d_loss, s, st);
      ++n.adam_t;
      const double b1 = 0.9, b2 = 0.999;
      k_adam<<<(unsigned)((np + 255) / 256), 256, 0, st>>>(
          n.P, n.Mm, n.Vv, n.G, (int)np, (float)lr, (float)b1, (float)b2, 1e-8f,
          (float)(1.0 - std::pow(b1, (double)n.adam_t)), (float)(1.0 - std::pow(b2, (double)n.adam_t)), n.Wb,
          (int)n.s.nw());
    }
    hip_ok(hipGetLastError(), "train launch");
    std::vector<double> lh(steps);
    if (steps) hip_ok(hipMemcpyAsync(lh.data(), L->d_loss, (size_t)steps * 8, hipMemcpyDeviceToHost, st), "loss");
    hip_ok(hipStreamSynchronize(st), "train sync");
    hipFree(d_den);
    if (loss_out)
      for (int s = 0; s < steps; ++s) loss_out[s] = (float)lh[s];
    return PFFT_OK;
  } catch (const DeviceError &e) {
    return fail("pfft_learned_train", e.msg, e.code);
  }
}

pfft_status pfft_learned_eval(pfft_ctx *c, double *loss_out, void *hip_stream) {
  if (!c || !loss_out) return fail("pfft_learned_eval", "bad argument", PFFT_EINVAL);
  Learned *L = c->learned;
  if (!L || L->rows == 0) return fail("pfft_learned_eval", "the training set is empty", PFFT_EINVAL);
  if (!L->have) return fail("pfft_learned_eval", "no network", PFFT_EINVAL);
  double *d_den = nullptr, *part = nullptr;
  try {
    hip_ok(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t st = (hipStream_t)hip_stream;
    const int G = (int)L->den.size();
    constexpr int CH = 65536;
    dev_alloc((void **)&d_den, (size_t)G * 8, "group norms");
    dev_alloc((void **)&part, (size_t)(CH / 256) * 8, "loss partials");
    hip_ok(hipMemcpyAsync(d_den, L->den.data(), (size_t)G * 8, hipMemcpyHostToDevice, st), "group norms");
    Acts a;
    a.ensure(CH, L->net.s.H, true);
    double total = 0;
    std::vector<double> hp(CH / 256);
    for (long long o = 0; o < L->rows; o += CH) {
      const int n = (int)std::min<long long>(CH, L->rows - o);
      forward(L->net, n, L->Xs + o * F_IN, a, st);
      const int nb = (n + 255) / 256;
      k_set_loss<<<nb, 256, 0, st>>>(a.Y, L->Ts + o * 2, L->gs + o, d_den, G, n, part);
      hip_ok(hipMemcpyAsync(hp.data(), part, nb * 8, hipMemcpyDeviceToHost, st), "loss partials");
      hip_ok(hipStreamSynchronize(st), "eval sync");
      for (int i = 0; i < nb; ++i) total += hp[i];
    }
    a.release();
    hipFree(d_den);
    hipFree(part);
    *loss_out = total;
    return PFFT_OK;
  } catch (const DeviceError &e) {
    if (d_den) hipFree(d_den);
    if (part) hipFree(part);
    return fail("pfft_learned_eval", e.msg, e.code);
  }
}

pfft_status pfft_learned_clear(pfft_ctx *c) {
  if (!c) return fail("pfft_learned_clear", "bad argument", PFFT_EINVAL);
  if (c->learned) clear_set(c->learned);
  return PFFT_OK;
}

pfft_status pfft_learned_stats(pfft_ctx *c, int64_t out[3]) {
  if (!c || !out) return fail("pfft_learned_stats", "bad argument", PFFT_EINVAL);
  out[0] = out[1] = out[2] = 0;
  if (!c->learned) return PFFT_OK;
  try {
    hip_ok(hipSetDevice(c->device), "hipSetDevice");
    long long h[2];
    hip_ok(hipDeviceSynchronize(), "stats sync");
    hip_ok(hipMemcpy(h, c->learned->stats, sizeof(h), hipMemcpyDeviceToHost), "stats");
    out[0] = h[0];
    out[1] = h[1];
    out[2] = c->learned->judged_off;
    return PFFT_OK;
  } catch (const DeviceError &e) {
    return fail("pfft_learned_stats", e.msg, e.code);
  }
}

pfft_status pfft_mlp_grad(int32_t rows, const void *blob, int64_t nbytes, const void *X_dev, const float *T_dev,
                          const float *w_dev, float *Y_dev, float *grad_dev, double *loss_out, void *hip_stream) {
  Shape s;
  if (rows <= 0 || !X_dev || !T_dev || !w_dev || !Y_dev || !grad_dev || !loss_out)
    return fail("pfft_mlp_grad", "bad argument", PFFT_EINVAL);
  if (!parse_header(blob, nbytes, s) || s.O != F_OUT)
    return fail("pfft_mlp_grad", "malformed weight blob (O must be 2)", PFFT_EINVAL);
  Net n;
  Acts a;
  Grads g;
  double *lv = nullptr;
  auto cleanup = [&]() {
    net_free(n);
    a.release();
    g.release();
    if (lv) hipFree(lv);
  };
  try {
    hipStream_t st = (hipStream_t)hip_stream;
    net_from_blob(n, s, blob, st);
    a.ensure(rows, s.H, true);
    g.ensure(rows, s.H);
    dev_alloc((void **)&lv, 8, "loss");
    forward(n, rows, (const uint16_t *)X_dev, a, st);
    backward(n, rows, (const uint16_t *)X_dev, T_dev, w_dev, 1.0, a, g, lv, 0, st);
    hip_ok(hipMemcpyAsync(Y_dev, a.Y, (size_t)rows * F_OUT * 4, hipMemcpyDeviceToDevice, st), "y");
    hip_ok(hipMemcpyAsync(grad_dev, n.G, (size_t)s.np() * 4, hipMemcpyDeviceToDevice, st), "grad");
    hip_ok(hipMemcpyAsync(loss_out, lv, 8, hipMemcpyDeviceToHost, st), "loss");
    hip_ok(hipStreamSynchronize(st), "mlp grad sync");
    cleanup();
    return PFFT_OK;
  } catch (const DeviceError &e) {
    cleanup();
    return fail("pfft_mlp_grad", e.msg, e.code);
  }
}

}  // extern "C"
