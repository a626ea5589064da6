// Device kernels of the pFFT loop-space matrix-vector product for gfx950.
//
// Every product is a gather (no atomics), so results are bitwise
// reproducible run to run.  Complex numbers are float2/double2 (re, im).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <string>
#include <type_traits>

#include "kernels.h"
#include "xcd.h"

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

// Largest dynamic LDS allocation one workgroup may request (capped at 128 KB).
static int lds_budget() {
  static int v = -1;
  if (v < 0) {
    int dev = 0, q = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&q, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) q = 65536;
    v = std::max(65536, std::min(q, 131072));
  }
  return v;
}

// Raises a kernel's dynamic LDS limit above 64 KB once; false if refused.
static bool allow_lds(const void *fn, int bytes) {
  if (bytes <= 65536) return true;
  if (bytes > lds_budget()) return false;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return true;
}

// ===========================================================================
// batched prefix sums (complex128) down the columns of a [len][R] array
// (right-hand sides contiguous), three phases, deterministic: chunk sums,
// their scan, then each chunk's running sums
// ===========================================================================
constexpr int CS_RG = 64, CS_G = 8, CS_CH = 256;   // RHS per workgroup, row groups, rows per chunk

size_t scan_partials_size(int len, int R) { return (size_t)cdiv(len, CS_CH) * (size_t)R; }

__global__ void __launch_bounds__(CS_RG * CS_G) k_cscan_sums(const double2 *a, double2 *part, int len, int R) {
  __shared__ double2 sh[CS_G][CS_RG];
  const int lane = threadIdx.x % CS_RG, g = threadIdx.x / CS_RG, r = blockIdx.y * CS_RG + lane;
  const int ch = blockIdx.x;
  double sx = 0, sy = 0;
  if (r < R) {
    const int k0 = ch * CS_CH + g * (CS_CH / CS_G), k1 = min(len, k0 + CS_CH / CS_G);
    for (int k = k0; k < k1; ++k) {
      const double2 v = a[(size_t)k * R + r];
      sx += v.x;
      sy += v.y;
    }
  }
  sh[g][lane] = make_double2(sx, sy);
  __syncthreads();
  if (g == 0 && r < R) {
    double tx = 0, ty = 0;
    for (int j = 0; j < CS_G; ++j) {
      tx += sh[j][lane].x;
      ty += sh[j][lane].y;
    }
    part[(size_t)ch * R + r] = make_double2(tx, ty);
  }
}

// exclusive scan of the chunk sums over the nch chunks, per right-hand side;
// a thread's chunk sums are read 8 at a time (all loads in flight before
// the sums use them)
__global__ void __launch_bounds__(CS_RG * CS_G) k_cscan_part(double2 *part, int nch, int R) {
  constexpr int U = 8;
  __shared__ double2 sh[CS_G][CS_RG];
  const int lane = threadIdx.x % CS_RG, g = threadIdx.x / CS_RG, r = blockIdx.x * CS_RG + lane;
  const int per = (nch + CS_G - 1) / CS_G, c0 = g * per, c1 = min(nch, c0 + per);
  const int rr = min(r, R - 1);
  double sx = 0, sy = 0;
  for (int cb = c0; cb < c1; cb += U) {
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = part[(size_t)min(cb + u, c1 - 1) * R + rr];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (cb + u < c1) {
        sx += v[u].x;
        sy += v[u].y;
      }
  }
  sh[g][lane] = make_double2(sx, sy);
  __syncthreads();
  if (r >= R) return;
  double cx = 0, cy = 0;
  for (int j = 0; j < g; ++j) {
    cx += sh[j][lane].x;
    cy += sh[j][lane].y;
  }
  for (int cb = c0; cb < c1; cb += U) {
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = part[(size_t)min(cb + u, c1 - 1) * R + r];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (cb + u < c1) {
        part[(size_t)(cb + u) * R + r] = make_double2(cx, cy);
        cx += v[u].x;
        cy += v[u].y;
      }
  }
}

__global__ void __launch_bounds__(CS_RG * CS_G) k_cscan_final(const double2 *a, double2 *out, const double2 *part,
                                                              int len, int R, int inclusive) {
  __shared__ double2 sh[CS_G][CS_RG];
  const int lane = threadIdx.x % CS_RG, g = threadIdx.x / CS_RG, r = blockIdx.y * CS_RG + lane;
  const int ch = blockIdx.x;
  const int k0 = ch * CS_CH + g * (CS_CH / CS_G), k1 = min(len, k0 + CS_CH / CS_G);
  double sx = 0, sy = 0;
  if (r < R)
    for (int k = k0; k < k1; ++k) {
      const double2 v = a[(size_t)k * R + r];
      sx += v.x;
      sy += v.y;
    }
  sh[g][lane] = make_double2(sx, sy);
  __syncthreads();
  if (r >= R) return;
  const double2 p = part[(size_t)ch * R + r];
  double cx = p.x, cy = p.y;
  for (int j = 0; j < g; ++j) {
    cx += sh[j][lane].x;
    cy += sh[j][lane].y;
  }
  for (int k = k0; k < k1; ++k) {
    const double2 v = a[(size_t)k * R + r];
    if (inclusive) {
      cx += v.x;
      cy += v.y;
    }
    out[(size_t)k * R + r] = make_double2(cx, cy);
    if (!inclusive) {
      cx += v.x;
      cy += v.y;
    }
  }
}

// in place on a [len][R] array
static void scan_cols(double2 *a, int len, int R, bool inclusive, double2 *partials, hipStream_t st) {
  if (len <= 0 || R <= 0) return;
  const int nch = (int)cdiv(len, CS_CH), ng = (int)cdiv(R, CS_RG);
  k_cscan_sums<<<dim3(nch, ng), CS_RG * CS_G, 0, st>>>(a, partials, len, R);
  k_cscan_part<<<ng, CS_RG * CS_G, 0, st>>>(partials, nch, R);
  k_cscan_final<<<dim3(nch, ng), CS_RG * CS_G, 0, st>>>(a, a, partials, len, R, inclusive ? 1 : 0);
}

// ===========================================================================
// A^T: loop currents -> branch currents (Eq. CurT) by a subtree-sum scan.
// The scan runs down the preorder positions with the right-hand sides
// contiguous ([n'+1][R]), so every gather of a position or a link reads R
// consecutive values.  Threads are (position or branch, right-hand side) with
// 8 right-hand sides fastest.
// ===========================================================================
// scan[k][r] (k < nn, preorder position) = sum of +-x over links ending at the
// node; scan[nn][r] = 0.  xT: the loop vector as [l][R].
__global__ void k_inject(LoopMaps mp, const double2 *xT, double2 *scan, int R) {
  const int r = blockIdx.y * 8 + (threadIdx.x & 7);
  const int k = blockIdx.x * 32 + (threadIdx.x >> 3);
  if (k > mp.nn || r >= R) return;
  double sx = 0, sy = 0;
  if (k < mp.nn) {
    for (int q = mp.inj_off[k]; q < mp.inj_off[k + 1]; ++q) {
      const double2 v = xT[(size_t)mp.inj_link[q] * R + r];
      const double sg = mp.inj_sgn[q];
      sx += sg * v.x;
      sy += sg * v.y;
    }
  }
  scan[(size_t)k * R + r] = make_double2(sx, sy);
}

// after the exclusive scan: twig current = +-(P[hi] - P[lo]), link current = x;
// output alpha is RHS-contiguous: alpha[e][r]
__global__ void k_branch_out(LoopMaps mp, const double2 *xT, const double2 *pfx, double2 *alpha, int R) {
  const int r = blockIdx.y * 8 + (threadIdx.x & 7);
  const int e = blockIdx.x * 32 + (threadIdx.x >> 3);
  if (e >= mp.b || r >= R) return;
  const int a = mp.br_a[e];
  double2 v;
  if (a >= 0) {
    v = xT[(size_t)a * R + r];
  } else {
    const double2 hi = pfx[(size_t)mp.br_hi[e] * R + r], lo = pfx[(size_t)mp.br_lo[e] * R + r];
    const double sg = mp.br_sg[e];
    v = make_double2(sg * (hi.x - lo.x), sg * (hi.y - lo.y));
  }
  alpha[(size_t)e * R + r] = v;
}

// x: [R][l]; xT: scratch of l R complex values
void loop_to_branch(const LoopMaps &mp, const double2 *x, double2 *alpha, double2 *scan, double2 *partials,
                    double2 *xT, int R, hipStream_t st) {
  transpose(x, xT, R, mp.l, st);
  k_inject<<<dim3(cdiv(mp.nn + 1, 32), cdiv(R, 8)), 256, 0, st>>>(mp, xT, scan, R);
  scan_cols(scan, mp.nn + 1, R, false, partials, st);
  k_branch_out<<<dim3(cdiv(mp.b, 32), cdiv(R, 8)), 256, 0, st>>>(mp, xT, scan, alpha, R);
}

// ===========================================================================
// A: branch voltages -> loop voltages (Eq. VolT) by a potential scan, in the
// same [n'+1][R] layout
// ===========================================================================
// D[k] = s_k V(twig of k) - sum of s_j V(twig of j) over the nodes j whose
// subtree ends at k, from the flattened lists (same order of summation); the
// index loads of four entries are issued before their value loads
__global__ void k_drop_diff(LoopMaps mp, const double2 *yb, double2 *scan, int R) {
  const int r = blockIdx.y * 8 + (threadIdx.x & 7);
  const int k = blockIdx.x * 32 + (threadIdx.x >> 3);
  if (k >= mp.nn || r >= R) return;
  const int q0 = mp.dd_off[k], q1 = mp.dd_off[k + 1];
  double dx = 0, dy = 0;
  for (int q = q0; q < q1; q += 4) {
    int code[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) code[u] = q + u < q1 ? mp.dd_code[q + u] : -1;
    double2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = code[u] >= 0 ? yb[(size_t)(code[u] >> 1) * R + r] : make_double2(0, 0);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (code[u] >= 0) {
        if (code[u] & 1) {
          dx -= v[u].x;
          dy -= v[u].y;
        } else {
          dx += v[u].x;
          dy += v[u].y;
        }
      }
  }
  scan[(size_t)k * R + r] = make_double2(dx, dy);
}

// ylT[i][r]: the loop vector as [l][R]
__global__ void k_link_out(LoopMaps mp, const double2 *yb, const double2 *D, double2 *ylT, int R) {
  const int r = blockIdx.y * 8 + (threadIdx.x & 7);
  const int i = blockIdx.x * 32 + (threadIdx.x >> 3);
  if (i >= mp.l || r >= R) return;
  int e = mp.link_branch[i];
  double2 v = e < mp.b ? yb[(size_t)e * R + r] : make_double2(0, 0);
  int up = mp.link_upos[i], vp = mp.link_vpos[i];
  if (up >= 0) {
    const double2 dv = D[(size_t)vp * R + r], du = D[(size_t)up * R + r];
    v.x += dv.x - du.x;
    v.y += dv.y - du.y;
  }
  ylT[(size_t)i * R + r] = v;
}

// yl: [R][l]; ylT: scratch of l R complex values
void branch_to_loop(const LoopMaps &mp, const double2 *yb, double2 *yl, double2 *scan, double2 *partials,
                    double2 *ylT, int R, hipStream_t st) {
  k_drop_diff<<<dim3(cdiv(mp.nn, 32), cdiv(R, 8)), 256, 0, st>>>(mp, yb, scan, R);
  scan_cols(scan, mp.nn, R, true, partials, st);
  k_link_out<<<dim3(cdiv(mp.l, 32), cdiv(R, 8)), 256, 0, st>>>(mp, yb, scan, ylT, R);
  transpose(ylT, yl, mp.l, R, st);
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
  V2<T> *o = J + (size_t)idx * 4;   // J[t][r][4]
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
constexpr int PRG = 8;   // right-hand sides per thread in the projection

template <typename T>
__global__ void k_project(GridMaps g, const V2<T> *J, V2<T> *Q, int R) {
  const int r0 = blockIdx.y * PRG;
  const int node = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (node >= g.N) return;
  const int nr = min(PRG, R - r0);
  const T *w = (const T *)g.pg_w;
  T acc[PRG][6];
#pragma unroll
  for (int q = 0; q < PRG; ++q)
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[q][c] = 0;
  for (int k = g.pg_off[node]; k < g.pg_off[node + 1]; ++k) {
    const int t = g.pg_tri[k];
    const T m0 = w[4 * (size_t)k], m1x = w[4 * (size_t)k + 1], m1y = w[4 * (size_t)k + 2],
            m1z = w[4 * (size_t)k + 3];
    const V2<T> *jt = J + ((size_t)t * R + r0) * 4;
#pragma unroll
    for (int q = 0; q < PRG; ++q) {
      if (q < nr) {
        V2<T> j0 = jt[4 * q], jx = jt[4 * q + 1], jy = jt[4 * q + 2], jz = jt[4 * q + 3];
        acc[q][0] += j0.x * m1x - jx.x * m0;
        acc[q][1] += j0.y * m1x - jx.y * m0;
        acc[q][2] += j0.x * m1y - jy.x * m0;
        acc[q][3] += j0.y * m1y - jy.y * m0;
        acc[q][4] += j0.x * m1z - jz.x * m0;
        acc[q][5] += j0.y * m1z - jz.y * m0;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < PRG; ++q) {
    if (q < nr) {
      V2<T> *Qr = Q + (size_t)(r0 + q) * 3 * g.N;
      Qr[node] = cmk<T>(acc[q][0], acc[q][1]);
      Qr[g.N + node] = cmk<T>(acc[q][2], acc[q][3]);
      Qr[2 * (size_t)g.N + node] = cmk<T>(acc[q][4], acc[q][5]);
    }
  }
}

// Tiled projection: one workgroup per (tile, group of RC right-hand sides)
// stages the moments J of the tile's triangles in LDS once, then each node
// gathers its contributions from LDS (triangles beyond tcap from memory).
// Threads take the tile's nodes heaviest first, so a wavefront's lanes loop
// about equally long (most grid nodes have no contribution at all).  Every
// node is still a gather in a fixed order: no atomics.
template <typename T> struct ProjRC;
template <> struct ProjRC<float> { static constexpr int v = 4; };
template <> struct ProjRC<double> { static constexpr int v = 2; };
// groups of RC right-hand sides per workgroup: its wavefronts take (node
// chunk, group) pairs, so a tile's few active node chunks keep all of them
// busy
template <typename T> struct ProjRG;
template <> struct ProjRG<float> { static constexpr int v = 4; };
template <> struct ProjRG<double> { static constexpr int v = 1; };
// LDS pitch of one staged triangle: its RG x RC x 4 moments plus 16 bytes, so
// that the 16-byte reads of lanes gathering different triangles spread over
// the banks (a pitch that is a multiple of 128 bytes maps them to two bank
// groups)
template <typename T, int RG> constexpr int proj_pitch() {
  return RG * ProjRC<T>::v * 4 + 16 / (int)sizeof(V2<T>);
}

// skip_empty: node chunks without any contribution are not written (the
// pruned FFT passes never read inactive nodes)
template <typename T, int RG>
__global__ void __launch_bounds__(512) k_project_tiled(GridMaps g, const V2<T> *J, V2<T> *Q, int R, int skip_empty) {
  constexpr int RC = ProjRC<T>::v, RB = RC * RG;
  extern __shared__ unsigned char smraw[];
  constexpr int PS = proj_pitch<T, RG>();
  V2<T> *sJ = (V2<T> *)smraw;   // [tcap][PS]: (rr, comp) at rr * 4 + comp, rr < RB
  // one workgroup per (tile, group of RB right-hand sides), the groups of a
  // tile consecutive on one XCD: they read the tile's triangle and gather
  // lists through that XCD's L2
  const int ngrp = (R + RB - 1) / RB;
  const int lb = (int)xcd_block(blockIdx.x, gridDim.x), tile = lb / ngrp;
  const int rb0 = (lb - tile * ngrp) * RB, nrb = min(RB, R - rb0);
  const int t0 = g.tt_off[tile], nt = g.tt_off[tile + 1] - t0;
  const int ns = min(nt, g.tcap);
  // staging: SU (triangle index, moment) load pairs in flight per thread,
  // the index loads of a round issued before its moment loads
  constexpr int SU = 16;
  const int tot = ns * RB * 4;
  for (int i0 = threadIdx.x; i0 < tot; i0 += SU * blockDim.x) {
    int tri[SU];
#pragma unroll
    for (int u2 = 0; u2 < SU; ++u2) {
      const int i = min(i0 + u2 * (int)blockDim.x, tot - 1);
      tri[u2] = g.tt_tri[t0 + i / (RB * 4)];
    }
    V2<T> v[SU];
#pragma unroll
    for (int u2 = 0; u2 < SU; ++u2) {
      const int i = min(i0 + u2 * (int)blockDim.x, tot - 1);
      const int rem = i % (RB * 4), rr = rem >> 2, comp = rem & 3;
      v[u2] = rr < nrb ? J[((size_t)tri[u2] * R + rb0 + rr) * 4 + comp] : cmk<T>(0, 0);
    }
#pragma unroll
    for (int u2 = 0; u2 < SU; ++u2) {
      const int i = i0 + u2 * (int)blockDim.x;
      if (i < tot) {
        const int lt = i / (RB * 4), rem = i - lt * (RB * 4);
        sJ[lt * PS + rem] = v[u2];
      }
    }
  }
  __syncthreads();
  const int TX = g.tile[0], TY = g.tile[1], TZ = g.tile[2];
  const int tz = tile % g.ntile[2], ty = (tile / g.ntile[2]) % g.ntile[1], tx = tile / (g.ntile[2] * g.ntile[1]);
  const int Ny = g.dims[1], Nz = g.dims[2];
  const int TN = TX * TY * TZ;
  const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (int p = threadIdx.x >> 6; p < g.nwave * RG; p += nw) {
    const int chunk = p / RG, grp = p - chunk * RG;
    const int sidx = tile * g.nwave + chunk;
    const int off = g.ps_off[sidx], K = g.ps_k[sidx];
    if (skip_empty && K == 0) continue;
    const int uu = chunk * 64 + lane;
    const int r0 = rb0 + grp * RC, nr = min(RC, R - r0);
    if (uu >= TN || nr <= 0) continue;
    const int u = g.tn_perm[(size_t)tile * TN + uu];
    const int iz = u % TZ, iy = (u / TZ) % TY, ix = u / (TZ * TY);
    const int x = tx * TX + ix, y = ty * TY + iy, z = tz * TZ + iz;
    if (x >= g.dims[0] || y >= Ny || z >= Nz) continue;
    const int node = (x * Ny + y) * Nz + z;
    T acc[RC][6];
#pragma unroll
    for (int q = 0; q < RC; ++q)
#pragma unroll
      for (int c = 0; c < 6; ++c) acc[q][c] = 0;
    // the chunk's sliced list: entry k of this lane at 64 k + lane, in
    // groups of 4 so that several loads are in flight; pads add zero
    const int *ent = g.ps_ent + off + lane;
    const T *wl = (const T *)g.ps_w + 4 * ((size_t)off + lane);
    // entries are fetched one block of PB ahead (the copy at the end of a
    // trip is where the next block's loads are waited for)
    constexpr int PB = 8;
    auto fetch = [&](int k, int &loc, T (&w)[4]) {
      const int kk = min(k, K - 1);
      loc = ent[64 * (size_t)kk];
#pragma unroll
      for (int c = 0; c < 4; ++c) w[c] = wl[256 * (size_t)kk + c];
    };
    auto use = [&](int loc, const T (&w)[4]) {
      const T m0 = w[0], m1x = w[1], m1y = w[2], m1z = w[3];
      V2<T> jv[RC][4];
      if (loc >= 0) {
#pragma unroll
        for (int q = 0; q < RC; ++q)
#pragma unroll
          for (int c = 0; c < 4; ++c) jv[q][c] = sJ[loc * PS + (grp * RC + q) * 4 + c];
      } else {
        const V2<T> *jt = J + ((size_t)(-1 - loc) * R + r0) * 4;
#pragma unroll
        for (int q = 0; q < RC; ++q)
#pragma unroll
          for (int c = 0; c < 4; ++c) jv[q][c] = q < nr ? jt[4 * q + c] : cmk<T>(0, 0);
      }
      // two fused multiply-adds per output (J0 M1_c, then - J_c M0)
#pragma unroll
      for (int q = 0; q < RC; ++q) {
        const V2<T> j0 = jv[q][0], jx = jv[q][1], jy = jv[q][2], jz = jv[q][3];
        acc[q][0] = fma(-jx.x, m0, fma(j0.x, m1x, acc[q][0]));
        acc[q][1] = fma(-jx.y, m0, fma(j0.y, m1x, acc[q][1]));
        acc[q][2] = fma(-jy.x, m0, fma(j0.x, m1y, acc[q][2]));
        acc[q][3] = fma(-jy.y, m0, fma(j0.y, m1y, acc[q][3]));
        acc[q][4] = fma(-jz.x, m0, fma(j0.x, m1z, acc[q][4]));
        acc[q][5] = fma(-jz.y, m0, fma(j0.y, m1z, acc[q][5]));
      }
    };
    if (K > 0) {
      int lb[PB];
      T wb[PB][4];
#pragma unroll
      for (int u = 0; u < PB; ++u) fetch(u, lb[u], wb[u]);
      for (int kb = 0; kb < K; kb += PB) {
        int ln[PB];
        T wn[PB][4];
#pragma unroll
        for (int u = 0; u < PB; ++u) fetch(kb + PB + u, ln[u], wn[u]);
#pragma unroll
        for (int u = 0; u < PB; ++u)
          if (kb + u < K) use(lb[u], wb[u]);
#pragma unroll
        for (int u = 0; u < PB; ++u) {
          lb[u] = ln[u];
#pragma unroll
          for (int c = 0; c < 4; ++c) wb[u][c] = wn[u][c];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < RC; ++q) {
      if (q < nr) {
        V2<T> *Qr = Q + (size_t)(r0 + q) * 3 * g.N;
        Qr[node] = cmk<T>(acc[q][0], acc[q][1]);
        Qr[g.N + node] = cmk<T>(acc[q][2], acc[q][3]);
        Qr[2 * (size_t)g.N + node] = cmk<T>(acc[q][4], acc[q][5]);
      }
    }
  }
}

template <typename T>
static bool prune_ok(const GridMaps &g, long ch);

template <typename T, int RG>
static bool project_tiled(const GridMaps &g, const V2<T> *J, V2<T> *Q, int R, hipStream_t st) {
  constexpr int RC = ProjRC<T>::v;
  // largest staging any context asks for: 232 (FP32) or 376 (FP64) triangles
  constexpr int lds_max = (sizeof(T) == 4 ? 232 : 376) * proj_pitch<T, RG>() * (int)sizeof(V2<T>);
  static const bool lds_ok = allow_lds((const void *)k_project_tiled<T, RG>, lds_max);
  const size_t lds = (size_t)g.tcap * proj_pitch<T, RG>() * sizeof(V2<T>);
  if (!lds_ok || lds > (size_t)lds_max) return false;
  const unsigned ntile = (unsigned)g.ntile[0] * g.ntile[1] * g.ntile[2];
  k_project_tiled<T, RG><<<dim3(ntile * cdiv(R, RC * RG)), 512, lds, st>>>(g, J, Q, R, prune_ok<T>(g, 3L * R) ? 1 : 0);
  return true;
}

template <typename T>
void project(const GridMaps &g, const V2<T> *J, V2<T> *Q, int R, hipStream_t st) {
  if (g.proj_plan == 0) {
    // 16 (FP32, default) or 8 right-hand sides per workgroup: half the
    // staging per workgroup and twice the workgroups (at about 160 VGPRs one
    // 512-thread workgroup runs per CU either way)
    if (sizeof(T) == 4 && g.proj_rhs == 1 ? project_tiled<T, ProjRG<T>::v / 2 ? ProjRG<T>::v / 2 : 1>(g, J, Q, R, st)
                                          : project_tiled<T, ProjRG<T>::v>(g, J, Q, R, st))
      return;
  }
  k_project<T><<<dim3(cdiv(g.N, 256), cdiv(R, PRG)), 256, 0, st>>>(g, J, Q, R);
}

// ===========================================================================
// FFT along one axis of a [A][L][C] tensor: Stockham autosort passes of
// radix 8 (then 4 / 2), butterflies in registers, one LDS exchange per pass
// ===========================================================================
// A workgroup transforms LB consecutive lines (line = a * C + c), staged
// through LDS so global loads and stores are coalesced: for C == 1 the tile
// is one contiguous block, otherwise each row of the tile is LB consecutive
// elements.  Input holds n_in points per line (zero padding up to Lf), the
// output keeps the first n_out points.  fused: forward transform, multiply by
// the folded real spectrum, inverse transform (last-axis convolution).
struct FftArgs {
  int A, C, n_in, n_out, Lf, LB, ldl;   // ldl: LDS stride of one line (Lf + 1)
  int lb_sh, lf_sh;                     // log2 LB, log2 Lf
  int sign;         // -1 forward, +1 inverse
  float scale;      // applied on output
  int fused, two_nx, two_ny, nx, ny, nz;
};

// in-register DFT of size Rdx, forward (sign -1) or inverse (+1)
template <typename T, int Rdx>
__device__ __forceinline__ void dft(V2<T> *v, int sign) {
  if (Rdx == 2) {
    V2<T> a = v[0], b = v[1];
    v[0] = cadd<T>(a, b);
    v[1] = csub<T>(a, b);
  } else if (Rdx == 4) {
    V2<T> a0 = cadd<T>(v[0], v[2]), a1 = csub<T>(v[0], v[2]);
    V2<T> b0 = cadd<T>(v[1], v[3]), b1 = csub<T>(v[1], v[3]);
    // multiply b1 by -i (forward) or +i (inverse)
    V2<T> b1r = sign < 0 ? cmk<T>(b1.y, -b1.x) : cmk<T>(-b1.y, b1.x);
    v[0] = cadd<T>(a0, b0);
    v[2] = csub<T>(a0, b0);
    v[1] = cadd<T>(a1, b1r);
    v[3] = csub<T>(a1, b1r);
  } else {  // 8 = 2 x 4: even/odd halves, then twiddles W8^k
    V2<T> e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft<T, 4>(e, sign);
    dft<T, 4>(o, sign);
    const T h = (T)0.70710678118654752440;
    // W8^1 = (h, -h) forward, (h, h) inverse; W8^2 = -i / +i; W8^3 = (-h, -h) / (-h, h)
    V2<T> o1 = sign < 0 ? cmk<T>(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x))
                        : cmk<T>(h * (o[1].x - o[1].y), h * (o[1].y + o[1].x));
    V2<T> o2 = sign < 0 ? cmk<T>(o[2].y, -o[2].x) : cmk<T>(-o[2].y, o[2].x);
    V2<T> o3 = sign < 0 ? cmk<T>(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y))
                        : cmk<T>(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y));
    v[0] = cadd<T>(e[0], o[0]);
    v[4] = csub<T>(e[0], o[0]);
    v[1] = cadd<T>(e[1], o1);
    v[5] = csub<T>(e[1], o1);
    v[2] = cadd<T>(e[2], o2);
    v[6] = csub<T>(e[2], o2);
    v[3] = cadd<T>(e[3], o3);
    v[7] = csub<T>(e[3], o3);
  }
}

// One Stockham pass of radix Rdx over 2^lb_sh lines of length 2^lf_sh held
// in LDS, element (line, k) at sm[line * ls + k * es] (in place: every thread
// reads its butterflies into registers before anyone writes).  The
// butterfly loop is unrolled so the register arrays are never indexed at run
// time; at most 8192 points per call (32 per thread).
template <typename T, int Rdx>
__device__ __forceinline__ void stockham_pass(V2<T> *sm, const V2<T> *tw, int lb_sh, int ls, int es, int lf_sh,
                                              int Ns, int sign) {
  constexpr int MAXB = 32 / Rdx;
  const int Lf = 1 << lf_sh;
  const int nb = Lf / Rdx;                       // butterflies per line
  const int total = nb << lb_sh;
  const int LBm = (1 << lb_sh) - 1;
  const int tstep = Lf / (Ns * Rdx);
  V2<T> v[MAXB][Rdx];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    int idx = threadIdx.x + q * 256;
    if (idx < total) {
      int line = idx & LBm, j = idx >> lb_sh;
      const V2<T> *x = sm + line * ls;
      int k = j & (Ns - 1);
#pragma unroll
      for (int i = 0; i < Rdx; ++i) {
        V2<T> a = x[(j + i * nb) * es];
        if (i > 0 && Ns > 1) {
          V2<T> w = tw[(i * k * tstep) & (Lf - 1)];
          if (sign > 0) w.y = -w.y;
          a = cmul<T>(a, w);
        }
        v[q][i] = a;
      }
      dft<T, Rdx>(v[q], sign);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    int idx = threadIdx.x + q * 256;
    if (idx < total) {
      int line = idx & LBm, j = idx >> lb_sh;
      V2<T> *y = sm + line * ls;
      int k = j & (Ns - 1);
      int base = (j - k) * Rdx + k;
#pragma unroll
      for (int i = 0; i < Rdx; ++i) y[(base + i * Ns) * es] = v[q][i];
    }
  }
  __syncthreads();
}

// Full Stockham transform (radix 8 passes, then one 4 or 2); tw holds the
// 2^lf_sh twiddles of this length.
template <typename T>
__device__ __forceinline__ void stockham(V2<T> *sm, const V2<T> *tw, int lb_sh, int ls, int es, int lf_sh,
                                         int sign) {
  const int Lf = 1 << lf_sh;
  int Ns = 1;
  while (Ns * 8 <= Lf) {
    stockham_pass<T, 8>(sm, tw, lb_sh, ls, es, lf_sh, Ns, sign);
    Ns *= 8;
  }
  if (Ns * 4 <= Lf) {
    stockham_pass<T, 4>(sm, tw, lb_sh, ls, es, lf_sh, Ns, sign);
    Ns *= 4;
  }
  if (Ns * 2 <= Lf) {
    stockham_pass<T, 2>(sm, tw, lb_sh, ls, es, lf_sh, Ns, sign);
    Ns *= 2;
  }
}

template <typename T>
__device__ __forceinline__ void fill_twiddles(V2<T> *tw, int Lf) {
  for (int k = threadIdx.x; k < Lf; k += blockDim.x) {
    if (sizeof(T) == 4) {
      float sf, cf;
      sincospif(2.0f * (float)k / (float)Lf, &sf, &cf);
      tw[k] = cmk<T>((T)cf, (T)-sf);
    } else {
      double sd, cd;
      sincospi(2.0 * (double)k / (double)Lf, &sd, &cd);
      tw[k] = cmk<T>((T)cd, (T)-sd);
    }
  }
}

// Fused middle of the convolution for one (channel, kx) plane held in LDS:
// forward FFT along y (only the Nz non-zero columns), forward FFT along z,
// multiply by the real spectrum, inverse along z, inverse along y (only the
// Nz columns that are kept), crop to Ny x Nz.  In place on a [.][Ny][Nz]
// plane: reads and writes 2 Ny Nz points per channel instead of 10.
struct YZArgs {
  int ny, nz, ly_sh, lz_sh, pitch, nx, two_nx;
  float scale;
};

template <typename T>
__global__ void __launch_bounds__(256) k_fft_yz(YZArgs a, V2<T> *data, const T *ghat) {
  extern __shared__ unsigned char smraw[];
  const int Ly = 1 << a.ly_sh, Lz = 1 << a.lz_sh, P = a.pitch;
  V2<T> *twy = (V2<T> *)smraw;
  V2<T> *twz = twy + Ly;
  V2<T> *sm = twz + Lz;                     // Ly rows x pitch
  const long plane = blockIdx.x;            // (channel, kx)
  const int kx = (int)(plane & (a.two_nx - 1));
  V2<T> *io = data + plane * (long)a.ny * a.nz;
  fill_twiddles<T>(twy, Ly);
  fill_twiddles<T>(twz, Lz);
  for (int idx = threadIdx.x; idx < Ly * P; idx += blockDim.x) sm[idx] = cmk<T>(0, 0);
  __syncthreads();
  for (int idx = threadIdx.x; idx < a.ny * a.nz; idx += blockDim.x) {
    int y = idx / a.nz, z = idx - y * a.nz;
    sm[y * P + z] = io[idx];
  }
  __syncthreads();
  const int nz_sh = a.lz_sh - 1;
  // Y forward on the Nz non-zero columns: lines = columns (stride 1), elements stride P
  stockham<T>(sm, twy, nz_sh, 1, P, a.ly_sh, -1);
  // Z forward on all Ly rows
  stockham<T>(sm, twz, a.ly_sh, P, 1, a.lz_sh, -1);
  const int fx = kx <= a.nx ? kx : a.two_nx - kx;
  const int ny1 = Ly / 2 + 1, nz1 = Lz / 2 + 1;
  const T *gx = ghat + (long)fx * ny1 * nz1;
  for (int idx = threadIdx.x; idx < Ly * Lz; idx += blockDim.x) {
    int ky = idx >> a.lz_sh, kz = idx & (Lz - 1);
    int fy = ky < ny1 ? ky : Ly - ky;
    int fz = kz < nz1 ? kz : Lz - kz;
    sm[ky * P + kz] = cscale<T>(sm[ky * P + kz], gx[fy * nz1 + fz]);
  }
  __syncthreads();
  stockham<T>(sm, twz, a.ly_sh, P, 1, a.lz_sh, +1);
  stockham<T>(sm, twy, nz_sh, 1, P, a.ly_sh, +1);
  const T sc = (T)a.scale;
  for (int idx = threadIdx.x; idx < a.ny * a.nz; idx += blockDim.x) {
    int y = idx / a.nz, z = idx - y * a.nz;
    io[idx] = cscale<T>(sm[y * P + z], sc);
  }
}

// ---------------------------------------------------------------------------
// Register-resident variant of the fused plane kernel (FP32).  A zero-padded
// length-2N transform of N inputs splits into two N-point transforms: the
// even outputs are FFT_N(x), the odd ones FFT_N(x_n W_2N^n); a cropped
// length-2N inverse is the sum of the two N-point inverses, the odd one
// multiplied by conj(W_2N^n).  Each thread owns one N-point line in
// registers (decimation in frequency forward, in time inverse, so no
// reordering), the two halves of a line live in a lane pair and are summed
// with a lane exchange, and the plane crosses LDS twice (rows -> columns ->
// rows).  Twiddles are compile-time constants.
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846;
constexpr double taylor_sin(double x) {
  double t = x, s = x;
  for (int i = 1; i < 12; ++i) {
    t *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
    s += t;
  }
  return s;
}
constexpr double taylor_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int i = 1; i < 12; ++i) {
    t *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
    s += t;
  }
  return s;
}
// W_n^k = exp(-2 pi i k / n) by quadrant reduction to [0, pi/2]
struct TwTable {
  static constexpr int N = 1024;
  float c[N], s[N];
  constexpr TwTable() : c(), s() {
    for (int k = 0; k < N; ++k) {
      const int q = (4 * k) / N, r = 4 * k - q * N;
      const double a = kPi / 2 * r / N, ca = taylor_cos(a), sa = taylor_sin(a);
      const double cc = q == 0 ? ca : q == 1 ? -sa : q == 2 ? -ca : sa;
      const double ss = q == 0 ? sa : q == 1 ? ca : q == 2 ? -sa : -ca;
      c[k] = (float)cc;
      s[k] = (float)-ss;
    }
  }
};
constexpr TwTable kTw{};

// W_n^k (SIGN -1) or its conjugate (SIGN +1); n divides 1024
template <int SIGN>
__device__ __forceinline__ float2 tw(int k, int n) {
  // n is a power of two up to TwTable::N (all call sites use compile-time n)
  const int i = (k * (TwTable::N / n)) & (TwTable::N - 1);
  return make_float2(kTw.c[i], SIGN < 0 ? kTw.s[i] : -kTw.s[i]);
}

// x W_n^k (SIGN -1) or x conj(W_n^k) (SIGN +1).  k and n are constants after
// unrolling; quarter turns become exact swaps and negations (no multiply).
template <int SIGN>
__device__ __forceinline__ float2 twmul(float2 x, int k, int n) {
  if ((4 * k) % n == 0) {
    const int e = ((4 * k) / n) & 3;
    const int r = SIGN < 0 ? e : (4 - e) & 3;   // rotation by (-i)^r
    if (r == 0) return x;
    if (r == 1) return make_float2(x.y, -x.x);
    if (r == 2) return make_float2(-x.x, -x.y);
    return make_float2(-x.y, x.x);
  }
  const float2 w = tw<SIGN>(k, n);
  return make_float2(x.x * w.x - x.y * w.y, x.x * w.y + x.y * w.x);
}

constexpr int clog2(int n) { return n <= 1 ? 0 : 1 + clog2(n / 2); }
constexpr int brev(int k, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((k >> i) & 1) << (bits - 1 - i);
  return r;
}

// Radix-2^2 in-register FFTs: two radix-2 stages at a time, arranged as a
// radix-4 butterfly so that only three of every four points of a stage pair
// take a general twiddle (the others take a quarter turn, which twmul makes
// exact); the data order is that of the radix-2 algorithms.
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// decimation in frequency: natural order in, bit-reversed order out.  Stage
// pair on blocks of B = N >> S points, quarters q = B / 4: with s = a + b,
// d = a - b for the pairs (j, j + B/2), the four outputs of j < q are
// (s_j + s_{j+q}), (s_j - s_{j+q}) W_B^{2j}, (d_j + r d_{j+q}) W_B^j and
// (d_j - r d_{j+q}) W_B^{3j}, r the quarter turn W_4 of the transform's sign.
template <int N, int SIGN, int S = 0>
__device__ __forceinline__ void fft_dif(float2 (&v)[N]) {
  constexpr int B = N >> S;
  if constexpr (B >= 4) {
    constexpr int h = B / 2, q = B / 4;
#pragma unroll
    for (int blk = 0; blk < N / B; ++blk)
#pragma unroll
      for (int j = 0; j < q; ++j) {
        const int i0 = blk * B + j, i1 = i0 + q, i2 = i0 + h, i3 = i2 + q;
        const float2 s0 = cadd(v[i0], v[i2]), d0 = csub(v[i0], v[i2]);
        const float2 s1 = cadd(v[i1], v[i3]), d1 = twmul<SIGN>(csub(v[i1], v[i3]), 1, 4);
        v[i0] = cadd(s0, s1);
        v[i1] = twmul<SIGN>(csub(s0, s1), 2 * j, B);
        v[i2] = twmul<SIGN>(cadd(d0, d1), j, B);
        v[i3] = twmul<SIGN>(csub(d0, d1), 3 * j, B);
      }
    fft_dif<N, SIGN, S + 2>(v);
  } else if constexpr (B == 2) {
#pragma unroll
    for (int i = 0; i < N; i += 2) {
      const float2 a = v[i], c = v[i + 1];
      v[i] = cadd(a, c);
      v[i + 1] = csub(a, c);
    }
  }
}

// decimation in time: bit-reversed order in, natural order out.  Stage pair
// with halves h and 2h on blocks of B = 4 h: the inputs at j, j + h, j + 2h,
// j + 3h (j < h) take W_B^0, W_B^{2j}, W_B^j, W_B^{3j} and then a radix-4
// butterfly; a leftover last stage is radix 2.
template <int N, int SIGN, int S = 0>
__device__ __forceinline__ void fft_dit(float2 (&v)[N]) {
  constexpr int h = 1 << S, B = 4 * h;
  if constexpr (B <= N) {
#pragma unroll
    for (int blk = 0; blk < N / B; ++blk)
#pragma unroll
      for (int j = 0; j < h; ++j) {
        const int p0 = blk * B + j, p1 = p0 + h, p2 = p0 + 2 * h, p3 = p0 + 3 * h;
        const float2 a = v[p0], b = twmul<SIGN>(v[p1], 2 * j, B);
        const float2 c = twmul<SIGN>(v[p2], j, B), d = twmul<SIGN>(v[p3], 3 * j, B);
        const float2 x0 = cadd(a, b), x1 = csub(a, b), y2 = cadd(c, d);
        const float2 y3 = twmul<SIGN>(csub(c, d), 1, 4);
        v[p0] = cadd(x0, y2);
        v[p2] = csub(x0, y2);
        v[p1] = cadd(x1, y3);
        v[p3] = csub(x1, y3);
      }
    fft_dit<N, SIGN, S + 2>(v);
  } else if constexpr (2 * h == N) {
#pragma unroll
    for (int j = 0; j < h; ++j) {
      const float2 a = v[j], c = twmul<SIGN>(v[j + h], j, 2 * h);
      v[j] = cadd(a, c);
      v[j + h] = csub(a, c);
    }
  }
}

// Lane-quad exchange (DPP quad_perm): lane q of each quad of 4 receives the
// value of lane q ^ 1, q ^ 2 or q ^ 3.
template <int CTRL>
__device__ __forceinline__ float qperm(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ float2 qperm2(float2 v) {
  return make_float2(qperm<CTRL>(v.x), qperm<CTRL>(v.y));
}
// value of lane ^ 4: the half-row mirror (lane ^ 7 within each group of 8)
// followed by the quad reversal (lane ^ 3), both DPP moves in registers
__device__ __forceinline__ float xor4(float v) { return qperm<0x1B>(qperm<0x141>(v)); }
__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One-hot weights of a quad lane q for lane-dependent twiddles W^{q k} with
// compile-time k (arithmetic, no branches).
struct QuadLane {
  float f[4];
};
template <int SIGN>
__device__ __forceinline__ QuadLane quad_lane(int q) {
  QuadLane L;
#pragma unroll
  for (int j = 0; j < 4; ++j) L.f[j] = q == j ? 1.f : 0.f;
  return L;
}
// W_n^{q k} for the lane's q (one-hot blend of compile-time constants)
template <int SIGN>
__device__ __forceinline__ float2 tw_q(const QuadLane &L, int k, int n) {
  const float2 w1 = tw<SIGN>(k, n), w2 = tw<SIGN>(2 * k, n), w3 = tw<SIGN>(3 * k, n);
  return make_float2(L.f[0] + L.f[1] * w1.x + L.f[2] * w2.x + L.f[3] * w3.x,
                     L.f[1] * w1.y + L.f[2] * w2.y + L.f[3] * w3.y);
}
// exact branch-free select: a where mask is all ones, b where it is zero
__device__ __forceinline__ float selb(int mask, float a, float b) {
  return __int_as_float((__float_as_int(a) & mask) | (__float_as_int(b) & ~mask));
}
__device__ __forceinline__ float2 selb2(int mask, float2 a, float2 b) {
  return make_float2(selb(mask, a.x, b.x), selb(mask, a.y, b.y));
}
// w on the odd half (hmask all ones), 1 on the even half
__device__ __forceinline__ float2 half_tw(int hmask, float2 w) {
  return selb2(hmask, w, make_float2(1.f, 0.f));
}

// X passes of the convolution (FP32), lines of NX = 4 M points along x with
// stride C between points; a zero-padded length-2 NX transform splits into
// even/odd halves h, each an NX-point transform done as a radix-4 step
// across a lane quad (lane q) and M-point register FFTs.  Lanes: 8 columns
// per wave, lane = 8 col + 4 h + q.
//   forward: in [ch][NX][C] -> out [ch][2NX][C]
//   inverse: in [ch][2NX][C] -> out [ch][NX][C] (crop, times 1 / (2 NX))
typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(__amdgpu_buffer_rsrc_t(), 0, 0, 0)) b64_t;

// Buffer access with a per-lane byte offset (VGPR) and a uniform one (SGPR):
// no per-element 64-bit addresses, and the hardware drops accesses beyond
// the buffer's size.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float2 buf_load2(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_store2(float2 v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(b64_t, v), r, voff, soff, 0);
}

// Pruned passes: workgroups whose 32 columns hold no active node exit, the
// forward pass reads only active nodes (zero elsewhere), the inverse pass
// writes only active nodes.  Skipped accesses take a per-lane byte offset of
// 2^31, beyond the buffer of every launch (launch_x_reg keeps those below
// 2^31 bytes, and with them every uniform offset), so the hardware's range
// check turns the load into zero and drops the store.
constexpr unsigned X_DROP = 0x80000000u;

// Forward X pass, decimation in frequency across the quad.  With x = m + M q
// and k = 4 k1 + k2, the NX-point DFT of half h (input times W_{2NX}^{h x})
// is: a radix-4 DFT over q for each m (after the lane constant W_8^{h q}),
// the twiddle W_{2NX}^{(2 k2 + h) m}, then an M-point DFT over m in
// registers; output row kx = 2 k + h = 8 k1 + 2 k2 + h.  The radix-4 step is
// two radix-2 steps across lanes (DPP, partners q ^ 2 then q ^ 1), whose
// lane signs and the -i of the second step are folded into the per-lane
// factors and into the twiddle table xtw[lane & 7][m] (which holds the sign
// of the second step times W_{2NX}^{(2 k2 + h) m}).  The block's 32 columns
// of each 64 output rows are staged in LDS, so every store writes whole
// 256-byte rows (two per wavefront instruction).  Pruned (PR): as
// described above.
template <int NX, bool PR>
__global__ void __launch_bounds__(256, 3) k_fft_x_fwd(const float2 *in, float2 *out, int C, int ncol,
                                                   const float2 *xtw, const uint32_t *xmask, const uint8_t *cgrp) {
  constexpr int M = NX / 4, LM = clog2(M), WPC = NX / 32;
  constexpr int TP = M + 1;     // twiddle table pitch: the 8 rows fall in different banks
  constexpr int LP = 36;        // staging pitch (4 mod 32 slots of 8 bytes: conflict-free)
  constexpr int NCH = 2 * NX / 64;
  __shared__ float2 s_tw[8 * TP];
  __shared__ float2 s_out[2][64 * LP];
  const unsigned c0 = (unsigned)(blockIdx.x * 32) % (unsigned)C;   // block's first column in its channel
  if (PR && !cgrp[c0 / 32u]) return;
  const int t = threadIdx.x, lane = t & 63, q = lane & 3, h = (lane >> 2) & 1, r = lane & 7;
  const int cl = (t >> 6) * 8 + (lane >> 3);
  const int col = blockIdx.x * 32 + cl;
  const int chn = col / C, c = col - chn * C;
  for (int i = t; i < 8 * M; i += 256) s_tw[(i / M) * TP + i % M] = xtw[i];
  __syncthreads();
  const unsigned nin = (unsigned)ncol * NX * 8u, nout = (unsigned)ncol * 2 * NX * 8u;
  const __amdgpu_buffer_rsrc_t rin = buf_rsrc(in, nin), rout = buf_rsrc(out, nout);
  const unsigned C8 = (unsigned)C * 8u;
  float2 v[M];
  {
    // rows x = m + M q
    const unsigned vo = ((unsigned)chn * NX * C + c + (unsigned)(q * M) * C) * 8u;
    if (PR) {
      constexpr int NW = M >= 32 ? M / 32 : 1;
      uint32_t mw[NW];
#pragma unroll
      for (int j = 0; j < NW; ++j) mw[j] = xmask[(size_t)c * WPC + (q * M) / 32 + j];
      const int b0 = (q * M) % 32;   // 0 when M >= 32
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const uint32_t bit = M >= 32 ? (mw[m / 32] >> (m % 32)) & 1u : (mw[0] >> (b0 + m)) & 1u;
        v[m] = buf_load2(rin, bit ? vo : X_DROP, (unsigned)m * C8);
      }
    } else {
#pragma unroll
      for (int m = 0; m < M; ++m) v[m] = buf_load2(rin, vo, (unsigned)m * C8);
    }
  }
  // lane constants
  const QuadLane L = quad_lane<-1>(q);
  const float2 cq = half_tw(-h, tw_q<-1>(L, M, 2 * NX));   // W_8^{h q}
  const float sA = q < 2 ? 1.f : -1.f, sB = (q & 1) ? -1.f : 1.f, sk = q == 2 ? -1.f : 1.f;
  const bool q3 = q == 3;
  const float2 *tr = s_tw + r * TP;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const float2 w = cmulf(v[m], cq);
    const float2 pw = qperm2<0x4E>(w);                       // lane q ^ 2
    const float2 a = make_float2(fmaf(sA, pw.x, w.x), fmaf(sA, pw.y, w.y));
    const float2 p = make_float2(q3 ? -a.y : sk * a.x, q3 ? a.x : sk * a.y);
    const float2 pp = qperm2<0xB1>(p);                       // lane q ^ 1
    const float2 x = make_float2(fmaf(sB, pp.x, p.x), fmaf(sB, pp.y, p.y));
    v[m] = cmulf(x, tr[m]);
  }
  fft_dif<M, -1>(v);                       // position p holds k1 = brev(p)
  // 64 output rows at a time: rows 64 ch + 8 i + 2 k2 + h hold k1 = 8 ch + i
  const int k2 = (q >> 1) | ((q & 1) << 1);
  const int lrow = 2 * k2 + h;
  const unsigned ob = ((unsigned)chn * 2 * NX * C + c0) * 8u;
#pragma unroll
  for (int ck = 0; ck < NCH; ++ck) {
    float2 *so = s_out[ck & 1];
#pragma unroll
    for (int i = 0; i < 8; ++i) so[(8 * i + lrow) * LP + cl] = v[brev(8 * ck + i, LM)];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int rr = (t >> 5) + 8 * i, cc = t & 31;
      buf_store2(so[rr * LP + cc], rout, ob + ((unsigned)(64 * ck + rr) * C + cc) * 8u, 0);
    }
  }
}

// Inverse X pass in the same form: with k = m + M q and x = 4 k1 + k2 the
// inverse NX-point DFT of half h (rows kx = 2 k + h) is a radix-4 inverse DFT
// over q for each m, the twiddle W_{NX}^{-k2 m}, an M-point inverse DFT over
// m in registers, then the factor W_{2NX}^{-h x} before the two halves are
// summed (lanes 4 apart).  As in the forward pass the lane signs of the two
// DPP steps (+i in place of -i), the lane constant W_{2NX}^{-h k2} and the
// scale are folded into the table itw[lane & 7][m]; the k1-dependent factor
// W_{2M}^{-h k1} is applied per element.  Pruned (PR): as described above.
template <int NX, bool PR>
__global__ void __launch_bounds__(256) k_fft_x_inv(const float2 *in, float2 *out, int C, int ncol,
                                                   const float2 *itw, const uint32_t *xmask, const uint8_t *cgrp) {
  constexpr int M = NX / 4, LM = clog2(M), WPC = NX / 32;
  constexpr int TP = M + 1;
  __shared__ float2 s_tw[8 * TP];
  __shared__ float2 s_in[NX * 33];   // one half of the workgroup's input rows
  const unsigned c0 = (unsigned)(blockIdx.x * 32) % (unsigned)C;
  if (PR && !cgrp[c0 / 32u]) return;
  const int t = threadIdx.x, lane = t & 63, q = lane & 3, h = (lane >> 2) & 1, r = lane & 7;
  const int hm = -h;
  const int col = blockIdx.x * 32 + (t >> 6) * 8 + (lane >> 3);
  const int chn = col / C, c = col - chn * C;
  for (int i = t; i < 8 * M; i += 256) s_tw[(i / M) * TP + i % M] = itw[i];
  __syncthreads();
  const unsigned nin = (unsigned)ncol * 2 * NX * 8u, nout = (unsigned)ncol * NX * 8u;
  const __amdgpu_buffer_rsrc_t rin = buf_rsrc(in, nin), rout = buf_rsrc(out, nout);
  const unsigned C8 = (unsigned)C * 8u;
  float2 v[M];
  {
    // rows kx = 2 (m + M q) + h, read as whole 256-byte segments of the
    // workgroup's 32 columns and handed over through LDS, in two halves of
    // m: half ph holds row 2 M q + ph M + j (j < M) at local row q M + j,
    // column (cl + 8 q) mod 32 (the skew puts the four q of a lane's column
    // in different banks)
    const int cl = (t >> 6) * 8 + (lane >> 3);   // this lane's column in the workgroup
    const unsigned base = ((unsigned)chn * 2 * NX * C + c0) * 8u;
    constexpr int NL = NX / 8;                  // staged elements per thread and half
    float2 g[NL];
    auto fetch = [&](int ph) {
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        const int rl = (t >> 5) + 8 * i, qq = rl / M, j = rl - qq * M;
        g[i] = buf_load2(rin, base + (unsigned)((2 * M * qq + ph * M + j) * C + (t & 31)) * 8u, 0);
      }
    };
    auto put = [&]() {
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        const int rl = (t >> 5) + 8 * i, qq = rl / M;
        s_in[rl * 33 + (((t & 31) + 8 * qq) & 31)] = g[i];
      }
    };
    auto take = [&](int ph) {
#pragma unroll
      for (int mm = 0; mm < M / 2; ++mm)
        v[ph * (M / 2) + mm] = s_in[(q * M + 2 * mm + h) * 33 + ((cl + 8 * q) & 31)];
    };
    fetch(0);
    put();
    __syncthreads();
    fetch(1);   // in flight while the first half is read
    take(0);
    __syncthreads();
    put();
    __syncthreads();
    take(1);
  }
  const float sA = q < 2 ? 1.f : -1.f, sB = (q & 1) ? -1.f : 1.f, sk = q == 2 ? -1.f : 1.f;
  const bool q3 = q == 3;
  const float2 *tr = s_tw + r * TP;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const float2 w = v[m];
    const float2 pw = qperm2<0x4E>(w);                       // lane q ^ 2
    const float2 a = make_float2(fmaf(sA, pw.x, w.x), fmaf(sA, pw.y, w.y));
    // lane 3 takes +i (the inverse's W_4^{-1}) where the forward pass takes -i
    const float2 p = make_float2(q3 ? a.y : sk * a.x, q3 ? -a.x : sk * a.y);
    const float2 pp = qperm2<0xB1>(p);                       // lane q ^ 1
    const float2 x = make_float2(fmaf(sB, pp.x, p.x), fmaf(sB, pp.y, p.y));
    v[m] = cmulf(x, tr[m]);
  }
  fft_dif<M, +1>(v);                       // position p holds k1 = brev(p)
  // W_{2M}^{-h k1}, then the halves: lane h keeps positions [h M/2, (h+1) M/2)
#pragma unroll
  for (int p = 0; p < M; ++p) v[p] = cmulf(v[p], half_tw(hm, tw<+1>(brev(p, LM), 2 * M)));
  const int k2 = (q >> 1) | ((q & 1) << 1);
  uint32_t mw[PR ? WPC : 1];
  if (PR) {
#pragma unroll
    for (int w = 0; w < WPC; ++w) mw[w] = xmask[(size_t)c * WPC + w];
  }
  const unsigned ob = ((unsigned)chn * NX * C + c + (unsigned)k2 * C) * 8u;
#pragma unroll
  for (int j = 0; j < M / 2; ++j) {
    const float2 lo = v[j], hi = v[j + M / 2];
    const float2 send = selb2(hm, lo, hi), keep = selb2(hm, hi, lo);
    const float2 rv = make_float2(xor4(send.x), xor4(send.y));   // lane ^ 4
    const float2 o = make_float2(keep.x + rv.x, keep.y + rv.y);
    // row x = 4 k1 + k2, k1 = brev(p), p = j + h M / 2
    const int k1a = brev(j, LM), k1b = brev(j + M / 2, LM);
    unsigned om = ob + (unsigned)(h ? 4 * k1b : 4 * k1a) * C8;
    if (PR) {
      const int xa = 4 * k1a, xb = 4 * k1b;   // + k2 (< 4, same word)
      const uint32_t wv = h ? mw[xb / 32] : mw[xa / 32];
      const int sh = (h ? xb % 32 : xa % 32) + k2;
      om = ((wv >> sh) & 1u) ? om : X_DROP;
    }
    buf_store2(o, rout, om, 0);
  }
}

// One (channel, kx) plane per workgroup of 2 NY threads (NY = 2 NZ).  Block
// b works on channel ch - 1 - b / 2Nx, kx = b % 2Nx: the X passes run over the
// channels in ascending order, so this pass first reads the planes the
// forward X pass wrote last and ends with the ones the inverse X pass reads
// first, both while they are still in the memory-side cache.  The whole
// spectrum fits in every L2.
// Pruned (PR): column (y, z) enters as zero unless bit y of zmask[z] is set
// (it holds no active node, and whatever the buffer holds there is not the
// forward X pass's output); every column is still written.
template <int NY, int NZ, bool PR>
__global__ void __launch_bounds__(2 * NY) k_fft_yz_reg(YZArgs a, float2 *data, const float *ghat, long ch,
                                                       const uint64_t *zmask) {
  static_assert(NY == 2 * NZ, "one thread per (row, half) and per (column, half)");
  constexpr int PT = NY + 1;                 // T[kz][y] pitch
  constexpr int P0 = NZ + 1;                 // staging [y][z] pitch
  constexpr int LZ = 2 * NZ, LY = 2 * NY;
  __shared__ float2 sm[LZ * PT];
  // stages A and C: thread t works on line (row or column) t % NY, half
  // t / NY; with NY = 64 the half is the wave index, so a half's twiddles are
  // a scalar branch
  const int t = threadIdx.x;
  const int wl = t % NY;
  const int wh = NY % 64 == 0 ? __builtin_amdgcn_readfirstlane(t / NY) : t / NY;
  const long cb = blockIdx.x / a.two_nx, kx = blockIdx.x - cb * a.two_nx, chan = ch - 1 - cb;
  float2 *io = data + (chan * a.two_nx + kx) * (long)(NY * NZ);
  // stage 0: coalesced load of the NY x NZ plane (2 NY is a multiple of NZ,
  // so a thread's z is the same for every q).  Pruned: an inactive column's
  // load takes an offset beyond the plane's buffer and reads zero (no
  // branch, so all loads are in flight together).
  const uint64_t zm = PR ? zmask[t % NZ] : 0;
  const __amdgpu_buffer_rsrc_t rio = buf_rsrc(io, (unsigned)(NY * NZ * 8));
#pragma unroll
  for (int q = 0; q < NZ / 2; ++q) {
    const int idx = t + q * 2 * NY, y = idx / NZ, z = idx - y * NZ;
    if (PR) {
      const unsigned off = ((zm >> y) & 1u) ? (unsigned)idx * 8u : X_DROP;
      sm[y * P0 + z] = buf_load2(rio, off, 0);
    } else {
      sm[y * P0 + z] = io[idx];
    }
  }
  __syncthreads();
  // stage A: forward z half wh of row wl
  {
    float2 v[NZ];
#pragma unroll
    for (int z = 0; z < NZ; ++z) v[z] = sm[wl * P0 + z];
    if (wh) {
#pragma unroll
      for (int z = 0; z < NZ; ++z) v[z] = twmul<-1>(v[z], z, LZ);
    }
    fft_dif<NZ, -1>(v);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NZ; ++k) sm[(2 * k + wh) * PT + wl] = v[brev(k, clog2(NZ))];
  }
  __syncthreads();
  // stage C: column kz = wl, y half wh: forward, spectrum, inverse
  {
    const int kz = wl, half = wh;
    float2 v[NY];
#pragma unroll
    for (int y = 0; y < NY; ++y) v[y] = sm[kz * PT + y];
    if (half) {
#pragma unroll
      for (int y = 0; y < NY; ++y) v[y] = twmul<-1>(v[y], y, LY);
    }
    fft_dif<NY, -1>(v);
    const int fx = kx <= a.nx ? (int)kx : a.two_nx - (int)kx;
    const int fz = kz <= NZ ? kz : LZ - kz;
    // Ghat(fx, fy, fz) with fy the folded ky = k0 + half, k0 = 2 brev(p):
    // fy = k0 + half for k0 < NY, (LY - k0 - 1) + (1 - half) otherwise.  The
    // lane's part of the offset is one of two registers, the rest is uniform
    // (scalar offset), so no vector address arithmetic per element.
    constexpr unsigned K4 = (NZ + 1) * 4u;
    const __amdgpu_buffer_rsrc_t rg =
        buf_rsrc(ghat + (long)fx * (NY + 1) * (NZ + 1), (unsigned)((NY + 1) * (NZ + 1) * 4));
    const unsigned va = (unsigned)fz * 4u + (unsigned)half * K4, vb = (unsigned)fz * 4u + (unsigned)(1 - half) * K4;
#pragma unroll
    for (int p = 0; p < NY; ++p) {
      const int k0 = 2 * brev(p, clog2(NY));
      const float g = k0 < NY ? __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rg, va, k0 * K4, 0))
                              : __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rg, vb, (LY - k0 - 1) * K4, 0));
      v[p] = make_float2(v[p].x * g, v[p].y * g);
    }
    fft_dit<NY, +1>(v);
    if (half) {
#pragma unroll
      for (int n = 0; n < NY; ++n) v[n] = twmul<+1>(v[n], n, LY);
    }
    // sum of the two halves through column kz: half h finishes n in
    // [h NY/2, (h+1) NY/2) and hands the other range to its partner
    __syncthreads();   // both halves have read the column
    float2 *col = sm + kz * PT;
    if (half) {
#pragma unroll
      for (int j = 0; j < NY / 2; ++j) col[j] = v[j];
    } else {
#pragma unroll
      for (int j = 0; j < NY / 2; ++j) col[NY / 2 + j] = v[NY / 2 + j];
    }
    __syncthreads();
    if (half) {
#pragma unroll
      for (int j = 0; j < NY / 2; ++j) {
        const float2 r = col[NY / 2 + j];
        col[NY / 2 + j] = make_float2(v[NY / 2 + j].x + r.x, v[NY / 2 + j].y + r.y);
      }
    } else {
#pragma unroll
      for (int j = 0; j < NY / 2; ++j) {
        const float2 r = col[j];
        col[j] = make_float2(v[j].x + r.x, v[j].y + r.y);
      }
    }
  }
  __syncthreads();
  // stage D: row n = line, z half `half` (lane pairs, t = 2 line + half):
  // inverse, crop, lane-pair sum, store
  {
    const int half = t & 1, line = t >> 1;
    float2 v[NZ];
#pragma unroll
    for (int k = 0; k < NZ; ++k) v[k] = sm[(2 * k + half) * PT + line];
    fft_dif<NZ, +1>(v);                     // position p holds z = brev(p)
    if (half) {
#pragma unroll
      for (int p = 0; p < NZ; ++p) v[p] = twmul<+1>(v[p], brev(p, clog2(NZ)), LZ);
    }
    const float sc = a.scale;
    float2 *row = io + (long)line * NZ + half * (NZ / 2);
#pragma unroll
    for (int j = 0; j < NZ / 2; ++j) {
      const float2 lo = v[brev(j, clog2(NZ))], hi = v[brev(j + NZ / 2, clog2(NZ))];
      const float2 send = half ? lo : hi, keep = half ? hi : lo;
      const float2 r = qperm2<0xB1>(send);   // lane ^ 1
      row[j] = make_float2((keep.x + r.x) * sc, (keep.y + r.y) * sc);
    }
  }
}

// Fused plane kernel for (channel, k_x) planes too large for one LDS tile:
// N_y N_z = 8192 (256 x 32 or 512 x 16).  The zero-padded 2N_y x 2N_z plane
// (256 KB) is never formed: its rows split into the even and odd y halves
// ky = 2k + e_y, which are independent from the forward y transform up to
// the cropped inverse one.  The workgroup has two groups of 256 threads
// (four wavefronts each), one per half, each with its own N_y x N_z working
// set in LDS (2 x 66-68 KB), and 32 points a thread.  Per half:
//   A  forward y transform of every column z of x(y) W_{2N_y}^{y e_y}, as a
//      four-step FFT N_y = 32 x N2 (N2 = N_y / 32): 32-point register FFTs
//      over j1 (y = j2 + N2 j1, one thread per (z, j2)), the cross twiddle
//      W_{N_y}^{j2 k1} from an LDS table, then N2-point register FFTs over j2
//      after an exchange through LDS (k = k1 + 32 k2);
//   B  rows k through LDS; per row both z halves e_z: forward N_z-point
//      transform of r(z) W_{2N_z}^{z e_z}, times Ghat(k_x, 2k + e_y,
//      2m + e_z), inverse transform, times W_{2N_z}^{-z e_z}, summed;
//   C  the four-step inverse y transform back to the (z, j2) threads, times
//      W_{2N_y}^{-y e_y}.
// The halves are then summed through LDS (each finishes half of the
// points), scaled by 1 / (4 N_y N_z) and stored in place.
constexpr int BIG_T = 256;   // threads per half

template <int NY, int NZ>
struct BigPlane {
  static_assert(NY * NZ == 32 * BIG_T, "32 points per thread");
  static constexpr int N2 = NY / 32;            // second factor of the y transform
  static constexpr int KS = 32 / N2;            // k1 values per thread in the N2 stage
  static constexpr int RPT = NY / BIG_T;        // rows per thread in the z stage
  static constexpr int PB = NZ + 1;             // row pitch (rows of consecutive lanes in different banks)
  static constexpr int SZ_A = 32 * N2 * NZ + 2 * 32;
  static constexpr int SZ_B = NY * PB;
  static constexpr int SZ = SZ_A > SZ_B ? SZ_A : SZ_B;
  static constexpr size_t LDS = sizeof(float2) * (2 * SZ + NY + N2);
  // (k1, j2, z) layout, skewed by 2 slots per k1 so that the two k1 values
  // of a wavefront in the N2 stage fall in different banks
  __device__ static int ia(int k1, int j2, int z) { return (k1 * N2 + j2) * NZ + z + 2 * k1; }
  __device__ static int ib(int k, int z) { return k * PB + z; }
};

__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

template <int NY, int NZ, bool PR>
__global__ void __launch_bounds__(2 * BIG_T) k_fft_yz_big(YZArgs a, float2 *data, const float *ghat, long ch,
                                                          const uint32_t *colact) {
  using L = BigPlane<NY, NZ>;
  constexpr int N2 = L::N2, KS = L::KS, LY = 2 * NY, LZ = 2 * NZ;
  constexpr int B2 = clog2(N2), BZ = clog2(NZ);
  extern __shared__ float2 big_sm[];
  float2 *twy = big_sm + 2 * L::SZ;      // W_{N_y}^k, k < N_y
  float2 *twh = twy + NY;                // W_{2 N_y}^j, j < N2
  const int ey = __builtin_amdgcn_readfirstlane(threadIdx.x / BIG_T);   // the half (wavefront-uniform)
  const int t = threadIdx.x - ey * BIG_T;
  float2 *S = big_sm + ey * L::SZ;
  for (int k = threadIdx.x; k < NY; k += 2 * BIG_T) twy[k] = tw<-1>(k, NY);
  if (threadIdx.x < N2) twh[threadIdx.x] = tw<-1>(threadIdx.x, LY);
  // planes k_x-major over the channels, in XCD-contiguous ranges: the
  // channels of one k_x read the same spectrum plane, which then stays in
  // the XCD's L2 (in channel-major order every workgroup refetched its
  // 34 KB plane)
  const long lb = (long)xcd_block(blockIdx.x, gridDim.x);
  const long kx = lb / ch, chan = lb - kx * ch;
  float2 *io = data + (chan * a.two_nx + kx) * (long)(NY * NZ);
  const int fx = kx <= a.nx ? (int)kx : a.two_nx - (int)kx;
  const float *gpl = ghat + (long)fx * (NY + 1) * (NZ + 1);
  const int za = t % NZ, j2 = t / NZ;     // column and y = j2 + N2 j1 (stages A, C); k1 = j2 + N2 i (N2 stage)
  // the plane is read from memory once: each half loads 16 of a thread's
  // 32 points (j1 = 16 e_y + j) into its own LDS area, in the plane's own
  // order (y, z), and both halves then take all 32 from there
  float2 v[32];
  {
    float2 *P0 = big_sm, *P1 = big_sm + L::SZ;
    float2 *Pm = ey ? P1 : P0;
    if (PR) {
      // pruned: a column without an active node enters as zero (whatever the
      // buffer holds there); the load's offset then lies beyond the plane
      const __amdgpu_buffer_rsrc_t rio = buf_rsrc(io, (unsigned)(NY * NZ * 8));
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int cidx = (j2 + N2 * (16 * ey + j)) * NZ + za;
        const unsigned on = (colact[cidx >> 5] >> (cidx & 31)) & 1u;
        v[j] = buf_load2(rio, on ? (unsigned)cidx * 8u : X_DROP, 0);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = io[(j2 + N2 * (16 * ey + j)) * NZ + za];
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) Pm[(j2 + N2 * j) * NZ + za] = v[j];
    __syncthreads();                                    // twiddle tables and the plane
#pragma unroll
    for (int j1 = 0; j1 < 32; ++j1) v[j1] = (j1 < 16 ? P0 : P1)[(j2 + N2 * (j1 & 15)) * NZ + za];
    __syncthreads();                                    // both halves done before S is reused
  }
  if (ey) {
    const float2 wl = twh[j2];
#pragma unroll
    for (int j1 = 0; j1 < 32; ++j1) v[j1] = twmul<-1>(cmulf(v[j1], wl), N2 * j1, LY);
  }
  fft_dif<32, -1>(v);                                   // v[p] = X(k1 = brev(p))
#pragma unroll
  for (int p = 1; p < 32; ++p) v[p] = cmulf(v[p], twy[j2 * brev(p, 5)]);
#pragma unroll
  for (int p = 0; p < 32; ++p) S[L::ia(brev(p, 5), j2, za)] = v[p];
  __syncthreads();
  {
    float2 w[KS][N2];
#pragma unroll
    for (int i = 0; i < KS; ++i)
#pragma unroll
      for (int jj = 0; jj < N2; ++jj) w[i][jj] = S[L::ia(j2 + N2 * i, jj, za)];
#pragma unroll
    for (int i = 0; i < KS; ++i) fft_dif<N2, -1>(w[i]);   // w[i][p2] = Y(k1 + 32 brev(p2))
    __syncthreads();
#pragma unroll
    for (int i = 0; i < KS; ++i)
#pragma unroll
      for (int p2 = 0; p2 < N2; ++p2) S[L::ib(j2 + N2 * i + 32 * brev(p2, B2), za)] = w[i][p2];
  }
  __syncthreads();
  // z stage on this thread's rows
#pragma unroll 1
  for (int rr = 0; rr < L::RPT; ++rr) {
    const int k = t + BIG_T * rr, ky = 2 * k + ey;
    const int fy = ky <= NY ? ky : LY - ky;
    const float *grow = gpl + fy * (NZ + 1);
    float2 o[NZ];
    {
      float2 u[NZ];
#pragma unroll
      for (int z = 0; z < NZ; ++z) u[z] = S[L::ib(k, z)];
      fft_dif<NZ, -1>(u);                               // u[p] = Z(m = brev(p)), kz = 2 m
#pragma unroll
      for (int p = 0; p < NZ; ++p) {
        const int kz = 2 * brev(p, BZ), fz = kz <= NZ ? kz : LZ - kz;
        const float g = grow[fz];
        u[p] = make_float2(u[p].x * g, u[p].y * g);
      }
      fft_dit<NZ, +1>(u);                               // natural z
#pragma unroll
      for (int z = 0; z < NZ; ++z) o[z] = u[z];
    }
    {
      float2 u[NZ];
#pragma unroll
      for (int z = 0; z < NZ; ++z) u[z] = twmul<-1>(S[L::ib(k, z)], z, LZ);
      fft_dif<NZ, -1>(u);                               // kz = 2 m + 1
#pragma unroll
      for (int p = 0; p < NZ; ++p) {
        const int kz = 2 * brev(p, BZ) + 1, fz = kz <= NZ ? kz : LZ - kz;
        const float g = grow[fz];
        u[p] = make_float2(u[p].x * g, u[p].y * g);
      }
      fft_dit<NZ, +1>(u);
#pragma unroll
      for (int z = 0; z < NZ; ++z) S[L::ib(k, z)] = cadd(o[z], twmul<+1>(u[z], z, LZ));
    }
  }
  __syncthreads();
  {
    // inverse N2-point transforms over k2
    float2 w[KS][N2];
#pragma unroll
    for (int i = 0; i < KS; ++i)
#pragma unroll
      for (int p2 = 0; p2 < N2; ++p2) w[i][p2] = S[L::ib(j2 + N2 * i + 32 * brev(p2, B2), za)];
#pragma unroll
    for (int i = 0; i < KS; ++i) fft_dit<N2, +1>(w[i]);   // w[i][j2'] natural
    __syncthreads();
#pragma unroll
    for (int i = 0; i < KS; ++i)
#pragma unroll
      for (int jj = 0; jj < N2; ++jj) S[L::ia(j2 + N2 * i, jj, za)] = w[i][jj];
  }
  __syncthreads();
  // inverse 32-point transforms over k1
#pragma unroll
  for (int p = 0; p < 32; ++p) v[p] = S[L::ia(brev(p, 5), j2, za)];
#pragma unroll
  for (int p = 1; p < 32; ++p) v[p] = cmulf(v[p], conjf2(twy[j2 * brev(p, 5)]));
  fft_dit<32, +1>(v);                                   // v[j1] natural
  if (ey) {
    const float2 wl = conjf2(twh[j2]);
#pragma unroll
    for (int j1 = 0; j1 < 32; ++j1) v[j1] = twmul<+1>(cmulf(v[j1], wl), N2 * j1, LY);
  }
  // sum of the halves: half e finishes j1 in [16 e, 16 e + 16) and hands the
  // other range to its partner through its own LDS area
  __syncthreads();
  float2 *X = big_sm + (1 - ey) * L::SZ;                // the partner reads here
  float2 keep[16];
  if (ey) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      X[t + BIG_T * j] = v[j];
      keep[j] = v[16 + j];
    }
  } else {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      X[t + BIG_T * j] = v[16 + j];
      keep[j] = v[j];
    }
  }
  __syncthreads();
  const float sc = a.scale;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int j1 = 16 * ey + j;
    const float2 r = S[t + BIG_T * j];
    io[(j2 + N2 * j1) * NZ + za] = make_float2((keep[j].x + r.x) * sc, (keep[j].y + r.y) * sc);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_fft_axis(FftArgs a, const V2<T> *in, V2<T> *out, const T *ghat) {
  extern __shared__ unsigned char smraw[];
  V2<T> *tw = (V2<T> *)smraw;                  // Lf twiddles exp(-2 pi i k / Lf)
  V2<T> *sm = tw + a.Lf;                       // LB lines, stride ldl
  const int Lf = a.Lf, LB = a.LB, ldl = a.ldl, C = a.C;
  const long nlines = (long)a.A * C;
  const long line0 = (long)blockIdx.x * LB;
  const int nl = (int)min((long)LB, nlines - line0);   // valid lines in this tile
  fill_twiddles<T>(tw, Lf);
  // coalesced load of the tile; zero padding beyond n_in
  const int nin = a.n_in;
  if (C == 1) {
    const V2<T> *src = in + line0 * nin;       // nl * nin contiguous elements
    for (int idx = threadIdx.x; idx < LB * Lf; idx += blockDim.x) {
      int line = idx / Lf, k = idx - line * Lf;
      V2<T> v = cmk<T>(0, 0);
      if (line < nl && k < nin) v = src[(long)line * nin + k];
      sm[line * ldl + k] = v;
    }
  } else {
    // lines line0..line0+nl-1 have the same a when C % LB == 0 (enforced)
    long aa = line0 / C, cc = line0 - aa * C;
    const V2<T> *src = in + aa * (long)nin * C + cc;
    for (int idx = threadIdx.x; idx < LB * Lf; idx += blockDim.x) {
      int k = idx / LB, line = idx - k * LB;
      V2<T> v = cmk<T>(0, 0);
      if (line < nl && k < nin) v = src[(long)k * C + line];
      sm[line * ldl + k] = v;
    }
  }
  __syncthreads();
  stockham<T>(sm, tw, a.lb_sh, ldl, 1, a.lf_sh, a.sign);
  if (a.fused) {
    for (int idx = threadIdx.x; idx < LB * Lf; idx += blockDim.x) {
      int line = idx / Lf, k = idx - line * Lf;
      if (line >= nl) continue;
      long gl = line0 + line;
      int ky = (int)(gl & (a.two_ny - 1)), kx = (int)((gl / a.two_ny) & (a.two_nx - 1));
      int fx = kx <= a.nx ? kx : a.two_nx - kx;
      int fy = ky <= a.ny ? ky : a.two_ny - ky;
      int fz = k <= a.nz ? k : Lf - k;
      sm[line * ldl + k] = cscale<T>(sm[line * ldl + k], ghat[((long)fx * (a.ny + 1) + fy) * (a.nz + 1) + fz]);
    }
    __syncthreads();
    stockham<T>(sm, tw, a.lb_sh, ldl, 1, a.lf_sh, +1);
  }
  // coalesced store of the first n_out points
  const T sc = (T)a.scale;
  const int nout = a.n_out;
  if (C == 1) {
    V2<T> *dst = out + line0 * nout;
    for (int idx = threadIdx.x; idx < nl * nout; idx += blockDim.x) {
      int line = idx / nout, k = idx - line * nout;
      dst[(long)line * nout + k] = cscale<T>(sm[line * ldl + k], sc);
    }
  } else {
    long aa = line0 / C, cc = line0 - aa * C;
    V2<T> *dst = out + aa * (long)nout * C + cc;
    for (int idx = threadIdx.x; idx < LB * nout; idx += blockDim.x) {
      int k = idx / LB, line = idx - k * LB;
      if (line < nl) dst[(long)k * C + line] = cscale<T>(sm[line * ldl + k], sc);
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
  a.ldl = Lf + 1;
  // tile of LB lines within the LDS budget; at most 8 butterflies per thread
  // in the pass with the smallest radix (radix 8 passes, then one 4 or 2)
  const int vs = (int)sizeof(V2<T>);
  static int lds_max = -1;
  if (lds_max < 0) lds_max = allow_lds((const void *)k_fft_axis<T>, lds_budget()) ? lds_budget() : 65536;
  int lb = (lds_max / vs - Lf) / a.ldl;
  lb = std::min(lb, 8192 / Lf);                // 32 points per thread per pass
  if (lb < 1) lb = 1;
  int p2 = 1;
  while (p2 * 2 <= lb) p2 *= 2;
  lb = p2;
  if (C > 1) {
    while (lb > 1 && (C % lb) != 0) lb /= 2;  // a tile never straddles two values of a
  } else {
    lb = std::min(lb, 64);
  }
  a.LB = lb;
  a.lb_sh = ilog2(lb);
  a.lf_sh = ilog2(Lf);
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
  size_t shm = (size_t)Lf * vs + (size_t)lb * a.ldl * vs;
  k_fft_axis<T><<<cdiv(lines, lb), 256, shm, st>>>(a, in, out, ghat);
}

// Plane-kernel choice: the register variant exists for (N_y, N_z) =
// (64, 32), (32, 16), (16, 8) in FP32; fft_plan 1 selects the LDS Stockham
// variant (both are exact transforms; the choice is a tuning knob).
template <typename T>
static bool reg_plane_ok(const GridMaps &g, int Ny, int Nz) {
  if (sizeof(T) != 4 || g.fft_plan == 1) return false;
  return (Ny == 64 && Nz == 32) || (Ny == 32 && Nz == 16) || (Ny == 16 && Nz == 8);
}

template <int NY, int NZ>
static void launch_yz_reg_n(float2 *data, const float *ghat, const YZArgs &y, long ch, const uint64_t *zmask,
                            hipStream_t st) {
  const unsigned nb = (unsigned)(ch * y.two_nx);
  if (zmask)
    k_fft_yz_reg<NY, NZ, true><<<nb, 2 * NY, 0, st>>>(y, data, ghat, ch, zmask);
  else
    k_fft_yz_reg<NY, NZ, false><<<nb, 2 * NY, 0, st>>>(y, data, ghat, ch, nullptr);
}
static void launch_yz_reg(float2 *data, const float *ghat, const YZArgs &y, long ch, const uint64_t *zmask,
                          hipStream_t st) {
  if (y.ny == 64) launch_yz_reg_n<64, 32>(data, ghat, y, ch, zmask, st);
  else if (y.ny == 32) launch_yz_reg_n<32, 16>(data, ghat, y, ch, zmask, st);
  else launch_yz_reg_n<16, 8>(data, ghat, y, ch, zmask, st);
}

// Big-plane kernel: FP32, (N_y, N_z) = (256, 32) or (512, 16), its LDS
// (about 140 KB) granted.
template <int NY, int NZ>
static bool big_plane_lds() {
  static int ok = -1;
  if (ok < 0) {
    int dev = 0, q = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&q, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) q = 0;
    const int need = (int)BigPlane<NY, NZ>::LDS;
    ok = need <= q &&
         hipFuncSetAttribute((const void *)k_fft_yz_big<NY, NZ, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             need) == hipSuccess &&
         hipFuncSetAttribute((const void *)k_fft_yz_big<NY, NZ, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             need) == hipSuccess;
    if (!ok) (void)hipGetLastError();
  }
  return ok == 1;
}
template <typename T>
static bool big_plane_ok(const GridMaps &g, int Ny, int Nz) {
  if (sizeof(T) != 4 || g.fft_plan == 1) return false;
  if (Ny == 256 && Nz == 32) return big_plane_lds<256, 32>();
  if (Ny == 512 && Nz == 16) return big_plane_lds<512, 16>();
  return false;
}
// colact non-null: pruned (columns without an active node read as zero)
static void launch_yz_big(float2 *data, const float *ghat, const YZArgs &y, long ch, const uint32_t *colact,
                          hipStream_t st) {
  const unsigned nb = (unsigned)(ch * y.two_nx);
  if (y.ny == 256) {
    if (colact)
      k_fft_yz_big<256, 32, true><<<nb, 2 * BIG_T, BigPlane<256, 32>::LDS, st>>>(y, data, ghat, ch, colact);
    else
      k_fft_yz_big<256, 32, false><<<nb, 2 * BIG_T, BigPlane<256, 32>::LDS, st>>>(y, data, ghat, ch, nullptr);
  } else {
    if (colact)
      k_fft_yz_big<512, 16, true><<<nb, 2 * BIG_T, BigPlane<512, 16>::LDS, st>>>(y, data, ghat, ch, colact);
    else
      k_fft_yz_big<512, 16, false><<<nb, 2 * BIG_T, BigPlane<512, 16>::LDS, st>>>(y, data, ghat, ch, nullptr);
  }
}

// Register X passes: FP32, N_x in {32, 64, 128, 256}, N_y N_z a multiple of
// 32, one channel of the padded grid below 2^31 bytes.
template <typename T>
static bool reg_x_ok(const GridMaps &g, int Nx, long C, long ch) {
  (void)ch;
  if (sizeof(T) != 4 || g.fft_plan == 1 || !g.xtw) return false;
  if (2.0 * Nx * (double)C * 8.0 >= 2147483647.0) return false;   // one channel per launch at least
  return (Nx == 256 || Nx == 128 || Nx == 64 || Nx == 32) && C % 32 == 0;
}

template <int NX, int SIGN>
static void launch_x_reg_n(const float2 *in, float2 *out, int C, int ncol, const float2 *xtw, const uint32_t *xmask,
                           const uint8_t *cgrp, unsigned nb, hipStream_t st) {
  if (SIGN < 0) {
    if (xmask)
      k_fft_x_fwd<NX, true><<<nb, 256, 0, st>>>(in, out, C, ncol, xtw, xmask, cgrp);
    else
      k_fft_x_fwd<NX, false><<<nb, 256, 0, st>>>(in, out, C, ncol, xtw, nullptr, nullptr);
  } else {
    const float2 *itw = xtw + 2 * NX;   // the inverse table follows the forward one
    if (xmask)
      k_fft_x_inv<NX, true><<<nb, 256, 0, st>>>(in, out, C, ncol, itw, xmask, cgrp);
    else
      k_fft_x_inv<NX, false><<<nb, 256, 0, st>>>(in, out, C, ncol, itw, nullptr, nullptr);
  }
}
// xmask / cgrp non-null: pruned passes.  The channels are split over
// launches so that each addresses less than 2^31 bytes (32-bit byte offsets,
// and the pruned passes' out-of-range offset stays beyond every buffer).
static void launch_x_reg(const float2 *in, float2 *out, int Nx, long C, long ch, int sign,
                         const float2 *xtw, const uint32_t *xmask, const uint8_t *cgrp, hipStream_t st) {
  const long per = 2L * Nx * C * 8;             // bytes of one channel's longer side
  const long cmax = std::max(1L, 2147483647L / per);
  if (ch > cmax) {
    const long in_ch = (sign < 0 ? Nx : 2L * Nx) * C, out_ch = (sign < 0 ? 2L * Nx : Nx) * C;
    for (long c0 = 0; c0 < ch; c0 += cmax)
      launch_x_reg(in + c0 * in_ch, out + c0 * out_ch, Nx, C, std::min(cmax, ch - c0), sign, xtw, xmask, cgrp,
                   st);
    return;
  }
  const int ncol = (int)(ch * C), Ci = (int)C;
  const unsigned nb = (unsigned)(ncol / 32);   // C % 32 == 0 (reg_x_ok)
  if (sign < 0) {
    if (Nx == 256) launch_x_reg_n<256, -1>(in, out, Ci, ncol, xtw, xmask, cgrp, nb, st);
    else if (Nx == 128) launch_x_reg_n<128, -1>(in, out, Ci, ncol, xtw, xmask, cgrp, nb, st);
    else if (Nx == 64) launch_x_reg_n<64, -1>(in, out, Ci, ncol, xtw, xmask, cgrp, nb, st);
    else launch_x_reg_n<32, -1>(in, out, Ci, ncol, xtw, xmask, cgrp, nb, st);
  } else {
    if (Nx == 256) launch_x_reg_n<256, 1>(in, out, Ci, ncol, xtw, xmask, cgrp, nb, st);
    else if (Nx == 128) launch_x_reg_n<128, 1>(in, out, Ci, ncol, xtw, xmask, cgrp, nb, st);
    else if (Nx == 64) launch_x_reg_n<64, 1>(in, out, Ci, ncol, xtw, xmask, cgrp, nb, st);
    else launch_x_reg_n<32, 1>(in, out, Ci, ncol, xtw, xmask, cgrp, nb, st);
  }
}

// The pruned passes run where both register passes do and the masks exist.
template <typename T>
static bool prune_ok(const GridMaps &g, long ch) {
  const int Nx = g.dims[0], Ny = g.dims[1], Nz = g.dims[2];
  if (!(g.prune && g.xmask && reg_x_ok<T>(g, Nx, (long)Ny * Nz, ch))) return false;
  return (reg_plane_ok<T>(g, Ny, Nz) && g.zmask) || (big_plane_ok<T>(g, Ny, Nz) && g.colact);
}

template <typename T>
void convolve(const GridMaps &g, V2<T> *Q, V2<T> *T1, V2<T> *T2, int R, hipStream_t st, PassHook *hook) {
  const int Nx = g.dims[0], Ny = g.dims[1], Nz = g.dims[2];
  long ch = 3L * R;
  const bool xreg = reg_x_ok<T>(g, Nx, (long)Ny * Nz, ch);
  const bool pr = prune_ok<T>(g, ch);
  const uint32_t *xm = pr ? g.xmask : nullptr;
  const uint8_t *cg = pr ? g.cgrp : nullptr;
  // X forward: [ch][Nx][Ny*Nz] -> [ch][2Nx][Ny*Nz]
  if (hook) hook->pass(0, st);
  if (xreg)
    launch_x_reg((const float2 *)Q, (float2 *)T1, Nx, (long)Ny * Nz, ch, -1, g.xtw, xm, cg, st);
  else
    fft_axis<T>(Q, T1, ch, (long)Ny * Nz, Nx, 2 * Nx, 2 * Nx, -1, 1.0f, nullptr, nullptr, st);
  const int vs = (int)sizeof(V2<T>);
  const int pitch = 2 * Nz + 1;
  const size_t yz_lds = (size_t)(2 * Ny + 2 * Nz + 2 * Ny * pitch) * vs;
  if (reg_plane_ok<T>(g, Ny, Nz)) {
    if (hook) hook->pass(1, st);
    YZArgs y{};
    y.ny = Ny;
    y.nz = Nz;
    y.nx = Nx;
    y.two_nx = 2 * Nx;
    y.scale = 1.0f / (4.0f * Ny * Nz);
    launch_yz_reg((float2 *)T1, (const float *)g.ghat, y, ch, pr ? g.zmask : nullptr, st);
    if (hook) hook->pass(4, st);
    if (xreg)
      launch_x_reg((const float2 *)T1, (float2 *)Q, Nx, (long)Ny * Nz, ch, +1, g.xtw, xm, cg, st);
    else
      fft_axis<T>(T1, Q, ch, (long)Ny * Nz, 2 * Nx, Nx, 2 * Nx, +1, 1.0f / (2.0f * Nx), nullptr, nullptr, st);
    if (hook) hook->done(st);
    return;
  }
  if (big_plane_ok<T>(g, Ny, Nz)) {
    if (hook) hook->pass(1, st);
    YZArgs y{};
    y.ny = Ny;
    y.nz = Nz;
    y.nx = Nx;
    y.two_nx = 2 * Nx;
    y.scale = 1.0f / (4.0f * Ny * Nz);
    launch_yz_big((float2 *)T1, (const float *)g.ghat, y, ch, pr ? g.colact : nullptr, st);
    if (hook) hook->pass(4, st);
    if (xreg)
      launch_x_reg((const float2 *)T1, (float2 *)Q, Nx, (long)Ny * Nz, ch, +1, g.xtw, xm, cg, st);
    else
      fft_axis<T>(T1, Q, ch, (long)Ny * Nz, 2 * Nx, Nx, 2 * Nx, +1, 1.0f / (2.0f * Nx), nullptr, nullptr, st);
    if (hook) hook->done(st);
    return;
  }
  if (4L * Ny * Nz <= 8192 && allow_lds((const void *)k_fft_yz<T>, (int)yz_lds)) {
    // fused Y, Z(+ spectrum), inverse Z, inverse Y on each (channel, kx) plane
    if (hook) hook->pass(1, st);
    YZArgs y{};
    y.ny = Ny;
    y.nz = Nz;
    y.ly_sh = ilog2(2 * Ny);
    y.lz_sh = ilog2(2 * Nz);
    y.pitch = pitch;
    y.nx = Nx;
    y.two_nx = 2 * Nx;
    y.scale = 1.0f / (4.0f * Ny * Nz);
    k_fft_yz<T><<<(unsigned)(ch * 2 * Nx), 256, yz_lds, st>>>(y, T1, (const T *)g.ghat);
    if (hook) hook->pass(4, st);
    fft_axis<T>(T1, Q, ch, (long)Ny * Nz, 2 * Nx, Nx, 2 * Nx, +1, 1.0f / (2.0f * Nx), nullptr, nullptr, st);
    if (hook) hook->done(st);
    return;
  }
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

// Whether convolve needs the T2 buffer (the unfused Y / Z passes): false
// wherever a fused plane kernel takes the Y, Z and inverse passes.
bool convolve_uses_t2(const GridMaps &g, int fp64) {
  const int Ny = g.dims[1], Nz = g.dims[2];
  if (!fp64 && (reg_plane_ok<float>(g, Ny, Nz) || big_plane_ok<float>(g, Ny, Nz))) return false;
  const int vs = fp64 ? (int)sizeof(double2) : (int)sizeof(float2);
  const size_t yz_lds = (size_t)(2 * Ny + 2 * Nz + 2 * Ny * (2 * Nz + 1)) * vs;
  const void *fn = fp64 ? (const void *)k_fft_yz<double> : (const void *)k_fft_yz<float>;
  return !(4L * Ny * Nz <= 8192 && allow_lds(fn, (int)yz_lds));
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
constexpr int IRG = 4;   // right-hand sides per thread in the interpolation

template <typename T>
__global__ void k_interp_tri(GridMaps g, const V2<T> *phi, double2 *U, int R) {
  const int r0 = blockIdx.y * IRG;
  const int t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t >= g.n) return;
  const int nr = min(IRG, R - r0);
  const int Ny = g.dims[1], Nz = g.dims[2];
  const T *w = (const T *)g.tri_w + (size_t)t * 256;
  const int ax = g.anchor[3 * t], ay = g.anchor[3 * t + 1], az = g.anchor[3 * t + 2];
  double acc[IRG][8];
#pragma unroll
  for (int q = 0; q < IRG; ++q)
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[q][c] = 0;
  for (int k = 0; k < 64; ++k) {
    const int i = k >> 4, j = (k >> 2) & 3, l = k & 3;
    const long node = ((long)(ax + i) * Ny + (ay + j)) * Nz + (az + l);
    const double m0 = w[4 * k], m1x = w[4 * k + 1], m1y = w[4 * k + 2], m1z = w[4 * k + 3];
#pragma unroll
    for (int q = 0; q < IRG; ++q) {
      if (q < nr) {
        const V2<T> *P = phi + (size_t)(r0 + q) * 3 * g.N + node;
        V2<T> vx = P[0], vy = P[g.N], vz = P[2 * (size_t)g.N];
        acc[q][0] += m1x * vx.x + m1y * vy.x + m1z * vz.x;
        acc[q][1] += m1x * vx.y + m1y * vy.y + m1z * vz.y;
        acc[q][2] += m0 * vx.x;
        acc[q][3] += m0 * vx.y;
        acc[q][4] += m0 * vy.x;
        acc[q][5] += m0 * vy.y;
        acc[q][6] += m0 * vz.x;
        acc[q][7] += m0 * vz.y;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < IRG; ++q) {
    if (q < nr) {
      double2 *o = U + ((size_t)t * R + r0 + q) * 4;   // U[t][r][4]
      o[0] = make_double2(acc[q][0], acc[q][1]);
      o[1] = make_double2(acc[q][2], acc[q][3]);
      o[2] = make_double2(acc[q][4], acc[q][5]);
      o[3] = make_double2(acc[q][6], acc[q][7]);
    }
  }
}

// FP32 path: phi ([R][3][N], grid channel 3r + c) is first transposed to
// node-major [N_a][3][R] (component-major, right-hand side innermost) over
// the N_a active nodes only (those some triangle's stencil touches; every
// other node is never read).  One workgroup per (active-node tile of 64,
// component c, block of 32 right-hand sides): reads of 32 channels' runs of
// 64 active nodes, writes of 32 consecutive right-hand sides of a node,
// through an LDS tile (16.6 KB; a 64 x 64 tile took twice that and ran
// slower).
__global__ void __launch_bounds__(256) k_transpose_c64(const float2 *in, float2 *out, int R, int N, int na,
                                                       const int *act) {
  __shared__ float2 tile[32][65];   // [right-hand side][node]
  const int a0 = (int)xcd_block(blockIdx.x, gridDim.x) * 64;
  const int c = blockIdx.y % 3, r0 = (blockIdx.y / 3) * 32;
  {
    const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;   // 64 x 4
    const bool ok = a0 + lane < na;
    const int node = ok ? act[a0 + lane] : 0;
    for (int k = row; k < 32; k += 4) {
      const int r = r0 + k;
      if (r < R && ok) tile[k][lane] = in[(size_t)(3 * r + c) * N + node];
    }
  }
  __syncthreads();
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int k = ty; k < 64; k += 8) {
    const int a = a0 + k, r = r0 + tx;
    if (r < R && a < na) out[(size_t)a * 3 * R + (size_t)c * R + r] = tile[tx][k];
  }
}

// Triangles with the same anchor read the same 64 stencil nodes: a
// workgroup takes up to INTERP_GROUP of them and a block of 64 right-hand
// sides, each of its three wavefronts one component c of the grid
// potential (lane = right-hand side), and reads a node's value once for all
// of the group's triangles.  The nodes' active positions and the triangles'
// FP64 weights (M0 and the wavefront's M1 component) are uniform, so they
// are scalar loads; a lane's node values are loaded KC at a time before they
// are used.  Per (triangle, channel) the sums run over k = 0 .. 63 in order.
// read-only data addressed uniformly: through the constant address space the
// compiler may use scalar loads even though the kernel also stores to memory
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T *uniform_ro(const T *p) {
  return (const __attribute__((address_space(4))) T *)p;
}

__global__ void __launch_bounds__(192) k_interp_grp(GridMaps g, const float2 *phiT, double2 *U, int R) {
  constexpr int IG = INTERP_GROUP;
  __shared__ double2 s0[IG][3][64];
  // one workgroup per (block of 64 right-hand sides, group), the groups of
  // one block consecutive: an XCD's workgroups then read neighbouring
  // groups' stencil nodes within one block of channels, a working set that
  // fits its L2
  const int ch = 3 * R;
  const int lb = (int)xcd_block(blockIdx.x, gridDim.x), rbk = lb / g.nig, grp = lb - rbk * g.nig;
  const int q0 = g.ig_off[grp], gn = g.ig_off[grp + 1] - q0;
  const int c = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const int r = rbk * 64 + lane;
  const bool ok = r < R;
  const int cc = c * R + min(r, R - 1);   // phiT[a][c][r]
  int tq[IG];
  const __attribute__((address_space(4))) double *wq[IG];
#pragma unroll
  for (int q = 0; q < IG; ++q) {
    tq[q] = g.ig_tri[q0 + min(q, gn - 1)];
    wq[q] = uniform_ro(g.tri_wd + (size_t)tq[q] * 256);
  }
  const __attribute__((address_space(4))) int *ia = uniform_ro(g.ig_act + (size_t)grp * 64);
  constexpr int KC = 16;   // node values in flight per lane
  double a0x[IG], a0y[IG], a1x[IG], a1y[IG];
#pragma unroll
  for (int q = 0; q < IG; ++q) a0x[q] = a0y[q] = a1x[q] = a1y[q] = 0;
  for (int kh = 0; kh < 64; kh += KC) {
    float2 v[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) v[k] = phiT[(size_t)ia[kh + k] * ch + cc];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const double vx = ok ? (double)v[k].x : 0.0, vy = ok ? (double)v[k].y : 0.0;
#pragma unroll
      for (int q = 0; q < IG; ++q) {
        const auto *w = wq[q] + 4 * (kh + k);   // (M0, M1x, M1y, M1z)
        const double m0 = w[0], m1 = w[1 + c];
        a0x[q] += m1 * vx;
        a0y[q] += m1 * vy;
        a1x[q] += m0 * vx;
        a1y[q] += m0 * vy;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < IG; ++q) s0[q][c][lane] = make_double2(a0x[q], a0y[q]);
  __syncthreads();
  if (ok) {
#pragma unroll
    for (int q = 0; q < IG; ++q) {
      if (q < gn) {
        double2 *o = U + ((size_t)tq[q] * R + r) * 4;   // U[t][r][4]
        o[1 + c] = make_double2(a1x[q], a1y[q]);
        if (c == 0) {
          const double2 p0 = s0[q][0][lane], p1 = s0[q][1][lane], p2 = s0[q][2][lane];
          o[0] = make_double2(p0.x + p1.x + p2.x, p0.y + p1.y + p2.y);
        }
      }
    }
  }
}

template <typename T>
void interp_tri(const GridMaps &g, const V2<T> *phi, double2 *U, int R, hipStream_t st, void *scratch) {
  (void)scratch;
  k_interp_tri<T><<<dim3(cdiv(g.n, 128), cdiv(R, IRG)), 128, 0, st>>>(g, phi, U, R);
}

template <>
void interp_tri<float>(const GridMaps &g, const float2 *phi, double2 *U, int R, hipStream_t st, void *scratch) {
  // node-major copy of phi ([N_a][3][R] complex64) in the caller's free scratch
  float2 *phiT = (float2 *)scratch;
  k_transpose_c64<<<dim3(cdiv(g.nact, 64), 3 * cdiv(R, 32)), 256, 0, st>>>(phi, phiT, R, g.N, g.nact, g.act);
  if (g.nig > 0) k_interp_grp<<<(unsigned)g.nig * cdiv(R, 64), 192, 0, st>>>(g, phiT, U, R);
}

// ===========================================================================
// edge phase: far field from the two triangles, near-field CSR, Gram, combine
// ===========================================================================
// One thread per (edge, RHS), RHS fastest: the near-field row's values and
// columns are shared by the RHS lanes and each gathered column alpha[col][.]
// is one contiguous segment, so every load of the sparse product coalesces.
__global__ void k_combine(CombineMaps c, const double2 *alpha, const double2 *U, const double2 *zs,
                          const double2 *jw, double2 *y, int R, int mode) {
  const long idx = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
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
  if (mode & 8) {
    // near part already in y (dense-tile product)
    const double2 v = y[idx];
    kx += v.x;
    ky += v.y;
  } else if (mode & 2) {
    // four nonzeros per step: their column and value loads, then the four
    // gathers, are independent (more loads in flight).  Summation order, the
    // same in every near-field kernel: nonzero j of the row goes to the even
    // (far part included) or odd partial sum by its parity, in order; then
    // even += odd.
    const int64_t q0 = c.nf_rowptr[e], q1 = c.nf_rowptr[e + 1];
    int64_t q = q0;
    double ax = 0, ay = 0;
    for (; q + 4 <= q1; q += 4) {
      const int c0 = c.nf_col[q], c1 = c.nf_col[q + 1], c2 = c.nf_col[q + 2], c3 = c.nf_col[q + 3];
      const double v0 = c.nf_val[q], v1 = c.nf_val[q + 1], v2 = c.nf_val[q + 2], v3 = c.nf_val[q + 3];
      const double2 x0 = alpha[(size_t)c0 * R + r], x1 = alpha[(size_t)c1 * R + r];
      const double2 x2 = alpha[(size_t)c2 * R + r], x3 = alpha[(size_t)c3 * R + r];
      kx += v0 * x0.x;
      ky += v0 * x0.y;
      ax += v1 * x1.x;
      ay += v1 * x1.y;
      kx += v2 * x2.x;
      ky += v2 * x2.y;
      ax += v3 * x3.x;
      ay += v3 * x3.y;
    }
    for (; q < q1; ++q) {
      const double v = c.nf_val[q];
      const double2 x = alpha[(size_t)c.nf_col[q] * R + r];
      if ((q - q0) & 1) {
        ax += v * x.x;
        ay += v * x.y;
      } else {
        kx += v * x.x;
        ky += v * x.y;
      }
    }
    kx += ax;
    ky += ay;
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

// Tiled near-field product: one workgroup per (row tile, group of CRC
// right-hand sides).  The tile's rows touch few distinct columns (geometric
// neighbours share most of their near lists), so alpha of those columns is
// staged in LDS once and every nonzero reads it from there; the CSR values
// and slots are shared by the CRC lanes of a row.  The chunks of one tile
// are consecutive on one XCD, so its CSR rows are read from HBM once.
constexpr int CLDS = 120 * 1024;   // staging bytes

// lane K of each 16-lane row to the whole row (DPP row_newbcast; no old value)
template <int K>
__device__ __forceinline__ int row_bcast(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + K, 0xF, 0xF, false);
}
// lane K of each quad of lanes to the whole quad (DPP quad_perm [K,K,K,K])
template <int K>
__device__ __forceinline__ int quad_bcast(int v) {
  return __builtin_amdgcn_mov_dpp(v, K * 0x55, 0xF, 0xF, false);
}
// f(integral_constant<int, K>) for K = B .. E - 1
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

int combine_tile_cap(int rc) { return std::min(CLDS / (rc * 16), 65535); }

template <int CRC>
__global__ void __launch_bounds__(512) k_combine_tiled(CombineMaps c, const double2 *alpha, const double2 *U,
                                                       const double2 *zs, const double2 *jw, double2 *y, int R,
                                                       int mode) {
  extern __shared__ double2 sA[];   // [column slot][CRC]
  const int nch = (R + CRC - 1) / CRC;
  const int lb = (int)xcd_block(blockIdx.x, gridDim.x);
  const int tile = lb / nch, r0 = (lb - tile * nch) * CRC;
  const int u0 = c.ct_off[tile], nu = c.ct_off[tile + 1] - u0;
  // staging: eight (column index, alpha) load pairs in flight per thread
  // (each pair is two dependent loads, so one at a time would leave the CU
  // idle for most of the staging)
  {
    constexpr int SU = 8;
    const int tot = nu * CRC;
    for (int i0 = threadIdx.x; i0 < tot; i0 += SU * (int)blockDim.x) {
      int col[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int i = min(i0 + u * (int)blockDim.x, tot - 1);
        col[u] = c.ct_col[u0 + i / CRC];
      }
      double2 v[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int i = min(i0 + u * (int)blockDim.x, tot - 1), rr = i % CRC;
        v[u] = r0 + rr < R ? alpha[(size_t)col[u] * R + r0 + rr] : make_double2(0, 0);
      }
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int i = i0 + u * (int)blockDim.x;
        if (i < tot) sA[i] = v[u];
      }
    }
  }
  __syncthreads();
  // every lane stays to the end (the rows' nonzeros are shared across lanes);
  // lanes past the last row or right-hand side read clamped indices and
  // store nothing
  const int rr = threadIdx.x % CRC, e0 = tile * c.ctr + threadIdx.x / CRC, r0c = r0 + rr;
  const bool live = e0 < c.b && r0c < R;
  const int e = min(e0, c.b - 1), r = min(r0c, R - 1);
  double kx = 0, ky = 0;
  if (mode & 1) {
    for (int side = 0; side < 2; ++side) {
      const int t = c.efar_t[2 * e + side];
      const double sg = c.efar_s[2 * e + side];
      const double *p = c.efar_pl + 6 * (size_t)e + 3 * side;
      const double2 *u = U + ((size_t)t * R + r) * 4;
      const double vx = u[0].x - (p[0] * u[1].x + p[1] * u[2].x + p[2] * u[3].x);
      const double vy = u[0].y - (p[0] * u[1].y + p[1] * u[2].y + p[2] * u[3].y);
      kx += sg * vx;
      ky += sg * vy;
    }
  }
  if ((mode & 2) && CRC == 16) {
    // the 16 lanes of a row (one DPP row) load 16 nonzeros at a time, one
    // each, and broadcast them in turn (row_newbcast).  Loads run four
    // batches ahead: the next four batches are loaded (clamped index, no
    // branch) before the current four are used.  Lanes past their row's end
    // carry zeros.
    const int64_t q0 = c.nf_rowptr[e], q1 = e0 < c.b ? c.nf_rowptr[e + 1] : q0;
    const int64_t qlast = max(c.nf_rowptr[c.b] - 1, (int64_t)0);   // empty arrays hold 16 bytes
    double ax = 0, ay = 0;
    auto batch = [&](double vc, int sc) {
      double2 xv[16];
      static_for<0, 16>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        xv[K] = sA[row_bcast<K>(sc) * CRC + rr];
      });
      const int vlo = __double2loint(vc), vhi = __double2hiint(vc);
      static_for<0, 16>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        const double v = __hiloint2double(row_bcast<K>(vhi), row_bcast<K>(vlo));
        if (K & 1) {
          ax += v * xv[K].x;
          ay += v * xv[K].y;
        } else {
          kx += v * xv[K].x;
          ky += v * xv[K].y;
        }
      });
    };
    constexpr int NB = 4;
    auto fetch = [&](int64_t q, double &v, int &sl) {
      const int64_t qc = min(q, qlast);
      const double vv = c.nf_val[qc];
      const int ss = (int)c.nf_slot[qc];
      v = q < q1 ? vv : 0.0;
      sl = q < q1 ? ss : 0;
    };
    double vb[NB];
    int sb[NB];
    int64_t qb = q0;
#pragma unroll
    for (int j = 0; j < NB; ++j) fetch(qb + 16 * j + rr, vb[j], sb[j]);
    while (__any(qb < q1)) {
      double vn[NB];
      int sn[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) fetch(qb + 16 * (NB + j) + rr, vn[j], sn[j]);
#pragma unroll
      for (int j = 0; j < NB; ++j)
        if (__any(qb + 16 * j < q1)) batch(vb[j], sb[j]);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        vb[j] = vn[j];
        sb[j] = sn[j];
      }
      qb += 16 * NB;
    }
    kx += ax;
    ky += ay;
  } else if ((mode & 2) && CRC == 4) {
    // the 4 lanes of a row (a DPP quad) load 4 nonzeros at a time, one each,
    // and broadcast them in turn (quad_perm); loads run eight batches ahead.
    // Same summation order as above (nonzero j of the row to the partial
    // sum of its parity, in order).
    const int64_t q0 = c.nf_rowptr[e], q1 = e0 < c.b ? c.nf_rowptr[e + 1] : q0;
    const int64_t qlast = max(c.nf_rowptr[c.b] - 1, (int64_t)0);
    double ax = 0, ay = 0;
    auto batch = [&](double vc, int sc) {
      double2 xv[4];
      static_for<0, 4>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        xv[K] = sA[quad_bcast<K>(sc) * CRC + rr];
      });
      const int vlo = __double2loint(vc), vhi = __double2hiint(vc);
      static_for<0, 4>([&](auto KK) {
        constexpr int K = decltype(KK)::value;
        const double v = __hiloint2double(quad_bcast<K>(vhi), quad_bcast<K>(vlo));
        if (K & 1) {
          ax += v * xv[K].x;
          ay += v * xv[K].y;
        } else {
          kx += v * xv[K].x;
          ky += v * xv[K].y;
        }
      });
    };
    constexpr int NB = 8;
    auto fetch = [&](int64_t q, double &v, int &sl) {
      const int64_t qc = min(q, qlast);
      const double vv = c.nf_val[qc];
      const int ss = (int)c.nf_slot[qc];
      v = q < q1 ? vv : 0.0;
      sl = q < q1 ? ss : 0;
    };
    double vb[NB];
    int sb[NB];
    int64_t qb = q0;
#pragma unroll
    for (int j = 0; j < NB; ++j) fetch(qb + 4 * j + rr, vb[j], sb[j]);
    while (__any(qb < q1)) {
      double vn[NB];
      int sn[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) fetch(qb + 4 * (NB + j) + rr, vn[j], sn[j]);
#pragma unroll
      for (int j = 0; j < NB; ++j)
        if (__any(qb + 4 * j < q1)) batch(vb[j], sb[j]);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        vb[j] = vn[j];
        sb[j] = sn[j];
      }
      qb += 4 * NB;
    }
    kx += ax;
    ky += ay;
  } else if (mode & 2) {
    const int64_t q0 = c.nf_rowptr[e], q1 = e0 < c.b ? c.nf_rowptr[e + 1] : q0;
    int64_t q = q0;
    double ax = 0, ay = 0;
    for (; q + 4 <= q1; q += 4) {
      const int s0 = c.nf_slot[q], s1 = c.nf_slot[q + 1], s2 = c.nf_slot[q + 2], s3 = c.nf_slot[q + 3];
      const double v0 = c.nf_val[q], v1 = c.nf_val[q + 1], v2 = c.nf_val[q + 2], v3 = c.nf_val[q + 3];
      const double2 x0 = sA[s0 * CRC + rr], x1 = sA[s1 * CRC + rr];
      const double2 x2 = sA[s2 * CRC + rr], x3 = sA[s3 * CRC + rr];
      kx += v0 * x0.x;
      ky += v0 * x0.y;
      ax += v1 * x1.x;
      ay += v1 * x1.y;
      kx += v2 * x2.x;
      ky += v2 * x2.y;
      ax += v3 * x3.x;
      ay += v3 * x3.y;
    }
    for (; q < q1; ++q) {
      const double v = c.nf_val[q];
      const double2 x = sA[c.nf_slot[q] * CRC + rr];
      if ((q - q0) & 1) {
        ax += v * x.x;
        ay += v * x.y;
      } else {
        kx += v * x.x;
        ky += v * x.y;
      }
    }
    kx += ax;
    ky += ay;
  }
  double2 out;
  if (mode & 4) {
    double gx = 0, gy = 0;
    for (int q = 0; q < 5; ++q) {
      const double v = c.gram_val[5 * e + q];
      const double2 x = alpha[(size_t)c.gram_col[5 * e + q] * R + r];
      gx += v * x.x;
      gy += v * x.y;
    }
    const double2 z = zs[r], j = jw[r];
    out.x = z.x * gx - z.y * gy + j.x * kx - j.y * ky;
    out.y = z.x * gy + z.y * gx + j.x * ky + j.y * kx;
  } else {
    out = make_double2(kx, ky);
  }
  if (live) y[(size_t)e * R + r] = out;
}

// Near-field product on FP64 matrix cores over dense row tiles: y_near =
// L_T a for each tile T (32 rows x its column list), with the right-hand
// sides as 2R real columns (re, im interleaved, which is alpha's memory
// layout).  One workgroup per (tile, 64 right-hand sides): wave w computes
// the 32 rows x real columns [32 w, 32 w + 32) of its chunk as 2 x 2 blocks
// of v_mfma_f64_16x16x4 (lane l holds A: row l % 16, k l / 16; B: k l / 16,
// column l % 16; D register i: row l / 16 + 4 i, column l % 16), k in
// steps of 4 over the tile's columns.  A comes from the tile's values (shared by the tile's
// workgroups through the caches), B from alpha's rows of the tile's columns.
// Real columns past 2R read a clamped address and are not stored.
typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int DN_RHS = 64;   // right-hand sides per workgroup

__global__ void __launch_bounds__(256) k_near_dense(CombineMaps c, const double *alpha, double *y, int R) {
  const int nch = (R + DN_RHS - 1) / DN_RHS;
  const int lb = (int)xcd_block(blockIdx.x, gridDim.x);
  const int T = lb / nch, r0 = (lb - T * nch) * DN_RHS;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ka = lane >> 4, ra = lane & 15;
  const int64_t k0 = c.dn_off[T], nk = c.dn_off[T + 1] - k0;   // a multiple of 16
  const double *A = c.dn_val + 32 * k0 + ra * 4 + ka;
  const int *cols = c.dn_col + k0 + ka;
  const long R2 = 2L * R;
  const long n0 = 2L * r0 + 32 * w + ra, n1 = n0 + 16;
  const long m0 = min(n0, R2 - 1), m1 = min(n1, R2 - 1);
  dbl4 acc00 = {0, 0, 0, 0}, acc01 = {0, 0, 0, 0}, acc10 = {0, 0, 0, 0}, acc11 = {0, 0, 0, 0};
  for (int64_t kq = 0; kq < nk; kq += 16) {
    // four k-steps: all loads first, then the sixteen products
    long col[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) col[s] = cols[kq + 4 * s];
    double a0[4], a1[4], b0[4], b1[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      a0[s] = A[(kq + 4 * s) * 32];
      a1[s] = A[(kq + 4 * s) * 32 + 64];
      b0[s] = alpha[col[s] * R2 + m0];
      b1[s] = alpha[col[s] * R2 + m1];
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      acc00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[s], b0[s], acc00, 0, 0, 0);
      acc01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[s], b1[s], acc01, 0, 0, 0);
      acc10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[s], b0[s], acc10, 0, 0, 0);
      acc11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[s], b1[s], acc11, 0, 0, 0);
    }
  }
  const int e0 = 32 * T + ka;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int e = e0 + 4 * i, f = e0 + 16 + 4 * i;
    if (e < c.b) {
      if (n0 < R2) y[(long)e * R2 + n0] = acc00[i];
      if (n1 < R2) y[(long)e * R2 + n1] = acc01[i];
    }
    if (f < c.b) {
      if (n0 < R2) y[(long)f * R2 + n0] = acc10[i];
      if (n1 < R2) y[(long)f * R2 + n1] = acc11[i];
    }
  }
}

void combine(const CombineMaps &c, const double2 *alpha, const double2 *U, const double2 *zs,
             const double2 *jw, double2 *y, int R, int mode, hipStream_t st) {
  static const bool lds16 = allow_lds((const void *)k_combine_tiled<16>, CLDS);
  static const bool lds8 = allow_lds((const void *)k_combine_tiled<8>, CLDS);
  static const bool lds4 = allow_lds((const void *)k_combine_tiled<4>, CLDS);
  // the choice does not depend on R, so a product gives the same result
  // however its right-hand sides are split
  const bool lds_ok = c.crc == 16 ? lds16 : c.crc == 8 ? lds8 : lds4;
  if ((mode & 2) && c.dn_tiles > 0 && c.near_dense) {
    // near part on the matrix cores into y, then far, Gram and coefficients
    const unsigned nb = (unsigned)c.dn_tiles * (unsigned)cdiv(R, DN_RHS);
    k_near_dense<<<nb, 256, 0, st>>>(c, (const double *)alpha, (double *)y, R);
    k_combine<<<cdiv((long)c.b * R, 256), 256, 0, st>>>(c, alpha, U, zs, jw, y, R, (mode & ~2) | 8);
    return;
  }
  if (c.ctile > 0 && c.comb_plan == 0 && (mode & 2) && lds_ok) {
    const unsigned nb = (unsigned)c.ctile * (unsigned)cdiv(R, c.crc);
    const size_t lds = (size_t)c.cmax * c.crc * sizeof(double2);
    if (c.crc == 16)
      k_combine_tiled<16><<<nb, c.ctr * 16, lds, st>>>(c, alpha, U, zs, jw, y, R, mode);
    else if (c.crc == 8)
      k_combine_tiled<8><<<nb, c.ctr * 8, lds, st>>>(c, alpha, U, zs, jw, y, R, mode);
    else
      k_combine_tiled<4><<<nb, c.ctr * 4, lds, st>>>(c, alpha, U, zs, jw, y, R, mode);
  } else {
    k_combine<<<cdiv((long)c.b * R, 256), 256, 0, st>>>(c, alpha, U, zs, jw, y, R, mode);
  }
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

// ===========================================================================
// post-processing (branch currents, voltages, centroid current, potentials)
// ===========================================================================
__global__ void k_post_branch(LoopMaps lm, PostOut o, const double2 *x, const double2 *alpha, const double2 *yb,
                              int R) {
  const int r = blockIdx.y, e = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = lm.b;
  if (e < b) {
    if (o.Ib) o.Ib[(size_t)r * (b + o.p) + e] = alpha[(size_t)e * R + r];
    if (o.Vb) o.Vb[(size_t)r * b + e] = yb[(size_t)e * R + r];
  } else if (e < b + o.p) {
    // a source branch is a link: its current is its own loop current
    if (o.Ib) o.Ib[(size_t)r * (b + o.p) + e] = x[(size_t)r * lm.l + o.port_loop[e - b]];
  }
}

// J(centroid) = sum_e s_e I_e (c - v_e) / (2A) = -sum_e s_e I_e (v_e - c) / (2A)
__global__ void k_post_tri(GridMaps g, PostOut o, const double2 *alpha, const double2 *pot, int nn, int R) {
  const int r = blockIdx.y, t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.n) return;
  if (o.J) {
    double dx[3] = {0, 0, 0}, dy[3] = {0, 0, 0};
    for (int i = 0; i < 3; ++i) {
      const double2 v = alpha[(size_t)g.tri_edge[3 * t + i] * R + r];
      const double s = g.tri_sign[3 * t + i];
      for (int c = 0; c < 3; ++c) {
        const double p = g.pl[9 * t + 3 * i + c];
        dx[c] += s * v.x * p;
        dy[c] += s * v.y * p;
      }
    }
    const double f = -g.inv2A[t];
    double2 *out = o.J + ((size_t)r * g.n + t) * 3;
    for (int c = 0; c < 3; ++c) out[c] = make_double2(dx[c] * f, dy[c] * f);
  }
  if (o.phi) {   // pot: [nn + 1][R]
    const double2 a = pot[(size_t)o.tri_pos[t] * R + r], z = pot[(size_t)o.tri_ref[t] * R + r];
    o.phi[(size_t)r * g.n + t] = make_double2(a.x - z.x, a.y - z.y);
  }
}

void post_outputs(const GridMaps &g, const LoopMaps &lm, const PostOut &o, const double2 *x, const double2 *alpha,
                  const double2 *yb, const double2 *pot, int R, hipStream_t st) {
  if (o.Ib || o.Vb) k_post_branch<<<dim3(cdiv(lm.b + o.p, 256), R), 256, 0, st>>>(lm, o, x, alpha, yb, R);
  if (o.J || o.phi) k_post_tri<<<dim3(cdiv(g.n, 256), R), 256, 0, st>>>(g, o, alpha, pot, lm.nn, R);
}

// explicit instantiations
template void tri_currents<float>(const GridMaps &, const double2 *, V2<float> *, int, hipStream_t);
template void tri_currents<double>(const GridMaps &, const double2 *, V2<double> *, int, hipStream_t);
template void project<float>(const GridMaps &, const V2<float> *, V2<float> *, int, hipStream_t);
template void project<double>(const GridMaps &, const V2<double> *, V2<double> *, int, hipStream_t);
template void convolve<float>(const GridMaps &, V2<float> *, V2<float> *, V2<float> *, int, hipStream_t, PassHook *);
template void convolve<double>(const GridMaps &, V2<double> *, V2<double> *, V2<double> *, int, hipStream_t, PassHook *);
template void interp_tri<double>(const GridMaps &, const V2<double> *, double2 *, int, hipStream_t, void *);
template void fold_spectrum<float>(const double2 *, float *, const int *, hipStream_t);
template void fold_spectrum<double>(const double2 *, double *, const int *, hipStream_t);

}  // namespace pfft
