// Device kernels of the pFFT loop-space matrix-vector product (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace pfft {

template <typename T> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };
template <typename T> using V2 = typename vec2<T>::type;

// ---- host launchers (all asynchronous on `st`) ----

// complex128 entries of the partial-sum scratch of a prefix scan down the
// columns of a [len][R] array
size_t scan_partials_size(int len, int R);

struct LoopMaps {
  // loop -> branch (A^T): injections per preorder position, per-branch read-out
  const int *inj_off, *inj_link;
  const int8_t *inj_sgn;
  const int *br_a, *br_lo, *br_hi;
  const int8_t *br_sg;
  // branch -> loop (A): per position, the signed twig voltages entering its
  // potential difference (code 2 e + (sign < 0)); link ends
  const int *dd_off, *dd_code;
  const int *link_branch, *link_upos, *link_vpos;
  int nn, b, l;
};

// x, yl: loop vectors [R][l]; alpha, yb: branch vectors RHS-contiguous [b][R];
// scan: [nn + 1][R] (after branch_to_loop it holds the node potentials);
// lT: scratch of l R complex128 values (the loop vector transposed).
void loop_to_branch(const LoopMaps &mp, const double2 *x, double2 *alpha, double2 *scan,
                    double2 *partials, double2 *lT, int R, hipStream_t st);
void branch_to_loop(const LoopMaps &mp, const double2 *yb, double2 *yl, double2 *scan,
                    double2 *partials, double2 *lT, int R, hipStream_t st);
// out[c][r] = in[r][c] (complex128)
void transpose(const double2 *in, double2 *out, int rows, int cols, hipStream_t st);


constexpr int INTERP_GROUP = 2;

struct GridMaps {
  int n, b, N, dims[3];
  const int *tri_edge;
  const int8_t *tri_sign;
  const double *inv2A;   // [n] 1/(2A)
  const double *pl;      // [n][3][3] vertex - centroid
  const int *anchor;     // [n][3]
  const int *pg_off;     // [N+1] node-major projection lists
  const int *pg_tri;
  const void *pg_w;      // [nnz][4] (M0, M1x, M1y, M1z) in T
  const void *tri_w;     // [n][64][4] same weights, triangle-major, in T
  const double *tri_wd;  // the same in FP64 (the grouped interpolation's scalar weights)
  const void *ghat;      // [(Nx+1)(Ny+1)(Nz+1)] real spectrum in T
  // projection tiles of tile[0] x tile[1] x tile[2] nodes (z fastest):
  // triangles whose stencil meets tile T are tt_tri[tt_off[T] .. tt_off[T+1])
  // (ascending); pg_loc[q] = position of pg_tri[q] in its node's tile list;
  // the first tcap triangles of a tile are staged in LDS
  int tile[3], ntile[3], tcap;
  int proj_rhs;          // tiled projection (FP32): 0 16 right-hand sides per workgroup, 1 eight
  const int *tt_off, *tt_tri, *pg_loc;
  // per tile, its local node indices with the most contributions first, so
  // the nodes of one wavefront have similar gather lengths
  const uint16_t *tn_perm;
  // the same gathers sliced per (tile, wavefront of that order): slice s
  // holds ps_k[s] entries per lane stored k-major from ps_off[s] (entry
  // ps_off[s] + 64 k + lane), so a wavefront's index and weight loads are
  // contiguous.  An entry is the triangle's LDS slot (>= 0) or -1 - triangle
  // (beyond tcap, read from memory); shorter lists are padded with slot 0
  // and zero weights.
  // active nodes (touched by some triangle's stencil): act[a] is the a-th in
  // ascending order, act_of[node] its position (-1 for the others)
  int nact;
  const int *act, *act_of;
  // interpolation groups: triangles with the same anchor, at most
  // INTERP_GROUP a group; group q = ig_tri[ig_off[q] .. ig_off[q+1])
  int nig;
  const int *ig_off, *ig_tri;
  const int *ig_act;     // [nig][64] active-node positions of each group's stencil nodes
  int nwave;
  const int *ps_off, *ps_k, *ps_ent;
  const void *ps_w;      // [entries][4] (M0, M1x, M1y, M1z) in T
  // plan choices (set by the context's options or the autotuner):
  // fft_plan 0 register-resident passes where the shape allows, 1 LDS
  // Stockham passes; proj_plan 0 tiled (LDS-staged), 1 node-major gather
  int fft_plan, proj_plan;
  // Pruned register FFT passes (prune = 1): only the active nodes feed the
  // convolution and only they are read from it, so the X passes skip every
  // group of 32 (y, z) columns without an active node, the forward X pass
  // reads only active nodes, the inverse one writes only those, and the
  // plane kernel reads only the columns that hold an active node.
  // xmask[c (Nx / 32) + w] bit b: node (x = 32 w + b, column c = y Nz + z)
  // active; cgrp[k]: columns [32 k, 32 k + 32) hold an active node;
  // zmask[z] bit y: column (y, z) holds one (Ny <= 64); colact[c / 32] bit
  // c % 32: column c holds one (any Ny).  Null where the grid shape does not
  // allow it.
  const uint32_t *xmask;
  const uint64_t *zmask;
  const uint8_t *cgrp;
  const uint32_t *colact;
  int prune;
  // twiddles of the register X passes (FP32 grid), k2 the 2-bit reversal of
  // q, m < Nx / 4: forward xtw[4 h + q][m] = (-1)^q W_{2Nx}^{(2 k2 + h) m};
  // inverse (from xtw + 2 Nx) (-1)^q W_{2Nx}^{-(2 k2 m + h k2)} / (2 Nx)
  const float2 *xtw;
};

// alpha [b][R] -> J [n][R][4]
template <typename T>
void tri_currents(const GridMaps &g, const double2 *alpha, V2<T> *J, int R, hipStream_t st);
template <typename T>
void project(const GridMaps &g, const V2<T> *J, V2<T> *Q, int R, hipStream_t st);
// Called between the five FFT passes (stage numbers 3..7) for timing.
struct PassHook {
  virtual void pass(int k, hipStream_t st) = 0;
  virtual void done(hipStream_t st) = 0;
};
template <typename T>
void convolve(const GridMaps &g, V2<T> *Q, V2<T> *T1, V2<T> *T2, int R, hipStream_t st,
              PassHook *hook = nullptr);
// phi [R][3][N] -> U [n][R][4]; scratch: N * 3R complex values of T that
// the FP32 path uses for a node-major copy of phi
template <typename T>
void interp_tri(const GridMaps &g, const V2<T> *phi, double2 *U, int R, hipStream_t st, void *scratch);
template <>
void interp_tri<float>(const GridMaps &g, const float2 *phi, double2 *U, int R, hipStream_t st, void *scratch);

// Whether convolve needs its T2 argument (12 N values a right-hand side).
bool convolve_uses_t2(const GridMaps &g, int fp64);
// Full-length forward 3-D FFT of a (2Nx, 2Ny, 2Nz) complex128 array in place.
void fft3_full_fp64(double2 *data, const int dims2[3], hipStream_t st);
template <typename T>
void fold_spectrum(const double2 *full, T *ghat, const int dims[3], hipStream_t st);

struct CombineMaps {
  int b, n;
  const int *efar_t;        // [b][2] triangles T+, T-
  const double *efar_s;     // [b][2] s / (2A)
  const double *efar_pl;    // [b][2][3] free vertex - centroid
  const int64_t *nf_rowptr;
  const int *nf_col;
  const double *nf_val;
  const int *gram_col;      // [b][5]
  const double *gram_val;
  // Row tiles of the near-field matrix for the LDS-staged product: rows
  // [T ctr, (T+1) ctr) read only the columns ct_col[ct_off[T] .. ct_off[T+1])
  // (ascending), nf_slot[q] is nf_col[q]'s position in its tile's list and
  // no list is longer than cmax.  ctile = 0: no tiles (gather only).
  int ctr, ctile, cmax, crc;   // crc: right-hand sides per workgroup (4, 8 or 16)
  const int *ct_off, *ct_col;
  const uint16_t *nf_slot;
  int comb_plan;            // 0 tiled product when available, 1 gather
  // Dense row tiles of the near-field matrix for the FP64 matrix-core
  // product: tile T covers rows [32 T, 32 T + 32) and the columns
  // dn_col[dn_off[T] .. dn_off[T+1]) (ascending, padded with zero values to
  // a multiple of 4); its values are dn_val[32 dn_off[T] ..] in k-major
  // quads: entry (row, k) at 32 dn_off[T] + ((k / 4) 32 + row) 4 + k % 4.
  // dn_tiles = 0: not built (tiles too sparse).  near_dense 1: use them.
  int dn_tiles, near_dense;
  const int64_t *dn_off;
  const int *dn_col;
  const double *dn_val;
};

// y[e][r] = zs[r] * (G a)[e] + jw[r] * (far[e] + (L_d a)[e]); far from U;
// alpha, y RHS-contiguous [b][R], U [n][R][4].
// mode bits: 1 far, 2 near, 4 gram (zs, jw ignored when gram bit is clear
// and kscale = 1: y = far + near).  With dense near-field tiles (dn_tiles >
// 0, near_dense 1) the near part is a matrix-core product written to y
// first and read back by the combining kernel.
void combine(const CombineMaps &c, const double2 *alpha, const double2 *U, const double2 *zs,
             const double2 *jw, double2 *y, int R, int mode, hipStream_t st);
// Longest column list of a near-field row tile that the tiled product can
// stage in LDS with rc (8 or 16) right-hand sides per workgroup.
int combine_tile_cap(int rc);

// Post-processing outputs of solved loop currents (any pointer may be null),
// RHS-major: Ib [R][b+p] branch currents (mesh branches, then the port
// source branches), Vb [R][b] branch voltages, J [R][n][3] surface current
// density at the triangle centroids, phi [R][n] panel potentials.
struct PostOut {
  double2 *Ib, *Vb, *J, *phi;
  int p;
  const int *port_loop;   // [p] loop of each port's source branch
  const int *tri_pos;     // [n] preorder position of the triangle's node
  const int *tri_ref;     // [n] preorder position of its conductor's reference node
};
// x: loop currents [R][l]; alpha, yb: [b][R]; pot: [R][nn+1] node potentials
// (prefix scan of the twig drops, any constant per conductor)
void post_outputs(const GridMaps &g, const LoopMaps &lm, const PostOut &o, const double2 *x, const double2 *alpha,
                  const double2 *yb, const double2 *pot, int R, hipStream_t st);

}  // namespace pfft
