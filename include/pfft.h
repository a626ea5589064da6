/*
 * pfft.h -- C ABI of the MI355X (gfx950) pre-corrected-FFT loop-analysis
 * RL extractor.
 *
 * The library computes the magneto-quasi-static surface-integral-equation
 * model of Zhu, Chen & Yang ("An SIE Formulation with Triangular
 * Discretization and Loop Analysis for Parameter Extraction of Arbitrarily
 * Shaped Interconnects"): modified RWG currents on a closed triangle mesh
 * (Sec. II-C), the circuit graph and fundamental-loop basis (Sec. III), the
 * preconditioned GMRES solve (Sec. IV-A) with the pFFT matrix-vector product
 * (Sec. IV-B) and port R/L extraction (Sec. V).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units SI, time convention e^{j omega t}, mu = mu0 = 4 pi 1e-7 H/m.
 * Complex numbers are interleaved (re, im) IEEE doubles ("complex128").
 * Branch space: the b mesh edges, numbered in lexicographic order of
 *   (lower vertex id, higher vertex id); T+ of an edge is its lower triangle
 *   index; the coefficient is the current (A) from T+ to T- (Eq. RWG without
 *   the edge length).
 * Loop space: the l = b - n' + s + p fundamental loops (Eq. FinalME), one per
 *   link, links numbered in branch order (mesh edges, then one zero-impedance
 *   source branch per port, from the sink node to the source node).  Each
 *   contact face (a port's source or sink triangle set) is one node whose id
 *   is its lowest triangle index; the spanning tree is the breadth-first
 *   forest rooted at each conductor's lowest node id, neighbours visited in
 *   (neighbour id, branch id) order.
 * Device buffers are caller-owned and must stay valid until the stream has
 *   executed the call; host arrays are borrowed for the duration of the call.
 * Every entry point returns a pfft_status; on failure pfft_last_error()
 *   gives a thread-local message.  No exceptions cross the ABI.
 * Calls on one context are not thread-safe; use one context per thread.
 */
#ifndef PFFT_H
#define PFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pfft_ctx pfft_ctx; /* opaque; owns every internal device buffer */

typedef enum {
  PFFT_OK = 0,
  PFFT_EINVAL = -1,   /* bad argument (null pointer, size, option)             */
  PFFT_ETOPO = -2,    /* non-manifold edge, degenerate triangle, overlapping
                         contacts, port source/sink on different conductors   */
  PFFT_ENOMEM = -3,   /* device or host allocation failed                      */
  PFFT_EDEVICE = -4,  /* HIP runtime error                                     */
  PFFT_ENOCONV = -5,  /* GMRES reached maxit before the tolerance              */
  PFFT_EFACTOR = -6   /* zero pivot in the preconditioner factorization       */
} pfft_status;

/* Problem description (Sec. V: mesh, conductivity, ports, frequencies). */
typedef struct {
  int32_t nv;            /* vertices                                           */
  const double *V;       /* [nv][3] coordinates in metres (host)               */
  int32_t nt;            /* triangles                                          */
  const int32_t *T;      /* [nt][3] vertex ids, counter-clockwise seen from
                            outside (closed 2-manifold, host)                  */
  int32_t nport;         /* ports p (>= 0)                                     */
  const int32_t *src_off;/* [nport+1] CSR offsets into src_tri                 */
  const int32_t *src_tri;/* source-face triangle ids of each port              */
  const int32_t *snk_off;/* [nport+1] CSR offsets into snk_tri                 */
  const int32_t *snk_tri;/* sink-face triangle ids of each port                */
  double sigma;          /* conductivity (S/m), e.g. 5.8e7                     */
  double mu_r;           /* relative permeability (1.0)                        */
  int32_t grid[3];       /* pFFT grid nodes N_x, N_y, N_z (Sec. IV-B)          */
  int32_t stencil;       /* stencil order O_s (only 4 is supported)            */
  double near_kappa;     /* near-field radius in units of (O_s-1) max h (1.5)  */
  int32_t grid_fp64;     /* 1: grid convolution in FP64, 0: FP32 complex       */
  int32_t contact_zs;    /* 0: ideal contacts (Z_s = 0 on contact faces), 1: Z_s*/
  int32_t max_rhs_chunk; /* right-hand sides per grid pass; 0 = automatic      */
} pfft_problem;

/* Build a context: topology, loop basis, Gram blocks, grid and projection
 * weights, kernel spectrum, near-field pre-correction (Sec. II-IV).  The
 * near pairs' blocks (direct integral minus the grid's own interaction,
 * Eq. Lb) are computed on the current device, one thread per pair; lists
 * and the edge-level CSR are built on the host.  Work that needs the GPU
 * runs on hip_stream (a hipStream_t, may be NULL).  Device-side failures
 * return PFFT_EDEVICE (or PFFT_ENOMEM).  *out is owned by the caller and
 * released with pfft_destroy. */
pfft_status pfft_setup(const pfft_problem *pb, void *hip_stream, pfft_ctx **out);

/* out[0..9] = n, n', b, l, s, p, nnz of the near-field matrix, N_g,
 *             near triangle pairs, device bytes held by the context. */
pfft_status pfft_sizes(const pfft_ctx *c, int64_t out[10]);

/* Flags of pfft_matvec. */
#define PFFT_FAR_ONLY   1  /* only the grid term I H B (no near field)          */
#define PFFT_NEAR_ONLY  2  /* only the pre-corrected near field L_d              */
#define PFFT_PRECOND    4  /* loop space: return P^-1 (Z_l x) (Eqs. Precond,
                              LoopWithP)                                       */
#define PFFT_PRECOND_ONLY 8 /* loop space: return P^-1 x                         */
#define PFFT_LEARNED_ONLY 16 /* loop space: return M(x) = P^-1 x plus the learned
                              correction (P^-1 x when no network is loaded)   */

/* y = op(x) for nrhs right-hand sides (Eqs. CurT, Lb, VolT).
 * space 0: branch space, y = K x with K the pFFT approximation of the
 *          kernel matrix int int f_i . f_j / |r - r'| (no 1/(4 pi), no
 *          j omega mu); x, y are complex128 [nrhs][b]; omega unused.
 * space 1: loop space, y = Z_l(omega_r) x = A [Z_s(omega_r) G +
 *          (j omega_r mu / 4 pi) K] A^T x for right-hand side r; x, y are
 *          complex128 [nrhs][l]; omega is a host array [nrhs] (rad/s).
 * x_dev, y_dev: device pointers (must not alias); launched on hip_stream. */
pfft_status pfft_matvec(pfft_ctx *c, int32_t nrhs, const double *omega, int32_t space,
                        int32_t flags, const void *x_dev, void *y_dev, void *hip_stream);

/* pfft_matvec without any device allocation inside the call, for callers
 * that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, layouts and results as
 * pfft_matvec, except that the preconditioner flags (PRECOND, PRECOND_ONLY,
 * LEARNED_ONLY) are rejected with PFFT_EINVAL: they need per-frequency
 * factors.  The product's workspace is carved from a fixed 128 MiB scratch
 * array that the library holds on each GPU it runs on until the process
 * ends; right-hand sides are processed in chunks that fit it, and a problem
 * whose single right-hand side needs more returns PFFT_ENOMEM (message
 * states both sizes).  Every call on one GPU shares that GPU's scratch
 * (from every context): calls that overlap on one GPU race, so the caller
 * serialises them (one stream, or events).  Nothing in the scratch needs to
 * start at zero. */
pfft_status pfft_matvec_noalloc(pfft_ctx *c, int32_t nrhs, const double *omega, int32_t space,
                                int32_t flags, const void *x_dev, void *y_dev, void *hip_stream);

/* Solve A Z_b A^T I_l = V_l (Eq. FinalME) for every (frequency, port):
 * V_l = 1 V on the port's source loop, other ports shorted (Sec. V), with
 * right-preconditioned flexible GMRES (restart `restart`, x0 = 0, relative
 * true-residual tolerance tol).  precond: 0 none, 1 the paper's P = A Z_b^N A^T
 * (Eq. Precond), 2 P plus the learned correction loaded with
 * pfft_precond_load (falls back to 1 when none is loaded or it misbehaves).
 * Y_out: host complex128 [nfreq][nport][nport], Y[f][j][k] = I_l of port j's
 * loop when port k is driven.  iters_out, relres_out: host [nfreq][nport]
 * (may be NULL).  Returns PFFT_ENOCONV if some right-hand side missed tol
 * (outputs still written). */
pfft_status solve_ports(pfft_ctx *c, int32_t nfreq, const double *freq_hz, double tol,
                        int32_t maxit, int32_t restart, int32_t precond, void *Y_out,
                        int32_t *iters_out, double *relres_out, void *hip_stream);

/* The solver form of Sec. IV-A (Eq. LoopWithP): GMRES on the left-preconditioned
 * system P^-1 A Z_b A^T I_l = P^-1 V_l for every (frequency, port), restart
 * `restart`, x0 = 0.  tol applies to the preconditioned relative residual
 * |P^-1 (V_l - Z_l I_l)| / |P^-1 V_l| (the quantity left-preconditioned GMRES
 * minimises; Sec. V reports iteration counts at 1e-3), and relres_out
 * receives that quantity.  precond: 0 none (plain GMRES, the same iteration
 * as solve_ports with precond 0), 1 the paper's P; the learned correction
 * (2) is rejected with PFFT_EINVAL, since a left preconditioner must be a
 * fixed operator.  Arguments, layouts and errors otherwise as solve_ports. */
pfft_status solve_ports_lgmres(pfft_ctx *c, int32_t nfreq, const double *freq_hz, double tol,
                               int32_t maxit, int32_t restart, int32_t precond, void *Y_out,
                               int32_t *iters_out, double *relres_out, void *hip_stream);

/* solve_ports that also keeps the solution: Il_dev (device, caller-owned)
 * receives the loop currents I_l, complex128 [nfreq][nport][l] (row f*nport + k
 * is frequency f with port k driven at 1 V), for pfft_postprocess. */
pfft_status solve_ports_loops(pfft_ctx *c, int32_t nfreq, const double *freq_hz, double tol,
                              int32_t maxit, int32_t restart, int32_t precond, void *Y_out,
                              int32_t *iters_out, double *relres_out, void *Il_dev, void *hip_stream);

/* Post-processing of loop currents (Sec. V-A) for nrhs right-hand sides at
 * omega[nrhs] (host, rad/s).  Il_dev: device complex128 [nrhs][l] loop
 * currents.  Outputs (device, caller-owned, complex128, RHS-major; each may be
 * NULL):
 *   Vl_dev  [nrhs][l]    loop voltages Z_l I_l (Eq. LoopVandI; equal to the
 *                        excitation up to the solve's residual)
 *   Ib_dev  [nrhs][b+p]  branch currents A^T I_l (Eq. CurT): mesh edges in
 *                        edge order, then port k's source branch (sink face
 *                        to source face)
 *   Vb_dev  [nrhs][b]    mesh-branch voltages Z_b I_b (Eq. BranchVandI), the
 *                        T+ potential minus the T- potential (Eq. Vb)
 *   J_dev   [nrhs][n][3] surface current density at each triangle's centroid
 *                        (A/m), sum of I_e f_e (Eqs. ExpandJ, RWG)
 *   phi_dev [nrhs][n]    panel potentials (V): each conductor's reference
 *                        node (the sink face of its lowest-numbered port,
 *                        else its lowest triangle's node) at 0 V, every other
 *                        node by summing branch voltages along the spanning
 *                        tree; a contact face is one node.
 * Uses the same pFFT product as pfft_matvec (and its workspace). */
pfft_status pfft_postprocess(pfft_ctx *c, int32_t nrhs, const double *omega, const void *Il_dev,
                             void *Vl_dev, void *Ib_dev, void *Vb_dev, void *J_dev, void *phi_dev,
                             void *hip_stream);

/* Z = Y^-1, R = Re Z, L = Im Z / omega per frequency (Sec. V).  Y: host
 * complex128 [nfreq][nport][nport]; R_out, L_out: host [nfreq][nport][nport].
 * Pure host function; no context.  PFFT_EINVAL if some Y is singular. */
pfft_status extract_RL(int32_t nfreq, int32_t nport, const double *freq_hz, const void *Y,
                       double *R_out, double *L_out);

/* ---- Learned correction of the preconditioner (solve_ports precond = 2) ----
 * Not part of the paper: a per-loop network refines M(v) = P^-1 v inside
 * flexible GMRES (Sec. IV-A's P stays the fallback).  For a right-hand side
 * with loop vector v (length l) and z = P^-1 v, let s_v = sqrt(l)/|v|,
 * s_z = sqrt(l)/|z| (2-norms).  Loop i gets the features
 *   x_i = ( Re v_i s_v, Im v_i s_v, Re z_i s_z, Im z_i s_z,
 *           (log10 f - 8)/2, [i is a port source link], [i is a contact
 *           self-loop], Re D_e/|D_e| of its link branch e (0 for a port),
 *           a1_i, a2_i )
 * (D_e = Z_b(e,e) of Eq. Zb), where a1_i is the mean of (Re v_j s_v,
 * Im v_j s_v, Re z_j s_z, Im z_j s_z) over ring 1 of loop i (the other
 * loops whose link branch ends at one of the two end nodes of i's link
 * branch) and a2_i the same mean over ring 2 (loops whose link branch ends
 * at a node one branch away from those end nodes, not in ring 1; zeros for
 * an empty ring): 16 features, rounded to bf16, and the network
 *   y_i = W3 relu(W2 relu(W1 x_i + b1) + b2) + b3      (2 outputs)
 * gives M(v)_i = z_i + (y_i0 + j y_i1)/s_z.  If some y of a right-hand side
 * is not finite or sum_i |y_i|^2 > 16 l, that right-hand side keeps z.
 * The matrix products run on the matrix cores with bf16 operands and FP32
 * accumulation.  Inference stores activations as bf16; training keeps them
 * in FP32 and feeds each as a bf16 hi + lo pair (about 16 mantissa bits).
 *
 * Weight blob (little endian), exchanged by pfft_precond_load/_save:
 *   int32 magic 0x504D4C50, int32 F (= 16), int32 H (hidden width), int32 O (= 2)
 *   bf16 W1[H][F], W2[H][H], W3[O][H]   (row-major), zero-padded to 4 bytes
 *   float32 b1[H], b2[H], b3[O]
 * size = 16 + 4*ceil((H*F + H*H + O*H)/2) + 4*(2H + O) bytes.            */

/* Load weights (host blob, copied).  PFFT_EINVAL on a malformed blob. */
pfft_status pfft_precond_load(pfft_ctx *c, const void *blob, int64_t nbytes);

/* Copy the current weights into buf (host) when cap_bytes suffices; *nbytes
 * always receives the blob size.  PFFT_EINVAL when no network exists. */
pfft_status pfft_precond_save(pfft_ctx *c, void *buf, int64_t cap_bytes, int64_t *nbytes);

/* Training pairs from the solver itself: one cycle of plain-P FGMRES
 * (x0 = 0, no restart, at most maxit steps, tolerance tol) on every
 * (frequency, port).  Its Arnoldi relation Z_l z_k = sum_i H[i][k] v_i with
 * z_k = P^-1 v_k gives the exact errors e_k = Z_l^-1 v_k of the Krylov
 * vectors the preconditioner is applied to, by the backward recursion
 *   e_0 = x / |b|,   e_{k+1} = (z_k - sum_{i<=k} H[i][k] e_i) / H[k+1][k]
 * from the final iterate x; a pair is kept while |r_k| >= 1e3 |r_final|
 * (the error of x, amplified by the recursion, stays below ~1e-3).  Its rows
 * are the features of v = v_k and the targets t_i = (g e_i - z_i) s_z with
 * g = <z,z>/<z,e> (the component of g e along z equals z, so the target is
 * the change of direction that GMRES can use).  Rows are appended to the
 * context's training set; *rows_out (may be NULL) receives the set size.
 * Device memory: about 2 maxit nfreq p l complex128 for the Krylov basis. */
pfft_status pfft_learned_collect(pfft_ctx *c, int32_t nfreq, const double *freq_hz, double tol,
                                 int32_t maxit, int64_t *rows_out, void *hip_stream);

/* Adam (beta 0.9/0.999, eps 1e-8, step lr) on minibatches of `batch` rows
 * drawn uniformly (counter-based hash of seed, step, row) from the training
 * set.  Loss: mean over the collected right-hand sides of
 * sum_i |y_i - t_i|^2 / sum_i |t_i|^2, estimated per minibatch.  A network
 * of width `hidden` is initialised (seeded) when none exists.  loss_out:
 * host [steps] (may be NULL).  PFFT_EINVAL when the training set is empty. */
pfft_status pfft_learned_train(pfft_ctx *c, int32_t steps, int32_t batch, int32_t hidden, double lr,
                               uint64_t seed, float *loss_out, void *hip_stream);

/* Loss of the current network over the whole training set (the mean over
 * the collected right-hand sides of sum_i |y_i - t_i|^2 / sum_i |t_i|^2),
 * in training precision, into *loss_out (host).  PFFT_EINVAL when the set is
 * empty or no network exists. */
pfft_status pfft_learned_eval(pfft_ctx *c, double *loss_out, void *hip_stream);

/* Drops the training set (weights stay). */
pfft_status pfft_learned_clear(pfft_ctx *c);

/* Since the weights were loaded or initialised: out[0] = right-hand-side
 * applications of the network, out[1] = of those, numeric fallbacks to
 * P^-1, out[2] = right-hand sides that solve_ports switched back to plain P
 * because their residual fell more slowly over two steps than the plain
 * preconditioner's median per-step factor measured by pfft_learned_collect
 * (times 1.1; no switching when nothing was collected in this context). */
pfft_status pfft_learned_stats(pfft_ctx *c, int64_t out[3]);

/* Context-free evaluation of the network with gradients (training
 * precision), for checks:
 * X_dev bf16 [rows][F], T_dev, Y_dev float32 [rows][2], w_dev float32 [rows]
 * (device); loss = sum_i w_i |y_i - t_i|^2 (host double), grad_dev float32
 * device [H*F + H*H + 2*H + 2*H + 2] ordered W1, W2, W3, b1, b2, b3.  The
 * blob is a host pointer.  Allocates and frees its own scratch; synchronous. */
pfft_status pfft_mlp_grad(int32_t rows, const void *blob, int64_t nbytes, const void *X_dev,
                          const float *T_dev, const float *w_dev, float *Y_dev, float *grad_dev,
                          double *loss_out, void *hip_stream);

/* ---- Plans, graphs and the autotuner (batched execution of Sec. IV) ----
 * Options of a context (all 0 or 1; the results of every plan are the same
 * transform up to rounding):
 *   "fft_plan"     0 register-resident FFT passes where the grid shape allows
 *                    (FP32), 1 LDS Stockham passes
 *   "ldl_plan"     0 register-window band solve when both band widths are at
 *                    most 63, 1 LDS-window band solve
 *   "project_plan" 0 tiled projection (tile moments staged in LDS),
 *                  1 node-major gather
 *   "project_rhs"  tiled projection (FP32 grid): 0 (default) 16 right-hand
 *                    sides per workgroup, 1 eight (half the LDS staging per
 *                    workgroup, twice the workgroups; the sums are the same
 *                    bit for bit)
 *   "graphs"       1 solve_ports replays the product and P^-1 of each FGMRES
 *                    iteration as HIP graphs (after one eager iteration),
 *                  0 eager launches
 *   "stream_split" 1 the right-hand sides of a product (and of P^-1) are
 *                    split into two halves run on two streams of the
 *                    context (default priority), forked from and joined to
 *                    the caller's stream with events, so kernels of one half
 *                    can overlap those of the other (not while profiling);
 *                    0 (default) one stream
 *   "combine_plan" 0 near-field product over row tiles with the tile's
 *                    columns of x staged in LDS (when every tile's column list
 *                    fits), 1 per-nonzero gathers from memory
 *   "factor_plan"  0 (default) the LDL^T factors of the nodal matrix of P
 *                    (one per distinct frequency) are computed on the device,
 *                    one workgroup per conductor and frequency, when no
 *                    conductor carries more than 4 ports and the band window
 *                    fits in LDS (band width up to about 85), else on the
 *                    host; 1 always on the host (OpenMP over frequencies).
 *                    Changing it refactors at the next use of P.
 *   "fft_prune"    1 (default) with the register FFT passes, only the grid
 *                    nodes that some triangle's stencil touches enter and
 *                    leave the convolution (Eqs. Projection, Interpolation:
 *                    every other node of B is zero and no row of the
 *                    interpolation reads it): the X passes skip groups of 32
 *                    (y, z) grid lines without such a node, the forward X pass
 *                    reads and the inverse one writes only those nodes, the
 *                    (y, z) plane kernels read only the lines that hold
 *                    one (the small-plane kernel also writes only those),
 *                    and the tiled projection does not write
 *                    node chunks without a contribution; 0 dense passes.
 *                    The product is the same bit for bit.
 *   "near_dense"   1 (default) the near-field product runs over dense
 *                    32-row tiles on the FP64 matrix cores where the tiles
 *                    are at least half full, 0 the CSR paths of combine_plan
 *   "learned_judge_ppm" the learned correction's convergence judge: a
 *                    right-hand side whose residual falls by less than this
 *                    factor (parts per million) per step over two steps is
 *                    switched back to plain P; pfft_learned_collect sets it
 *                    (1.1 x the plain median factor), a caller may carry it
 *                    to another context; 0 disables switching.  Values in
 *                    [0, 1e6).
 * Read-only: "combine_tile_rows", "combine_tile_rhs" (the LDS row tile
 * chosen at setup, 0 when none fits), "precond_nd" (1 when the current
 * preconditioner uses nested dissection, -1 before the first use of P).
 * PFFT_EINVAL for an unknown name or value. */
pfft_status pfft_set_option(pfft_ctx *c, const char *name, int64_t value);
pfft_status pfft_get_option(pfft_ctx *c, const char *name, int64_t *value);

/* Times the preconditioned product P^-1 Z_l x (one FGMRES step) for nrhs
 * right-hand sides at omega[nrhs] (host, rad/s) for each value of fft_plan,
 * ldl_plan, project_plan, project_rhs, combine_plan, stream_split and
 * near_dense in turn (median of reps runs after one warm-up), keeps the
 * fastest value of each and writes a JSON report of the timings
 * (milliseconds) and choices into report[cap] (host, NUL-terminated, may be
 * NULL).  Allocates two nrhs x l complex128 device vectors for the run. */
pfft_status pfft_autotune(pfft_ctx *c, int32_t nrhs, const double *omega, int32_t reps, char *report,
                          int64_t cap, void *hip_stream);

void pfft_destroy(pfft_ctx *c);
const char *pfft_last_error(void);

/* Tracing: with profiling enabled, every stage of pfft_matvec records a pair
 * of HIP events on the caller's stream.  pfft_profile(c, on) clears the
 * totals; pfft_stage_times waits for the recorded events and returns the
 * summed milliseconds and launch counts per stage: 0 loop->branch (A^T),
 * 1 triangle currents, 2 projection, 3-7 the five FFT passes (X, Y, Z with
 * spectrum multiply, inverse Y, inverse X), 8 interpolation, 9 near field +
 * Gram combine, 10 branch->loop (A), 11 preconditioner; 12-15 unused. */
pfft_status pfft_profile(pfft_ctx *c, int32_t enable);
pfft_status pfft_stage_times(pfft_ctx *c, double ms[16], int64_t calls[16]);

/* Host-only inspection of the setup (no device work): builds the topology,
 * loop basis, Gram blocks, grid weights and near-field pre-correction of
 * pfft_setup and copies named arrays out.  Names (element type): "sizes"
 * (int64[10], as pfft_sizes), "links", "port_loop", "tplus", "tminus",
 * "node_of_tri", "parent", "parent_branch", "pre", "sub", "anchor" (int32),
 * "M0" [n][64], "M1" [n][64][3], "gram_val" [b][5], "near_val", "kdiag",
 * "grid" (double[9]: N, h, x0), "gram_col" [b][5], "near_col" (int32),
 * "near_rowptr" (int64[b+1]); the preconditioner's structure (built on
 * the host, Sec. IV-A): "precond_info" / "precond_info_nd" (int64[7]: nu, W,
 * Wc, nested dissection used, supernodes, largest front, levels; automatic
 * ordering / nested dissection forced) and "nd_check_1GHz" (double: relative
 * residual of a host supernodal solve of the nodal system at 1 GHz), and
 * "setup_ms" (double[8]: wall time of the set-up phases: topology, circuit,
 * Gram, grid, near lists, near pair blocks, near CSR, device build).
 * pfft_host_get writes *len_bytes always and copies when dst is non-null and
 * cap_bytes is large enough.  The host-only model computes the near-field
 * pair blocks (Sec. IV-B step 4, Eq. Lb) in a host loop; pfft_setup
 * computes them on the device with the same pair routine. */
typedef struct pfft_host_model pfft_host_model;
pfft_status pfft_host_setup(const pfft_problem *pb, pfft_host_model **out);
pfft_status pfft_host_get(const pfft_host_model *h, const char *name, void *dst, int64_t cap_bytes,
                          int64_t *len_bytes);
void pfft_host_free(pfft_host_model *h);
/* The same named arrays from a device context's host copy of its model
 * (after pfft_setup; its near-field values come from the device pair
 * blocks).  Same conventions and errors as pfft_host_get; the context owns
 * the data, dst is host memory of cap_bytes. */
pfft_status pfft_ctx_get(const pfft_ctx *c, const char *name, void *dst, int64_t cap_bytes, int64_t *len_bytes);

#ifdef __cplusplus
}
#endif
#endif
