// Host-side model built by pfft_setup: mesh topology, circuit graph and loop
// basis, Gram blocks, pFFT grid weights and the near-field pre-correction.
// Everything here is FP64/int and lives in host memory until uploaded.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace pfft {

struct SetupError {
  int code;
  std::string msg;
};

struct HostModel {
  // ---- mesh (Sec. II-B/C) ----
  int nv = 0, n = 0, b = 0, p = 0;
  std::vector<double> V;          // [nv][3]
  std::vector<int> T;             // [n][3]
  std::vector<double> area;       // [n]
  std::vector<double> cen;        // [n][3]
  std::vector<int> tri_edge;      // [n][3] edge opposite local vertex i
  std::vector<int8_t> tri_sign;   // [n][3] +1 on T+, -1 on T-
  std::vector<int> tplus, tminus; // [b]
  // ---- circuit graph and loops (Sec. III) ----
  int nn = 0;                     // n' nodes
  int s = 0;                      // conductors
  int l = 0;                      // loops = links
  std::vector<uint8_t> contact;   // [n]
  std::vector<int> node_of_tri;   // [n] compact node index
  std::vector<int> bu, bv;        // [b+p] branch end nodes (compact)
  std::vector<uint8_t> twig;      // [b+p]
  std::vector<int> links;         // [l] branch id of each link
  std::vector<int> port_loop;     // [p]
  std::vector<int> parent, parent_branch; // [nn] (-1 at roots)
  std::vector<int> pre, sub;      // [nn] preorder position and subtree size
  std::vector<int> order;         // [nn] node at preorder position
  // ---- Gram (second term of Eq. Zb) ----
  std::vector<double> gram;       // [n][3][3] scaled blocks int f_i . f_j
  std::vector<int> gram_col;      // [b][5]
  std::vector<double> gram_val;   // [b][5] (contact faces weighted 0 or 1)
  // ---- grid (Sec. IV-B) ----
  int dims[3] = {0, 0, 0};
  double h[3] = {0, 0, 0}, x0[3] = {0, 0, 0};
  std::vector<int> anchor;        // [n][3]
  std::vector<double> M0;         // [n][64]
  std::vector<double> M1;         // [n][64][3]
  std::vector<double> pl;         // [n][3][3] vertex - centroid
  // ---- near field ----
  std::vector<int> near_off;      // [n+1] ordered near lists incl. self
  std::vector<int> near_tri;
  int64_t npairs = 0;             // unordered near pairs incl. self
  std::vector<int64_t> nf_rowptr; // [b+1]
  std::vector<int> nf_col;
  std::vector<double> nf_val;
  // ---- diagonal of K for the preconditioner ----
  std::vector<double> kdiag;      // [b]
  // ---- wall time of the set-up phases, ms: topology, circuit, Gram, grid,
  // near lists, near blocks, near CSR (incl. diag K), device build (kernel
  // spectrum, product maps; device contexts only) ----
  double setup_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

struct SetupOptions {
  int grid[3];
  int stencil;
  double kappa;
  int contact_zs;
  int device_blocks = 0;          // near-field pair blocks on the current device
  void *stream = nullptr;         // (hipStream_t) for that work
};

// Unordered near pairs (t <= u) sorted by the class of t's outer rule (0:
// the pair touches; 1, 2, 3: separated, 7-point rule on 64, 16, 4
// sub-triangles); idx is the pair's position in the t-major order.
struct NearPairList {
  std::vector<int> t, u;
  std::vector<int64_t> idx;
  int64_t cls_end[4] = {0, 0, 0, 0};
};

// Builds everything except the kernel spectrum (computed on the device).
// Throws SetupError.
void build_model(HostModel &m, const double *V, int nv, const int *T, int n, int nport,
                 const int *src_off, const int *src_tri, const int *snk_off,
                 const int *snk_tri, const SetupOptions &opt);

// Host checks of the preconditioner's ordering and factorization (no
// device work): structure sizes [nu, W, Wc, nd, supernodes, largest front,
// levels] for nd_mode (0 automatic, 1 nested dissection), and the relative
// residual |L_w x - b| / |b| of a supernodal solve (host mirror of the
// device sweeps) with the nested-dissection factors at omega, for a fixed
// right-hand side.
std::vector<int64_t> precond_info(const HostModel &m, int nd_mode);
// The model's arrays by name: bytes (copied into dst when cap allows), or
// -1 for an unknown name.
int64_t model_get(const HostModel &m, const std::string &name, void *dst, int64_t cap);
double nd_solve_check(const HostModel &m, double omega);

// Scaled (direct - grid) blocks of every pair into blk[9 * idx] and the
// scaled direct blocks of the touching pairs (class 0, in list order) into
// dirb, on the current device (stream) or in a host loop.  Throws SetupError.
void near_pair_blocks(const HostModel &m, const NearPairList &pl, const std::vector<double> &Htab,
                      const int Dm[3], const int S[3], bool device, void *stream, double *blk, double *dirb);

}  // namespace pfft
