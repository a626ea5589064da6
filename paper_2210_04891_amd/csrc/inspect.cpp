// Host-only inspection of the setup model (no device work).
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "../../include/pfft.h"
#include "model.h"

namespace pfft {
void set_error(const std::string &msg);
}

using namespace pfft;

struct pfft_host_model {
  HostModel m;
};

template <typename V>
static int64_t put(const std::vector<V> &v, void *dst, int64_t cap) {
  int64_t bytes = (int64_t)(v.size() * sizeof(V));
  if (dst && cap >= bytes && bytes > 0) std::memcpy(dst, v.data(), bytes);
  return bytes;
}

namespace pfft {
// The model's arrays by name (bytes written, or -1 for an unknown name);
// shared by the host-only model and a device context's host copy.
int64_t model_get(const HostModel &m, const std::string &k, void *dst, int64_t cap) {
  int64_t n = -1;
  if (k == "links") n = put(m.links, dst, cap);
  else if (k == "port_loop") n = put(m.port_loop, dst, cap);
  else if (k == "tplus") n = put(m.tplus, dst, cap);
  else if (k == "tminus") n = put(m.tminus, dst, cap);
  else if (k == "node_of_tri") n = put(m.node_of_tri, dst, cap);
  else if (k == "parent") n = put(m.parent, dst, cap);
  else if (k == "parent_branch") n = put(m.parent_branch, dst, cap);
  else if (k == "pre") n = put(m.pre, dst, cap);
  else if (k == "sub") n = put(m.sub, dst, cap);
  else if (k == "anchor") n = put(m.anchor, dst, cap);
  else if (k == "M0") n = put(m.M0, dst, cap);
  else if (k == "M1") n = put(m.M1, dst, cap);
  else if (k == "gram_col") n = put(m.gram_col, dst, cap);
  else if (k == "gram_val") n = put(m.gram_val, dst, cap);
  else if (k == "near_rowptr") n = put(m.nf_rowptr, dst, cap);
  else if (k == "near_col") n = put(m.nf_col, dst, cap);
  else if (k == "near_val") n = put(m.nf_val, dst, cap);
  else if (k == "kdiag") n = put(m.kdiag, dst, cap);
  else if (k == "setup_ms") n = put(std::vector<double>(m.setup_ms, m.setup_ms + 8), dst, cap);
  else if (k == "grid") {
    std::vector<double> g = {(double)m.dims[0], (double)m.dims[1], (double)m.dims[2], m.h[0], m.h[1], m.h[2],
                             m.x0[0], m.x0[1], m.x0[2]};
    n = put(g, dst, cap);
  } else if (k == "precond_info" || k == "precond_info_nd") {
    n = put(precond_info(m, k == "precond_info_nd" ? 1 : 0), dst, cap);
  } else if (k == "nd_check_1GHz") {
    std::vector<double> v = {nd_solve_check(m, 2 * M_PI * 1e9)};
    n = put(v, dst, cap);
  } else if (k == "sizes") {
    std::vector<int64_t> sz = {m.n, m.nn, m.b, m.l, m.s, m.p,
                               m.nf_rowptr.empty() ? 0 : m.nf_rowptr.back(),
                               (int64_t)m.dims[0] * m.dims[1] * m.dims[2], m.npairs, 0};
    n = put(sz, dst, cap);
  }
  return n;
}
}  // namespace pfft

extern "C" {

pfft_status pfft_host_setup(const pfft_problem *pb, pfft_host_model **out) {
  if (!pb || !out) {
    set_error("pfft_host_setup: null argument");
    return PFFT_EINVAL;
  }
  *out = nullptr;
  pfft_host_model *h = nullptr;
  try {
    h = new pfft_host_model();
    SetupOptions opt;
    for (int d = 0; d < 3; ++d) opt.grid[d] = pb->grid[d];
    opt.stencil = pb->stencil;
    opt.kappa = pb->near_kappa;
    opt.contact_zs = pb->contact_zs;
    build_model(h->m, pb->V, pb->nv, pb->T, pb->nt, pb->nport, pb->src_off, pb->src_tri, pb->snk_off,
                pb->snk_tri, opt);
    *out = h;
    return PFFT_OK;
  } catch (const SetupError &e) {
    set_error("pfft_host_setup: " + e.msg);
    delete h;
    return (pfft_status)e.code;
  } catch (const std::bad_alloc &) {
    set_error("pfft_host_setup: host allocation failed");
    delete h;
    return PFFT_ENOMEM;
  }
}

pfft_status pfft_host_get(const pfft_host_model *h, const char *name, void *dst, int64_t cap_bytes,
                          int64_t *len_bytes) {
  if (!h || !name || !len_bytes) {
    set_error("pfft_host_get: null argument");
    return PFFT_EINVAL;
  }
  std::string k(name);
  int64_t n = -1;
  try {
    n = model_get(h->m, k, dst, cap_bytes);
  } catch (const SetupError &e) {
    set_error("pfft_host_get: " + e.msg);
    return (pfft_status)e.code;
  }
  if (n < 0) {
    set_error("pfft_host_get: unknown array " + k);
    return PFFT_EINVAL;
  }
  *len_bytes = n;
  if (dst && cap_bytes < n) {
    set_error("pfft_host_get: buffer too small");
    return PFFT_EINVAL;
  }
  return PFFT_OK;
}

void pfft_host_free(pfft_host_model *h) { delete h; }

}  // extern "C"
