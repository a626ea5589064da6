"""Mesh topology, modified RWG basis and its Gram matrix (oracle, FP64).

Conventions (paper Sec. II-C, Eqs. RWG and ExpandJ):

* Edge e joins two triangles; T+ is the lower triangle index, T- the other.
  Edges are numbered in lexicographic order of (lower vertex id, higher
  vertex id).
* Local edge i of triangle t is the edge opposite its vertex i, so that
  vertex is the free vertex of the basis function on t.
* On T+:  f_e(r) = (r - v+) / (2 A+);  on T-:  f_e(r) = (v- - r) / (2 A-).
  There is no edge-length factor, so the coefficient I_b is the current (A)
  crossing edge e from T+ to T-.  On triangle t the function is
  s (r - p_i) / (2 A_t) with s = +1 on T+ and -1 on T-.
"""
import numpy as np
import scipy.sparse as sp


class RWGMesh:
    def __init__(self, V, T):
        V = np.asarray(V, dtype=np.float64)
        T = np.asarray(T, dtype=np.int64)
        self.V, self.T = V, T
        n = T.shape[0]
        p0, p1, p2 = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
        cr = np.cross(p1 - p0, p2 - p0)
        self.area = 0.5 * np.linalg.norm(cr, axis=1)
        if np.any(self.area <= 0.0):
            raise ValueError("degenerate triangle")
        self.normal = cr / (2.0 * self.area[:, None])
        self.centroid = (p0 + p1 + p2) / 3.0
        owners = {}
        for t in range(n):
            for i in range(3):
                a, b = T[t, (i + 1) % 3], T[t, (i + 2) % 3]
                key = (a, b) if a < b else (b, a)
                owners.setdefault(key, []).append((t, i))
        keys = sorted(owners)
        self.nedge = len(keys)
        self.edge_vertices = np.array(keys, dtype=np.int64).reshape(-1, 2)
        self.tplus = np.empty(self.nedge, np.int64)
        self.tminus = np.empty(self.nedge, np.int64)
        self.tri_edge = np.empty((n, 3), np.int64)
        self.tri_sign = np.empty((n, 3), np.float64)
        for e, key in enumerate(keys):
            own = owners[key]
            if len(own) != 2:
                raise ValueError("edge %s shared by %d triangles" % (key, len(own)))
            (ta, ia), (tb, ib) = sorted(own)
            self.tplus[e], self.tminus[e] = ta, tb
            self.tri_edge[ta, ia], self.tri_sign[ta, ia] = e, 1.0
            self.tri_edge[tb, ib], self.tri_sign[tb, ib] = e, -1.0
        self.vplus = np.array([T[self.tplus[e]][list(self.tri_edge[self.tplus[e]]).index(e)]
                               for e in range(self.nedge)])
        self.vminus = np.array([T[self.tminus[e]][list(self.tri_edge[self.tminus[e]]).index(e)]
                                for e in range(self.nedge)])

    @property
    def ntri(self):
        return self.T.shape[0]

    def local_to_edge(self):
        """Sparse (3n x b) map C with C[3t+i, e(t,i)] = 1."""
        n = self.ntri
        rows = np.arange(3 * n)
        return sp.csr_matrix((np.ones(3 * n), (rows, self.tri_edge.reshape(-1))),
                             shape=(3 * n, self.nedge))

    def local_scale(self):
        """s_{t,i} / (2 A_t), the factor of the basis function on triangle t."""
        return self.tri_sign / (2.0 * self.area[:, None])

    def basis_at(self, e, r):
        """Value of f_e at points r (m x 3) lying on T+(e) or T-(e); used by
        tests to check the definition (Eq. RWG) point by point."""
        out = np.zeros_like(r)
        for t, s, v in ((self.tplus[e], 1.0, self.vplus[e]), (self.tminus[e], -1.0, self.vminus[e])):
            P = self.V[self.T[t]]
            lam = _barycentric(P, r)
            inside = np.all(lam >= -1e-12, axis=1)
            out[inside] = s * (r[inside] - self.V[v]) / (2.0 * self.area[t])
        return out


def _barycentric(P, r):
    a, b, c = P
    v0, v1, v2 = b - a, c - a, r - a
    d00, d01, d11 = v0 @ v0, v0 @ v1, v1 @ v1
    d20, d21 = v2 @ v0, v2 @ v1
    den = d00 * d11 - d01 * d01
    l1 = (d11 * d20 - d01 * d21) / den
    l2 = (d00 * d21 - d01 * d20) / den
    return np.stack([1 - l1 - l2, l1, l2], axis=1)


def gram_local(mesh):
    """Per-triangle 3x3 blocks  G_t[i, j] = int_t f_i . f_j dS  (the Z_s term
    of Eq. Zb, read as a same-point dot product).

    int_t (r - a).(r - b) dS = A [ (c - a).(c - b) + (1/12) sum_k |v_k - c|^2 ]
    with c the centroid (the cross terms vanish because int_t (r - c) = 0, and
    int_t |r - c|^2 = (A/36) (sum of squared side lengths))."""
    V, T = mesh.V, mesh.T
    P = V[T]                                   # (n, 3, 3)
    c = mesh.centroid
    A = mesh.area
    d = c[:, None, :] - P                      # c - p_i
    spread = np.sum((P - c[:, None, :]) ** 2, axis=(1, 2)) / 12.0
    raw = A[:, None, None] * (np.einsum('tik,tjk->tij', d, d) + spread[:, None, None])
    sc = mesh.local_scale()
    return raw * sc[:, :, None] * sc[:, None, :]


def gram_matrix(mesh, weight=None):
    """b x b sparse Gram matrix sum_t w_t G_t (w_t = surface impedance of
    triangle t; default 1)."""
    G = gram_local(mesh)
    if weight is not None:
        G = G * np.asarray(weight)[:, None, None]
    n = mesh.ntri
    rows = np.repeat(mesh.tri_edge, 3, axis=1).reshape(-1)
    cols = np.tile(mesh.tri_edge, (1, 3)).reshape(-1)
    M = sp.coo_matrix((G.reshape(-1), (rows, cols)), shape=(mesh.nedge, mesh.nedge))
    return M.tocsr()
