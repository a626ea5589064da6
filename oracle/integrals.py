"""Triangle integrals of the static kernel 1/|r - r'| (oracle, FP64).

The dense kernel matrix of the first term of Eq. Zb (static Green's function,
Eq. StaticGF, with the 1/(4 pi) and j omega mu factors left outside):

    K_ee' = sum_{t in supp e, t' in supp e'} int_t int_t' f_e(r).f_e'(r') / |r - r'|

On triangle t, f_e = s (r - p_i)/(2 A_t), so every triangle pair needs the
3 x 3 raw block

    M_tt'[i, j] = int_t int_t' (r - p_i).(r' - q_j) / |r - r'| dS' dS .

Both surface integrals are done numerically (the C helper csrc/pairs.c):
  * pairs that share the whole triangle, an edge or a vertex: Sauter-Schwab
    regularised cubature (the 4-D domain cut into 6 / 5 / 2 pieces, each
    mapped from the unit hypercube with a Jacobian that cancels the 1/R
    singularity; tensor Gauss-Legendre of order ``ss_q`` per dimension);
  * all other pairs: tensor products of collapsed Gauss rules on both
    triangles, the order set by the separation ratio, after recursive
    midpoint subdivision of the larger piece while the pieces are closer
    than one radius.
No closed-form potential is used, so nothing here follows the library's own
near-field integration (closed-form inner potential, graded outer rule).
"""
import ctypes
import os
import numpy as np

_LIB = None


def _clib():
    """The oracle's C helper, compiled with gcc on first use if missing."""
    global _LIB
    if _LIB is None:
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_pairs.so")
        if not os.path.exists(path):
            from oracle import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        lib.oracle_blocks_touching.restype = None
        lib.oracle_blocks_touching.argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_long, ctypes.c_void_p]
        lib.oracle_blocks_separated.restype = None
        lib.oracle_blocks_separated.argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_int, ctypes.c_void_p]
        lib.oracle_gauss01.restype = None
        lib.oracle_gauss01.argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p]
        _LIB = lib
    return _LIB


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def blocks_touching(P, Q, kind, ss_q=8):
    """Raw blocks of touching pairs by Sauter-Schwab cubature.  P, Q (m,3,3):
    vertex rows ordered so that the shared vertices come first, in the same
    order on both triangles; kind (m,): 3 same triangle, 2 common edge,
    1 common vertex."""
    P, Q = _f64(P), _f64(Q)
    kind = np.ascontiguousarray(kind, dtype=np.int32)
    out = np.empty((P.shape[0], 3, 3))
    if P.shape[0]:
        _clib().oracle_blocks_touching(P.shape[0], P.ctypes.data, Q.ctypes.data, kind.ctypes.data,
                                       int(ss_q), out.ctypes.data)
    return out


def blocks_separated(P, Q, refine=False):
    """Raw blocks of pairs that share no vertex (adaptive product rules;
    refine=True integrates far more finely, to check the default)."""
    P, Q = _f64(P), _f64(Q)
    out = np.empty((P.shape[0], 3, 3))
    if P.shape[0]:
        _clib().oracle_blocks_separated(P.shape[0], P.ctypes.data, Q.ctypes.data, 1 if refine else 0,
                                        out.ctypes.data)
    return out


def gauss01(q):
    """The helper's Gauss-Legendre rule on [0, 1] (nodes, weights)."""
    x, w = np.empty(q), np.empty(q)
    _clib().oracle_gauss01(q, x.ctypes.data, w.ctypes.data)
    return x, w

# ---------------------------------------------------------------------------
# quadrature rules on the unit triangle (barycentric points, weights sum 1)
# ---------------------------------------------------------------------------

def conical_rule(q):
    """Collapsed-coordinate (Stroud conical product) Gauss rule with q x q
    points; exact for polynomials of total degree <= 2q - 2."""
    x, w = np.polynomial.legendre.leggauss(q)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    xi, eta = np.meshgrid(x, x, indexing="ij")
    wx, we = np.meshgrid(w, w, indexing="ij")
    l1 = xi.reshape(-1)
    l2 = (eta * (1.0 - xi)).reshape(-1)
    wt = 2.0 * (wx * we * (1.0 - xi)).reshape(-1)
    return np.stack([1.0 - l1 - l2, l1, l2], axis=1), wt


def dunavant7():
    """Symmetric 7-point rule of degree 5 (Dunavant 1985)."""
    a1, b1 = 0.059715871789770, 0.470142064105115
    a2, b2 = 0.797426985353087, 0.101286507323456
    w0, w1, w2 = 0.225, 0.132394152788506, 0.125939180544827
    pts = [(1 / 3, 1 / 3, 1 / 3),
           (a1, b1, b1), (b1, a1, b1), (b1, b1, a1),
           (a2, b2, b2), (b2, a2, b2), (b2, b2, a2)]
    return np.array(pts), np.array([w0] + [w1] * 3 + [w2] * 3)


def subdivide_rule(lam, w, levels):
    """Apply a rule on each of the 4^levels congruent sub-triangles."""
    tris = [np.eye(3)]
    for _ in range(levels):
        nxt = []
        for P in tris:
            m01, m12, m20 = (P[0] + P[1]) / 2, (P[1] + P[2]) / 2, (P[2] + P[0]) / 2
            nxt += [np.array([P[0], m01, m20]), np.array([m01, P[1], m12]),
                    np.array([m20, m12, P[2]]), np.array([m01, m12, m20])]
        tris = nxt
    pts = np.concatenate([lam @ P for P in tris])
    wts = np.concatenate([w / len(tris) for _ in tris])
    return pts, wts


# ---------------------------------------------------------------------------
# triangle-pair blocks
# ---------------------------------------------------------------------------

def classify_pairs(mesh, ti, tj):
    """Return (shared-vertex count, separation ratio) for triangle pairs.
    The ratio is (centroid distance - r_t - r_t') / r_t with r the
    circumscribing radius about the centroid."""
    Ti, Tj = mesh.T[ti], mesh.T[tj]
    shared = (Ti[:, :, None] == Tj[:, None, :]).any(axis=2).sum(axis=1)
    rad = np.max(np.linalg.norm(mesh.V[mesh.T] - mesh.centroid[:, None, :], axis=2), axis=1)
    d = np.linalg.norm(mesh.centroid[ti] - mesh.centroid[tj], axis=1)
    ratio = (d - rad[ti] - rad[tj]) / np.maximum(rad[ti], rad[tj])
    return shared, ratio


def touching_orders(Ti, Tj):
    """Vertex orders (perm_i, perm_j), each (m, 3), that put the vertices a
    touching pair shares first, in the same order on both triangles (the
    order they have in Ti), then the free ones in their original order."""
    isin = (Ti[:, :, None] == Tj[:, None, :]).any(axis=2)
    perm_i = np.argsort(~isin, axis=1, kind="stable")
    Tip = np.take_along_axis(Ti, perm_i, axis=1)
    match = Tj[:, :, None] == Tip[:, None, :]          # [k, c, a]: Tj[k, c] is the a-th shared vertex
    key = np.where(match.any(axis=2), match.argmax(axis=2), 3 + np.arange(3)[None, :])
    perm_j = np.argsort(key, axis=1, kind="stable")
    return perm_i, perm_j


def shape_quality(P):
    """Per triangle (rows of P, (m, 3, 3)): the aspect ratio (longest edge
    over the altitude onto it) and the largest interior angle in degrees."""
    e = np.stack([np.linalg.norm(P[:, (i + 1) % 3] - P[:, i], axis=1) for i in range(3)], axis=1)
    area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    L = e.max(axis=1)
    # largest angle, opposite the longest edge (law of cosines)
    es = np.sort(e, axis=1)
    cos_big = (es[:, 0] ** 2 + es[:, 1] ** 2 - es[:, 2] ** 2) / (2 * es[:, 0] * es[:, 1])
    return L * L / (2 * area), np.degrees(np.arccos(np.clip(cos_big, -1, 1)))


def touching_order(P, Q, kind, ss_q=None):
    """Gauss order per dimension for Sauter-Schwab on touching pairs.  The
    same-triangle case has its near-singular direction regularised (sinh
    rule) and converges fast for any shape; common-edge and common-vertex
    pairs converge more slowly when a triangle is thin or obtuse, so they
    take a higher order there (per-pair error below about 1e-9 of the block
    on the meshes used here, aspect <= 8, angles <= 150 degrees)."""
    if ss_q is not None:
        return np.full(P.shape[0], int(ss_q))
    ap, gp = shape_quality(P)
    aq, gq = shape_quality(Q)
    asp, ang = np.maximum(ap, aq), np.maximum(gp, gq)
    q = np.where((asp <= 3.0) & (ang <= 100.0), 10, np.where((asp <= 5.0) & (ang <= 120.0), 16, 24))
    return np.where(kind == 3, 8, q)


def pair_blocks(mesh, ti, tj, ss_q=None):
    """Raw blocks M_tt'[i, j] for the pairs (ti[k], tj[k]): touching pairs by
    Sauter-Schwab cubature (order from touching_order, or ss_q everywhere),
    the rest by the adaptive product rules of blocks_separated."""
    ti = np.asarray(ti, dtype=np.int64)
    tj = np.asarray(tj, dtype=np.int64)
    out = np.empty((ti.size, 3, 3))
    Ti, Tj = mesh.T[ti], mesh.T[tj]
    shared = (Ti[:, :, None] == Tj[:, None, :]).any(axis=2).sum(axis=1)
    P = mesh.V[mesh.T]
    touch = np.nonzero(shared > 0)[0]
    if touch.size:
        pi, pj = touching_orders(Ti[touch], Tj[touch])
        Pp = np.take_along_axis(P[ti[touch]], pi[:, :, None], axis=1)
        Qp = np.take_along_axis(P[tj[touch]], pj[:, :, None], axis=1)
        kind = shared[touch]
        q = touching_order(Pp, Qp, kind, ss_q)
        res = np.empty((touch.size, 3, 3))
        for qq in np.unique(q):
            sel = np.nonzero(q == qq)[0]
            res[sel] = blocks_touching(Pp[sel], Qp[sel], kind[sel], qq)
        # back to the original vertex order of both triangles
        blk = np.empty_like(res)
        rows = np.arange(touch.size)[:, None, None]
        blk[rows, pi[:, :, None], pj[:, None, :]] = res
        out[touch] = blk
    sep = np.nonzero(shared == 0)[0]
    if sep.size:
        out[sep] = blocks_separated(P[ti[sep]], P[tj[sep]])
    return out


def kernel_dense(mesh, rows_tri=None):
    """Dense b x b matrix K (no 1/(4 pi)).  Built from the local (3n x 3n)
    block matrix, scaled by s/(2A) on both sides and summed onto edges."""
    n = mesh.ntri
    sc = mesh.local_scale().reshape(-1)
    Kloc = np.empty((3 * n, 3 * n))
    tj_all = np.arange(n)
    step = max(1, 200000 // n)
    for t0 in range(0, n, step):
        ts = np.arange(t0, min(n, t0 + step))
        ti = np.repeat(ts, n)
        tj = np.tile(tj_all, ts.size)
        B = pair_blocks(mesh, ti, tj).reshape(ts.size, n, 3, 3)
        Kloc[3 * t0:3 * (t0 + ts.size)] = B.transpose(0, 2, 1, 3).reshape(3 * ts.size, 3 * n)
    Kloc *= sc[:, None] * sc[None, :]
    C = mesh.local_to_edge()
    K = np.asarray((C.T @ (C.T @ Kloc.T).T))
    # K is symmetric by definition; (t, t') and (t', t) were integrated with
    # different outer triangles, so average the two evaluations
    return 0.5 * (K + K.T)


def kernel_rows(mesh, edges):
    """Exact rows K[edges, :] computed one triangle pair at a time (for
    sampled checks on meshes too large for a dense K)."""
    edges = np.asarray(edges)
    n = mesh.ntri
    sc = mesh.local_scale()
    out = np.zeros((edges.size, mesh.nedge))
    for k, e in enumerate(edges):
        for t, s in ((mesh.tplus[e], 1.0), (mesh.tminus[e], -1.0)):
            i = list(mesh.tri_edge[t]).index(e)
            B = pair_blocks(mesh, np.full(n, t), np.arange(n))[:, i, :]
            vals = B * (s / (2.0 * mesh.area[t])) * sc
            np.add.at(out[k], mesh.tri_edge.reshape(-1), vals.reshape(-1))
    return out


def quadratic_form(mesh, coef_local, tris):
    """sum over t, t' in ``tris`` of int_t int_t' J_t(r).J_t'(r') / |r - r'|
    for per-triangle current J_t = sum_i coef_local[t, i] (r - p_i)/(2 A_t)
    (local coefficients include the sign).  Used for closed-form checks."""
    tris = np.asarray(tris)
    m = tris.size
    ti = np.repeat(tris, m)
    tj = np.tile(tris, m)
    B = pair_blocks(mesh, ti, tj)
    a = coef_local[ti] / (2.0 * mesh.area[ti])[:, None]
    b = coef_local[tj] / (2.0 * mesh.area[tj])[:, None]
    return float(np.einsum('ki,kij,kj->', a, B, b))
