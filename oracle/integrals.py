"""Triangle integrals of the static kernel 1/|r - r'| (oracle, FP64).

The dense kernel matrix of the first term of Eq. Zb (static Green's function,
Eq. StaticGF, with the 1/(4 pi) and j omega mu factors left outside):

    K_ee' = sum_{t in supp e, t' in supp e'} int_t int_t' f_e(r).f_e'(r') / |r - r'|

On triangle t, f_e = s (r - p_i)/(2 A_t), so every triangle pair needs the
3 x 3 raw block

    M_tt'[i, j] = int_t int_t' (r - p_i).(r' - q_j) / |r - r'| dS' dS .

Method (chosen to be exact in the inner integral):
  * inner integral over t' in closed form: with V0(r) = int_t' 1/R dS' and
    V1(r) = int_t' (r' - r)/R dS' (classical flat-triangle potential formulas,
    derived from the surface gradient theorem), the inner factor is
    V1(r) + (r - q_j) V0(r);
  * outer integral over t by Gauss rules whose order grows as the pair gets
    closer; pairs that share a vertex, an edge or the whole triangle use a
    rule graded toward the edges of t, where the outer integrand is only
    continuous (t log t behaviour);
  * well-separated pairs use a plain product rule on both triangles.
"""
import ctypes
import os
import numpy as np

_LIB = None


def _clib():
    """The oracle's own C helper (same algorithm, compiled with gcc), or None
    when it has not been built; the numpy code below is then used."""
    global _LIB
    if _LIB is None:
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_pairs.so")
        if os.path.exists(path):
            lib = ctypes.CDLL(path)
            for name in ("oracle_blocks_analytic", "oracle_blocks_product"):
                fn = getattr(lib, name)
                fn.restype = None
                fn.argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_long,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
            _LIB = lib
        else:
            _LIB = False
    return _LIB or None


def _c_blocks(name, P, Q, rule):
    lib = _clib()
    lam, w = rule
    P = np.ascontiguousarray(P, dtype=np.float64)
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    out = np.empty((P.shape[0], 3, 3))
    getattr(lib, name)(P.shape[0], P.ctypes.data, Q.ctypes.data, lam.shape[0],
                       lam.ctypes.data, w.ctypes.data, out.ctypes.data)
    return out


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


def graded_rule(q, p=2):
    """Rule on the unit triangle that clusters points toward all three edges
    and vertices: the triangle is cut into three pieces from its centroid,
    each piece is parametrised by (s along the base edge, u toward the
    centroid), u = v^p and s = S(sigma) with S a symmetric polynomial grading,
    and Gauss-Legendre is used in (sigma, v)."""
    x, w = np.polynomial.legendre.leggauss(q)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    # u = v^p, du = p v^(p-1) dv
    u = x ** p
    wu = w * p * x ** (p - 1)
    # s = sigma^p / (sigma^p + (1 - sigma)^p)
    a, b = x ** p, (1.0 - x) ** p
    s = a / (a + b)
    ds = p * x ** (p - 1) * (1.0 - x) ** (p - 1) / (a + b) ** 2
    ws = w * ds
    S, U = np.meshgrid(s, u, indexing="ij")
    WS, WU = np.meshgrid(ws, wu, indexing="ij")
    S, U, W = S.reshape(-1), U.reshape(-1), (WS * WU).reshape(-1)
    cen = np.array([1 / 3, 1 / 3, 1 / 3])
    pts, wts = [], []
    eye = np.eye(3)
    for k in range(3):
        B0, B1 = eye[k], eye[(k + 1) % 3]
        base = B0[None, :] + S[:, None] * (B1 - B0)[None, :]
        lam = (1.0 - U)[:, None] * base + U[:, None] * cen[None, :]
        # dA = 2 A_sub (1 - u) ds du; each piece has area 1/3 of the triangle
        pts.append(lam)
        wts.append(2.0 * (1.0 / 3.0) * (1.0 - U) * W)
    return np.concatenate(pts), np.concatenate(wts)


def _graded_1d(q, p, both_ends):
    x, w = np.polynomial.legendre.leggauss(q)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    if both_ends:
        a, b = x ** p, (1.0 - x) ** p
        return a / (a + b), w * p * x ** (p - 1) * (1.0 - x) ** (p - 1) / (a + b) ** 2
    return x ** p, w * p * x ** (p - 1)


def vertex_rule(q, p=2):
    """Duffy rule from vertex 0: r = p0 + u((1 - s)(p1 - p0) + s (p2 - p0)),
    dA = 2 A u du ds, u graded toward the vertex (u = v^p); the r log r
    behaviour of the outer integrand at a shared vertex becomes smooth."""
    u, wu = _graded_1d(q, p, False)
    s, ws = _graded_1d(q, 1, False)
    U, S = np.meshgrid(u, s, indexing="ij")
    W = np.outer(wu, ws)
    lam = np.stack([1.0 - U, U * (1.0 - S), U * S], axis=-1).reshape(-1, 3)
    return lam, (2.0 * U * W).reshape(-1)


def edge_rule(q, p=2):
    """Rule graded toward the edge p0-p1: r = (1 - u)(p0 + s (p1 - p0)) + u p2,
    dA = 2 A (1 - u) du ds, u = v^p graded toward the edge."""
    u, wu = _graded_1d(q, p, False)
    s, ws = _graded_1d(q, 1, False)
    U, S = np.meshgrid(u, s, indexing="ij")
    W = np.outer(wu, ws)
    lam = np.stack([(1.0 - U) * (1.0 - S), (1.0 - U) * S, U], axis=-1).reshape(-1, 3)
    return lam, (2.0 * (1.0 - U) * W).reshape(-1)


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
# closed-form potential integrals of a flat triangle
# ---------------------------------------------------------------------------

def potentials(r, Q):
    """For observation points r (m x 3) and triangles Q (m x 3 x 3, vertex
    rows) return V0 = int_T 1/R dS' (m,) and V1 = int_T (r' - r)/R dS' (m, 3).

    With n the unit normal, w0 the signed height of r above the plane and
    rho its projection, for each edge i (from q_i to q_i+1, in-plane outward
    normal u_i = l_i x n):
      t0 = (q_i - rho).u_i, s+- = (q_i+1 / q_i - rho).l_i, R0^2 = t0^2 + w0^2,
      f_i = ln((R+ + s+)/(R- + s-)),
      beta_i = atan(t0 s+/(R0^2 + |w0| R+)) - atan(t0 s-/(R0^2 + |w0| R-));
      V0 = sum_i (t0 f_i - |w0| beta_i);
      int_T (rho' - rho)/R = sum_i u_i (R0^2 f_i + s+ R+ - s- R-)/2,
    the last from int_T grad'_s R dS' = sum over edges of u_i int R dl'."""
    q0, q1, q2 = Q[:, 0], Q[:, 1], Q[:, 2]
    nrm = np.cross(q1 - q0, q2 - q0)
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    w0 = np.einsum('ij,ij->i', r - q0, nrm)
    rho = r - w0[:, None] * nrm
    aw = np.abs(w0)
    V0 = np.zeros(r.shape[0])
    Vr = np.zeros_like(r)
    for i in range(3):
        qa, qb = Q[:, i], Q[:, (i + 1) % 3]
        L = qb - qa
        ln_ = np.linalg.norm(L, axis=1)
        l = L / ln_[:, None]
        u = np.cross(l, nrm)
        t0 = np.einsum('ij,ij->i', qa - rho, u)
        sm = np.einsum('ij,ij->i', qa - rho, l)
        sp_ = sm + ln_
        R02 = t0 * t0 + w0 * w0
        Rm = np.sqrt(R02 + sm * sm)
        Rp = np.sqrt(R02 + sp_ * sp_)
        # ln((Rp + sp)/(Rm + sm)), with R + s = R0^2/(R - s) used for s < 0
        # so that no cancellation occurs
        with np.errstate(divide="ignore", invalid="ignore"):
            Ap = np.where(sp_ >= 0.0, Rp + sp_, R02 / (Rp - sp_))
            Am = np.where(sm >= 0.0, Rm + sm, R02 / (Rm - sm))
            f = np.log(Ap) - np.log(Am)
        tiny = R02 <= (1e-14 * ln_) ** 2
        f = np.where(tiny, 0.0, f)
        with np.errstate(divide="ignore", invalid="ignore"):
            beta = (np.arctan2(t0 * sp_, R02 + aw * Rp) - np.arctan2(t0 * sm, R02 + aw * Rm))
        beta = np.where(tiny, 0.0, beta)
        V0 += t0 * f - aw * beta
        Vr += u * (0.5 * (R02 * f + sp_ * Rp - sm * Rm))[:, None]
    V1 = Vr - (w0 * V0)[:, None] * nrm
    return V0, V1


# ---------------------------------------------------------------------------
# triangle-pair blocks
# ---------------------------------------------------------------------------

_RULES = {}


def _rule(kind, q):
    key = (kind, q)
    if key not in _RULES:
        if kind == "conical":
            _RULES[key] = conical_rule(q)
        elif kind == "graded":
            _RULES[key] = graded_rule(q)
        elif kind == "sub4":
            _RULES[key] = subdivide_rule(*conical_rule(q), 1)
        elif kind == "d7":
            _RULES[key] = dunavant7()
        elif kind == "vertex":
            _RULES[key] = vertex_rule(q)
        elif kind == "edge":
            _RULES[key] = edge_rule(q)
    return _RULES[key]


def _blocks_inner_analytic(P, Q, rule):
    """Raw 3x3 blocks for pairs with outer triangle P (m,3,3) and inner
    triangle Q (m,3,3), outer rule ``rule``, inner integral in closed form."""
    lam, w = rule
    m, nq = P.shape[0], lam.shape[0]
    A = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    r = np.einsum('qk,mkd->mqd', lam, P).reshape(-1, 3)
    Qr = np.repeat(Q, nq, axis=0)
    V0, V1 = potentials(r, Qr)
    r = r.reshape(m, nq, 3)
    V0 = V0.reshape(m, nq)
    V1 = V1.reshape(m, nq, 3)
    out = np.empty((m, 3, 3))
    for i in range(3):
        a = r - P[:, None, i, :]
        for j in range(3):
            inner = V1 + (r - Q[:, None, j, :]) * V0[:, :, None]
            out[:, i, j] = A * np.einsum('q,mq->m', w, np.einsum('mqd,mqd->mq', a, inner))
    return out


def _blocks_product(P, Q, rule):
    """Raw 3x3 blocks with the same rule on both triangles (smooth kernel)."""
    lam, w = rule
    AP = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    AQ = 0.5 * np.linalg.norm(np.cross(Q[:, 1] - Q[:, 0], Q[:, 2] - Q[:, 0]), axis=1)
    r = np.einsum('qk,mkd->mqd', lam, P)
    rp = np.einsum('qk,mkd->mqd', lam, Q)
    D = r[:, :, None, :] - rp[:, None, :, :]
    invR = 1.0 / np.sqrt(np.einsum('mabd,mabd->mab', D, D))
    W = (w[:, None] * w[None, :])[None] * invR * (AP * AQ)[:, None, None]
    out = np.empty((P.shape[0], 3, 3))
    for i in range(3):
        a = r - P[:, None, i, :]
        for j in range(3):
            b = rp - Q[:, None, j, :]
            out[:, i, j] = np.einsum('mab,mab->m', W, np.einsum('mad,mbd->mab', a, b))
    return out


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


def pair_blocks(mesh, ti, tj, chunk=20000, graded_q=20):
    """Raw blocks M_tt'[i, j] for the pairs (ti[k], tj[k]); rules by class:
    touching -> graded rule (q = graded_q) + closed-form inner;
    ratio < 0.5 -> 4 x subdivided conical q=10 + closed-form inner;
    ratio < 2 -> conical q=10 + closed-form inner;
    ratio < 12 -> conical q=6 + closed-form inner;
    otherwise -> 7-point degree-5 product rule on both triangles."""
    ti = np.asarray(ti, dtype=np.int64)
    tj = np.asarray(tj, dtype=np.int64)
    out = np.empty((ti.size, 3, 3))
    shared, ratio = classify_pairs(mesh, ti, tj)
    P = mesh.V[mesh.T]
    # touching pairs: rule graded toward the shared set of the outer triangle
    # (whole triangle / shared edge / shared vertex), outer vertices permuted
    # so the shared ones come first, block rows permuted back afterwards
    touch = np.nonzero(shared > 0)[0]
    if touch.size:
        Ti, Tj = mesh.T[ti[touch]], mesh.T[tj[touch]]
        isin = (Ti[:, :, None] == Tj[:, None, :]).any(axis=2)
        perm = np.argsort(~isin, axis=1, kind="stable")
        Pp = np.take_along_axis(P[ti[touch]], perm[:, :, None], axis=1)
        Qt = P[tj[touch]]
        res = np.empty((touch.size, 3, 3))
        for ns, kind in ((3, "graded"), (2, "edge"), (1, "vertex")):
            sel = np.nonzero(shared[touch] == ns)[0]
            if sel.size == 0:
                continue
            rule = _rule(kind, graded_q)
            if _clib() is not None:
                res[sel] = _c_blocks("oracle_blocks_analytic", Pp[sel], Qt[sel], rule)
            else:
                res[sel] = _blocks_inner_analytic(Pp[sel], Qt[sel], rule)
        blk = np.empty_like(res)
        np.put_along_axis(blk, perm[:, :, None], res, axis=1)
        out[touch] = blk
    classes = [
        ((shared == 0) & (ratio < 0.5), "analytic", ("sub4", 10)),
        ((shared == 0) & (ratio >= 0.5) & (ratio < 2.0), "analytic", ("conical", 10)),
        ((shared == 0) & (ratio >= 2.0) & (ratio < 12.0), "analytic", ("conical", 6)),
        ((shared == 0) & (ratio >= 12.0), "product", ("d7", 0)),
    ]
    for mask, how, rk in classes:
        idx = np.nonzero(mask)[0]
        rule = _rule(*rk)
        step = max(1, chunk * 64 // max(len(rule[1]), 1)) if how == "analytic" else chunk
        if _clib() is not None and idx.size:
            name = "oracle_blocks_analytic" if how == "analytic" else "oracle_blocks_product"
            out[idx] = _c_blocks(name, P[ti[idx]], P[tj[idx]], rule)
            continue
        for s in range(0, idx.size, step):
            k = idx[s:s + step]
            if how == "analytic":
                out[k] = _blocks_inner_analytic(P[ti[k]], P[tj[k]], rule)
            else:
                out[k] = _blocks_product(P[ti[k]], P[tj[k]], rule)
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
