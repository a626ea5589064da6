"""The pre-corrected FFT operator, step by step (oracle, FP64).

Paper Sec. IV-B: the dense kernel matrix is approximated as
    L_b ~ L_d + I H B                                     (Eq. Lb)
with
  1. projection  Q_g = B alpha                            (Eq. Projection)
  2. convolution phi_g = H Q_g, H three-level Toeplitz    (Eq. FFTCal)
  3. interpolation Phi_g = I phi_g with I = B^T           (Eq. interpolation)
  4. near-field entries computed directly, pre-corrected  (Eq. Lb).

Readings fixed here (the paper leaves them open):
* grid: N_d nodes per dimension, spacing h_d = extent_d / (N_d - O_s),
  origin x0_d = min_d - (O_s - 1)/2 h_d, so every stencil fits;
* the stencil of triangle t is the O_s^3 block of nodes whose first index is
  floor((c_t - x0)/h) - (O_s/2 - 1) in each dimension (c_t: centroid), i.e.
  the O_s nodes around the centroid in each direction;
* B is built per triangle: each half of a basis function is projected
  through its own triangle's stencil, with B[(c, g), e] = int_t f_e,c W_g dS,
  W_g the tensor-product Lagrange polynomial of node g on the stencil, and
  the integral taken with the 7-point degree-5 rule;
* H(g - g') = 1/|x_g - x_g'| and H(0) := 0 (every pair whose stencils share
  a node is near, so H(0) never reaches a far pair);
* near pairs: stencil index boxes overlap in every dimension, or the
  centroid distance is below kappa * max_d (O_s - 1) h_d, or the two
  triangles share a vertex (their singular entries are always computed
  directly, also on a grid much finer than the triangles);
* pre-correction: L_d = sum over near triangle pairs of (exact block -
  the same pair through the grid), so near pairs get exact values and far
  pairs the grid values.
"""
import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree

from . import integrals


def dunavant7():
    return integrals.dunavant7()


class Grid:
    def __init__(self, V, dims, order=4):
        V = np.asarray(V, dtype=np.float64)
        self.dims = np.asarray(dims, dtype=np.int64)
        self.order = int(order)
        lo, hi = V.min(axis=0), V.max(axis=0)
        ext = hi - lo
        h = ext / (self.dims - self.order)
        if np.any(ext <= 0):
            h = np.where(ext > 0, h, h.max())
        self.h = h
        self.x0 = lo - 0.5 * (self.order - 1) * h
        self.N = int(np.prod(self.dims))

    def anchor(self, pts):
        a = np.floor((pts - self.x0) / self.h).astype(np.int64) - (self.order // 2 - 1)
        return np.clip(a, 0, self.dims - self.order)

    def node_pos(self, idx3):
        return self.x0 + idx3 * self.h


def lagrange_1d(order, x):
    """Values of the O_s Lagrange basis polynomials on nodes 0..O_s-1 at x
    (shape x.shape + (O_s,))."""
    out = np.ones(x.shape + (order,))
    for k in range(order):
        for m in range(order):
            if m != k:
                out[..., k] *= (x - m) / (k - m)
    return out


def projection_moments(mesh, grid):
    """Per-triangle stencil anchors and moments
        M0_t[g]    = int_t W_g dS
        M1_t[g, c] = int_t (r - c_t)_c W_g dS
    over the O_s^3 local stencil nodes g (x slowest), 7-point rule."""
    lam, w = dunavant7()
    P = mesh.V[mesh.T]                               # (n, 3, 3)
    r = np.einsum('qk,nkd->nqd', lam, P)             # (n, 7, 3)
    a = grid.anchor(mesh.centroid)                   # (n, 3)
    u = (r - grid.x0) / grid.h - a[:, None, :]       # local coordinates
    O = grid.order
    Lx = lagrange_1d(O, u[..., 0])
    Ly = lagrange_1d(O, u[..., 1])
    Lz = lagrange_1d(O, u[..., 2])
    Wg = np.einsum('nqi,nqj,nqk->nqijk', Lx, Ly, Lz).reshape(r.shape[0], r.shape[1], O ** 3)
    A = mesh.area
    M0 = A[:, None] * np.einsum('q,nqg->ng', w, Wg)
    rl = r - mesh.centroid[:, None, :]
    M1 = A[:, None, None] * np.einsum('q,nqg,nqc->ngc', w, Wg, rl)
    return a, M0, M1


def local_stencil_offsets(order):
    i = np.arange(order)
    return np.stack(np.meshgrid(i, i, i, indexing="ij"), axis=-1).reshape(-1, 3)


def triangle_grid_weights(mesh, grid):
    """b_t[c, g, i] = s_i/(2 A_t) (M1_t[g, c] - (p_i - c_t)_c M0_t[g]):
    the value B[(c, node), e(t, i)] receives from triangle t."""
    a, M0, M1 = projection_moments(mesh, grid)
    P = mesh.V[mesh.T]
    pl = P - mesh.centroid[:, None, :]               # (n, 3 local vertex, 3 comp)
    sc = mesh.local_scale()                          # (n, 3)
    bt = (M1[:, None, :, :] - pl[:, :, None, :] * M0[:, None, :, None])   # (n, i, g, c)
    bt = bt * sc[:, :, None, None]
    return a, bt.transpose(0, 3, 2, 1)               # (n, c, g, i)


def projection_matrix(mesh, grid):
    """Sparse B (3 N_g x b), rows ordered (component, gx, gy, gz)."""
    a, bt = triangle_grid_weights(mesh, grid)
    O = grid.order
    off = local_stencil_offsets(O)
    n = mesh.ntri
    g3 = a[:, None, :] + off[None, :, :]             # (n, O^3, 3)
    Ny, Nz = grid.dims[1], grid.dims[2]
    gl = (g3[..., 0] * Ny + g3[..., 1]) * Nz + g3[..., 2]      # (n, O^3)
    rows = (np.arange(3)[None, :, None, None] * grid.N + gl[:, None, :, None])
    rows = np.broadcast_to(rows, (n, 3, O ** 3, 3))
    cols = np.broadcast_to(mesh.tri_edge[:, None, None, :], (n, 3, O ** 3, 3))
    B = sp.coo_matrix((bt.reshape(-1), (rows.reshape(-1), cols.reshape(-1))),
                      shape=(3 * grid.N, mesh.nedge))
    return B.tocsr()


def green_grid(grid, h0=0.0):
    """H on the zero-padded (2N_x, 2N_y, 2N_z) circulant embedding:
    H(m) = 1/|(m_x h_x, m_y h_y, m_z h_z)| with m folded to [-N+1, N-1],
    H(0) = 0 and the unused offset N set to 0."""
    axes = []
    for d in range(3):
        Nd = grid.dims[d]
        m = np.arange(2 * Nd)
        off = np.where(m < Nd, m, m - 2 * Nd).astype(np.float64)
        off[Nd] = np.nan
        axes.append(off * grid.h[d])
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    R = np.sqrt(X * X + Y * Y + Z * Z)
    with np.errstate(divide="ignore"):
        H = 1.0 / R
    H[np.isnan(H)] = 0.0
    H[0, 0, 0] = h0
    return H


def kernel_spectrum(grid, h0=0.0):
    """FFT of the circulant-embedded H (real and even, so real)."""
    return np.fft.fftn(green_grid(grid, h0)).real


def convolve(grid, Q, Ghat=None):
    """phi[c] = H * Q[c] (Toeplitz product through the padded FFT);
    Q has shape (3, N_x, N_y, N_z) (or (..., N_x, N_y, N_z))."""
    if Ghat is None:
        Ghat = kernel_spectrum(grid)
    Nx, Ny, Nz = grid.dims
    s = (2 * Nx, 2 * Ny, 2 * Nz)
    F = np.fft.fftn(Q, s=s, axes=(-3, -2, -1))
    out = np.fft.ifftn(F * Ghat, axes=(-3, -2, -1))
    return out[..., :Nx, :Ny, :Nz]


def convolve_direct(grid, Q):
    """O(N^2) Toeplitz sum, for checking ``convolve`` on tiny grids."""
    idx = np.stack(np.meshgrid(*[np.arange(d) for d in grid.dims], indexing="ij"), -1).reshape(-1, 3)
    D = (idx[:, None, :] - idx[None, :, :]) * grid.h
    R = np.linalg.norm(D, axis=2)
    with np.errstate(divide="ignore"):
        H = np.where(R > 0, 1.0 / R, 0.0)
    q = Q.reshape(Q.shape[:-3] + (-1,))
    return (q @ H.T).reshape(Q.shape)


def near_pairs(mesh, grid, kappa=1.5):
    """All ordered near pairs (t, t') including t = t' (see module notes)."""
    c = mesh.centroid
    a = grid.anchor(c)
    O = grid.order
    rad = kappa * (O - 1) * grid.h.max()
    rbox = np.linalg.norm(O * grid.h)
    tree = cKDTree(c)
    pairs = tree.query_pairs(max(rad, rbox) * (1 + 1e-12), output_type="ndarray")
    ti, tj = pairs[:, 0], pairs[:, 1]
    d = np.linalg.norm(c[ti] - c[tj], axis=1)
    box = np.all(np.abs(a[ti] - a[tj]) <= O - 1, axis=1)
    keep = box | (d < rad)
    ti, tj = ti[keep], tj[keep]
    n = mesh.ntri
    # pairs that share a vertex are singular: always computed directly
    # (near), even where the grid is much finer than the triangles
    vt = mesh.T.reshape(-1)
    tri = np.repeat(np.arange(n), 3)
    order_v = np.argsort(vt, kind="stable")
    vs, ts = vt[order_v], tri[order_v]
    starts = np.searchsorted(vs, np.arange(mesh.V.shape[0] + 1))
    ta, tb = [], []
    for v in range(mesh.V.shape[0]):
        group = ts[starts[v]:starts[v + 1]]
        if group.size > 1:
            A, B = np.meshgrid(group, group, indexing="ij")
            sel = A < B
            ta.append(A[sel])
            tb.append(B[sel])
    if ta:
        tpair = np.unique(np.stack([np.concatenate(ta), np.concatenate(tb)], axis=1), axis=0)
        have = np.stack([np.minimum(ti, tj), np.maximum(ti, tj)], axis=1)
        allp = np.unique(np.concatenate([have, tpair]), axis=0)
        ti, tj = allp[:, 0], allp[:, 1]
    ti_all = np.concatenate([ti, tj, np.arange(n)])
    tj_all = np.concatenate([tj, ti, np.arange(n)])
    order = np.lexsort((tj_all, ti_all))
    return ti_all[order], tj_all[order]


def grid_pair_blocks(mesh, grid, ti, tj, bt=None, anchors=None, chunk=8192, h0=0.0):
    """(I H B) restricted to triangle pairs: C[k][i, j] =
    sum_c sum_{g in S_t, g' in S_t'} b_t[c, g, i] H(g - g') b_t'[c, g', j].
    Pairs are grouped by anchor offset, since the 64 x 64 block of H between
    two stencils depends only on that offset."""
    if bt is None:
        anchors, bt = triangle_grid_weights(mesh, grid)
    O = grid.order
    off = local_stencil_offsets(O)
    G = O ** 3
    out = np.empty((ti.size, 3, 3))
    delta = anchors[ti] - anchors[tj]
    keys, inv = np.unique(delta, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    order = np.argsort(inv, kind="stable")
    bounds = np.searchsorted(inv[order], np.arange(keys.shape[0] + 1))
    for kidx in range(keys.shape[0]):
        sel_all = order[bounds[kidx]:bounds[kidx + 1]]
        d = (keys[kidx][None, None, :] + off[:, None, :] - off[None, :, :]) * grid.h
        R = np.linalg.norm(d, axis=-1)
        with np.errstate(divide="ignore"):
            H = np.where(R > 0, 1.0 / R, h0)                   # (g, g')
        for s in range(0, sel_all.size, chunk):
            sel = sel_all[s:s + chunk]
            bj = bt[tj[sel]]                                    # (m, c, g', j)
            tmp = np.matmul(H[None, None], bj)                  # (m, c, g, j)
            out[sel] = np.einsum('mcgi,mcgj->mij', bt[ti[sel]], tmp, optimize=True)
    return out


def scaled_exact_blocks(mesh, ti, tj):
    """Exact K contributions of triangle pairs, scaled by s/(2A) on both sides."""
    raw = integrals.pair_blocks(mesh, ti, tj)
    sc = mesh.local_scale()
    return raw * sc[ti][:, :, None] * sc[tj][:, None, :]


def precorrection(mesh, grid, kappa=1.5, pairs=None, h0=0.0):
    """Sparse b x b L_d = sum over near pairs of (exact - grid) blocks."""
    ti, tj = near_pairs(mesh, grid, kappa) if pairs is None else pairs
    anchors, bt = triangle_grid_weights(mesh, grid)
    D = scaled_exact_blocks(mesh, ti, tj) - grid_pair_blocks(mesh, grid, ti, tj, bt, anchors, h0=h0)
    rows = np.repeat(mesh.tri_edge[ti], 3, axis=1).reshape(-1)
    cols = np.tile(mesh.tri_edge[tj], (1, 3)).reshape(-1)
    return sp.coo_matrix((D.reshape(-1), (rows, cols)), shape=(mesh.nedge, mesh.nedge)).tocsr()


class PFFTOperator:
    """K alpha ~ B^T (H * (B alpha)) + L_d alpha, every step explicit."""

    def __init__(self, mesh, dims, order=4, kappa=1.5, with_near=True, h0=0.0):
        self.mesh = mesh
        self.grid = Grid(mesh.V, dims, order)
        self.B = projection_matrix(mesh, self.grid)
        self.Ghat = kernel_spectrum(self.grid, h0)
        self.Ld = precorrection(mesh, self.grid, kappa, h0=h0) if with_near else None

    def far(self, alpha):
        g = self.grid
        shp = (3,) + tuple(g.dims)
        alpha = np.asarray(alpha)
        cols = alpha.reshape(alpha.shape[0], -1)
        out = np.empty_like(cols, dtype=np.complex128)
        for k in range(cols.shape[1]):
            Q = (self.B @ cols[:, k]).reshape(shp)
            phi = convolve(g, Q, self.Ghat)
            out[:, k] = self.B.T @ phi.reshape(-1)
        return out.reshape(alpha.shape)

    def apply(self, alpha):
        y = self.far(alpha)
        if self.Ld is not None:
            y = y + self.Ld @ alpha
        return y
