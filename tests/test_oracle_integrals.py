"""Pins for the oracle's kernel integrals (first term of Eq. Zb, Eq. StaticGF).

The oracle integrates both surfaces numerically (Sauter-Schwab on touching
pairs, adaptive product rules elsewhere).  It is pinned against:
* brute force: the classical closed-form potential of a flat triangle for the
  inner integral and scipy's adaptive cubature for the outer one
  (tests/brute.py), on full 3 x 3 blocks of coincident, edge-adjacent
  (coplanar and folded), vertex-adjacent (coplanar and not) pairs, with
  non-uniform currents, to 1e-9; the brute-force potential itself is pinned
  against dense product quadrature off the surface and the closed form of a
  rectangle in its plane;
* closed forms: the self-interaction of the unit square and the energy of a
  uniform axial current on a rectangular tube;
* symmetry and positivity of K, and convergence in the rule orders.
"""
import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle.mesh import RWGMesh
from oracle import integrals as I
from test_oracle_mesh import lateral_uniform_coefficients
import brute


def test_potentials_match_brute_force_off_surface():
    """Closed-form V0, V1 (the brute-force reference's inner integral) =
    dense subdivided Gauss quadrature for observation points away from the
    triangle (smooth integrand)."""
    rng = np.random.default_rng(11)
    Q = rng.standard_normal((1, 3, 3))
    lam, w = I.subdivide_rule(*I.conical_rule(12), 3)
    pts = lam @ Q[0]
    A = 0.5 * np.linalg.norm(np.cross(Q[0, 1] - Q[0, 0], Q[0, 2] - Q[0, 0]))
    for r in rng.standard_normal((6, 3)) * 3 + 4:
        R = np.linalg.norm(pts - r, axis=1)
        V0, V1 = brute.flat_triangle_potentials(r[None], Q[0])
        assert V0[0] == pytest.approx(A * np.sum(w / R), rel=1e-12)
        assert np.allclose(V1[0], A * np.sum(w[:, None] * (pts - r) / R[:, None], axis=0),
                           rtol=1e-11, atol=1e-14)


def rect_potential(x, y, a, b):
    """int over [0,a]x[0,b] of 1/|(x,y)-(u,v)|: sum of four corner terms
    X asinh(Y/X) + Y asinh(X/Y)."""
    def f(X, Y):
        return X * np.arcsinh(Y / X) + Y * np.arcsinh(X / Y)
    return f(x, y) + f(a - x, y) + f(x, b - y) + f(a - x, b - y)


@pytest.mark.parametrize("pt", [(0.5, 0.2), (1.7, 0.6), (1.0, 0.35)])
def test_potentials_in_plane_rectangle_closed_form(pt):
    """Two triangles tiling a rectangle: the in-plane potential equals the
    closed form of the rectangle, also at points on the shared diagonal."""
    a, b = 2.0, 0.7
    T = np.array([[[0, 0, 0], [a, 0, 0], [a, b, 0]], [[0, 0, 0], [a, b, 0], [0, b, 0]]], float)
    r = np.array([[pt[0], pt[1], 0.0]])
    V0 = sum(brute.flat_triangle_potentials(r, T[k])[0][0] for k in range(2))
    assert V0 == pytest.approx(rect_potential(pt[0], pt[1], a, b), rel=1e-13)


def _uniform_local_coef(P, J):
    """Local coefficients c_i with sum_i c_i (r - p_i)/(2A) = J on triangle P."""
    A = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
    M = np.vstack([np.ones(3), -P.T])
    rhs = np.concatenate([[0.0], 2 * A * J])
    return np.linalg.lstsq(M, rhs, rcond=None)[0]


def test_unit_square_self_interaction_closed_form():
    """int int over the unit square of 1/|r - r'| = 4/3 (1 - sqrt 2) +
    4 ln(1 + sqrt 2) (closed form), from coincident and edge-adjacent
    singular triangle pairs."""
    V = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], float)
    T = np.array([[0, 1, 2], [0, 2, 3]])
    P = V[T]
    class Mini:
        pass
    mm = Mini()
    mm.V, mm.T = V, T
    mm.centroid = P.mean(axis=1)
    mm.area = np.array([0.5, 0.5])
    coef = np.array([_uniform_local_coef(P[t], np.array([1.0, 0, 0])) for t in range(2)])
    ti = np.repeat(np.arange(2), 2)
    tj = np.tile(np.arange(2), 2)
    B = I.pair_blocks(mm, ti, tj)
    a = coef[ti] / (2 * mm.area[ti])[:, None]
    b = coef[tj] / (2 * mm.area[tj])[:, None]
    val = np.einsum('ki,kij,kj->', a, B, b)
    ref = 4.0 / 3.0 * (1 - np.sqrt(2)) + 4 * np.log(1 + np.sqrt(2))
    assert val == pytest.approx(ref, rel=2e-10)


def _strip_kernel(ell):
    """F(d) = int_0^l int_0^l dx dx' / sqrt((x - x')^2 + d^2) in closed form."""
    def F(d):
        return 2.0 * (ell * np.arcsinh(ell / d) - np.sqrt(ell * ell + d * d) + d)
    return F


def tube_kernel_energy(ell, w, t):
    """(1/P^2) sum over lateral face pairs of int int 1/R for uniform axial
    current on a w x t rectangular tube of length ell: the axial double
    integral in closed form F(d), the remaining cross-section integrals by
    adaptive quadrature (same face: 2 int_0^a (a - u) F(u) du; opposite faces
    at distance D: 2 int_0^a (a - u) F(sqrt(u^2 + D^2)) du; adjacent faces:
    int_0^w int_0^t F(sqrt(a^2 + b^2)) in polar coordinates)."""
    F = _strip_kernel(ell)
    opts = dict(epsabs=0, epsrel=1e-13, limit=200)

    def same(a):
        return 2 * integrate.quad(lambda u: (a - u) * F(u), 0, a, **opts)[0]

    def opposite(a, D):
        return 2 * integrate.quad(lambda u: (a - u) * F(np.hypot(u, D)), 0, a, **opts)[0]

    def corner(a, b):
        th0 = np.arctan2(b, a)
        def radial(th, rmax):
            return integrate.quad(lambda r: F(r) * r, 0, rmax, **opts)[0]
        i1 = integrate.quad(lambda th: radial(th, a / np.cos(th)), 0, th0, **opts)[0]
        i2 = integrate.quad(lambda th: radial(th, b / np.sin(th)), th0, np.pi / 2, **opts)[0]
        return i1 + i2

    P = 2 * (w + t)
    total = 2 * same(w) + 2 * same(t) + 2 * opposite(w, t) + 2 * opposite(t, w) + 8 * corner(w, t)
    return total / P ** 2


def test_bar_uniform_current_kernel_energy_closed_form():
    """Uniform axial current x/P on the lateral faces of a box bar: the
    oracle's triangle-pair sum equals the strip closed form (the surface
    analogue of the rectangular-bar partial self-inductance)."""
    ell, w, t = 100e-6, 20e-6, 10e-6
    s = W.box_bar(np.linspace(0, ell, 11), np.linspace(-w / 2, w / 2, 5),
                  np.linspace(-t / 2, t / 2, 3))
    m = RWGMesh(s.V, s.T)
    P = 2 * (w + t)
    coef = lateral_uniform_coefficients(m, s, np.array([1.0, 0, 0])) / P
    lateral = np.ones(m.ntri, bool)
    lateral[s.ports[0][0]] = False
    lateral[s.ports[0][1]] = False
    loc = coef[m.tri_edge] * m.tri_sign
    val = I.quadratic_form(m, loc, np.nonzero(lateral)[0])
    ref = tube_kernel_energy(ell, w, t)
    assert val == pytest.approx(ref, rel=2e-8)


def test_kernel_symmetric_and_positive(c1):
    K = c1["K"]
    # (t, t') and (t', t) use different outer triangles: symmetric to the
    # quadrature accuracy
    assert np.abs(K - K.T).max() <= 1e-9 * np.abs(K).max()
    u = np.random.default_rng(5).standard_normal((K.shape[0], 4))
    assert np.all(np.einsum('ik,ij,jk->k', u, K, u) > 0)
    assert np.all(np.diag(K) > 0)


def test_kernel_rows_match_dense(c1):
    """kernel_rows integrates each pair with the row triangle outermost;
    kernel_dense averages both orders, so the two differ by at most half the
    quadrature asymmetry bounded above."""
    m, K = c1["mesh"], c1["K"]
    rows = np.array([0, 17, 1499, 2999])
    R = I.kernel_rows(m, rows)
    assert np.abs(R - K[rows]).max() <= 0.5e-9 * np.abs(K).max()


def test_gauss_rule_of_the_helper():
    for q in (1, 2, 5, 12, 31):
        x, w = I.gauss01(q)
        xr, wr = np.polynomial.legendre.leggauss(q)
        assert np.allclose(np.sort(x), np.sort(0.5 * (1 - xr)), rtol=0, atol=1e-15)
        assert np.allclose(np.sort(w), np.sort(0.5 * wr), rtol=0, atol=1e-15)


# touching pairs in general position (shared vertices first, same order on
# both triangles), with non-uniform currents (all nine block entries)
_TOUCH = {
    "coincident": (np.array([[0, 0, 0], [1.0, 0, 0], [0.8, 0.6, 0]]),
                   np.array([[0, 0, 0], [1.0, 0, 0], [0.8, 0.6, 0]]), 3),
    "edge_coplanar": (np.array([[0, 0, 0], [1.0, 0, 0], [0.4, 0.7, 0]]),
                      np.array([[0, 0, 0], [1.0, 0, 0], [0.5, -0.8, 0]]), 2),
    "edge_folded": (np.array([[0, 0, 0], [1.0, 0, 0], [0.4, 0.7, 0]]),
                    np.array([[0, 0, 0], [1.0, 0, 0], [0.6, 0.0, -0.9]]), 2),
    "vertex_coplanar": (np.array([[0, 0, 0], [1.0, 0.2, 0], [0.3, 0.9, 0]]),
                        np.array([[0, 0, 0], [-0.8, 0.3, 0], [-0.4, -0.9, 0]]), 1),
    "vertex_skew": (np.array([[0, 0, 0], [1.0, 0.2, 0], [0.3, 0.9, 0]]),
                    np.array([[0, 0, 0], [-0.8, 0.3, 0.1], [-0.4, -0.9, 0.4]]), 1),
}


@pytest.mark.parametrize("case", sorted(_TOUCH))
def test_touching_blocks_match_brute_force(case):
    """Sauter-Schwab blocks = closed-form inner x adaptive outer cubature,
    all nine entries, to 1e-9 of the largest."""
    P, Q, kind = _TOUCH[case]
    ref = brute.pair_block(P, Q, rtol=1e-10)
    got = I.blocks_touching(P[None], Q[None], [kind], 12)[0]
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()


def test_mesh_pairs_match_brute_force():
    """Pairs of the paper's bar mesh through pair_blocks (vertex orders,
    permutations back, order by shape): an obtuse end-face triangle with
    itself, with an obtuse neighbour, a lateral triangle across the end-face
    corner (90 degree fold), a vertex neighbour, and a separated pair."""
    s = W.paper_bar_e1()
    m = RWGMesh(s.V, s.T)
    Pall = m.V[m.T]
    # the most obtuse triangle and its touching neighbours of each kind
    _, ang = I.shape_quality(Pall)
    t = int(np.argmax(ang))
    sh = (m.T[t][None, :, None] == m.T[:, None, :]).any(axis=2).sum(axis=1)
    nrm = np.cross(Pall[:, 1] - Pall[:, 0], Pall[:, 2] - Pall[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    coplanar = np.abs(nrm @ nrm[t]) > 0.999
    picks = [t]
    picks.append(int(np.nonzero((sh == 2) & coplanar)[0][0]))
    picks.append(int(np.nonzero((sh == 2) & ~coplanar)[0][0]))
    picks.append(int(np.nonzero((sh == 1) & ~coplanar)[0][0]))
    far = np.linalg.norm(m.centroid - m.centroid[t], axis=1)
    picks.append(int(np.nonzero((sh == 0) & (far < 2 * far[picks[-1]] + 1e-6))[0][0]))
    got = I.pair_blocks(m, np.full(len(picks), t), np.array(picks))
    for k, tj in enumerate(picks):
        P = Pall[t].copy()
        Q = Pall[tj].copy()
        # brute.pair_block wants the shared vertices first on the outer triangle
        shared = [i for i in range(3) if m.T[t][i] in m.T[tj]]
        perm = shared + [i for i in range(3) if i not in shared]
        ref = brute.pair_block(P[perm], Q, rtol=1e-9)
        blk = np.empty((3, 3))
        blk[perm, :] = ref
        assert np.abs(got[k] - blk).max() <= 1e-8 * np.abs(blk).max(), (k, tj)


def test_touching_order_converged():
    """The default orders for touching pairs of the paper's bar (thin and
    obtuse end-face triangles included) agree with much higher orders to
    1e-7 of each block."""
    s = W.paper_bar_e1()
    m = RWGMesh(s.V, s.T)
    ti, tj = np.repeat(np.arange(60), m.ntri), np.tile(np.arange(m.ntri), 60)
    sh = (m.T[ti][:, :, None] == m.T[tj][:, None, :]).any(axis=2).sum(axis=1)
    k = np.nonzero(sh > 0)[0]
    a = I.pair_blocks(m, ti[k], tj[k])
    b = I.pair_blocks(m, ti[k], tj[k], ss_q=30)
    err = np.abs(a - b).reshape(k.size, -1).max(axis=1) / np.abs(b).reshape(k.size, -1).max(axis=1)
    assert err.max() <= 1e-7


def test_separated_rules_converged():
    """Separated pairs (all of one triangle's row on the bar C1): the default
    rules agree with a far finer integration to 1e-8 of each block."""
    s = W.config1_bar()
    m = RWGMesh(s.V, s.T)
    P = m.V[m.T]
    for t in (0, 777):
        tj = np.arange(m.ntri)
        sh = (m.T[t][None, :, None] == m.T[tj][:, None, :]).any(axis=2).sum(axis=1)
        tj = tj[sh == 0]
        a = I.blocks_separated(P[np.full(tj.size, t)], P[tj])
        b = I.blocks_separated(P[np.full(tj.size, t)], P[tj], refine=True)
        err = np.abs(a - b).reshape(tj.size, -1).max(axis=1) / np.abs(b).reshape(tj.size, -1).max(axis=1)
        assert err.max() <= 1e-8
