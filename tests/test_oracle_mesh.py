"""Pins for the oracle's mesh, basis and Gram matrix (Sec. II-B/C)."""
import numpy as np
import pytest

import workloads as W
from oracle.mesh import RWGMesh, gram_local, gram_matrix
from oracle import integrals


@pytest.mark.parametrize("gen", [W.prism, W.paper_bar_e1, W.config1_bar])
def test_closed_surface_counts(gen):
    """Closed surfaces: b = 1.5 n (Sec. III-B) and Euler V - E + F = 2."""
    s = gen()
    m = RWGMesh(s.V, s.T)
    assert 2 * m.nedge == 3 * m.ntri
    assert s.V.shape[0] - m.nedge + m.ntri == 2


def test_wire_counts():
    s = W.config2_wires()
    assert s.n == 39936
    m = RWGMesh(s.V, s.T)
    assert m.nedge == 59904
    assert s.V.shape[0] - m.nedge + m.ntri == 2 * 8      # eight spheres


def test_prism_is_fig1():
    """Fig. 1: the prism has 8 triangular patches and 12 edges."""
    m = RWGMesh(*(lambda s: (s.V, s.T))(W.prism()))
    assert m.ntri == 8 and m.nedge == 12


def _edge_flux(m, e, t):
    """Line integral of f_e . nu over edge e, nu the in-plane unit normal of
    the edge pointing out of triangle t, by 5-point Gauss on the edge."""
    a, b = m.V[m.edge_vertices[e]]
    x, w = np.polynomial.legendre.leggauss(5)
    pts = a[None] + (0.5 * (x + 1))[:, None] * (b - a)[None]
    L = np.linalg.norm(b - a)
    tangent = (b - a) / L
    nu = np.cross(tangent, m.normal[t])
    cen = m.centroid[t]
    if np.dot(nu, pts[2] - cen) < 0:
        nu = -nu
    # evaluate f_e on t just inside the edge
    shrink = pts + 1e-9 * (cen - pts)
    f = np.zeros_like(shrink)
    P = m.V[m.T[t]]
    i = list(m.tri_edge[t]).index(e)
    s = m.tri_sign[t, i]
    f = s * (shrink - P[i]) / (2 * m.area[t])
    return 0.5 * L * np.sum(w * (f @ nu))


def test_rwg_unit_current_across_edge():
    """Eq. RWG without the edge length: the normal flux of f_e across edge e
    is 1 A, leaving T+ and entering T-; the normal component is continuous."""
    s = W.paper_bar_e1()
    m = RWGMesh(s.V, s.T)
    rng = np.random.default_rng(3)
    for e in rng.choice(m.nedge, 25, replace=False):
        out_plus = _edge_flux(m, e, m.tplus[e])
        out_minus = _edge_flux(m, e, m.tminus[e])
        assert out_plus == pytest.approx(1.0, abs=1e-9)
        assert out_minus == pytest.approx(-1.0, abs=1e-9)


def test_rwg_flux_zero_on_other_edges():
    """f_e has no normal component on the two other edges of each triangle."""
    s = W.prism()
    m = RWGMesh(s.V, s.T)
    for t in range(m.ntri):
        for i in range(3):
            e = m.tri_edge[t, i]
            for k in range(3):
                if k == i:
                    continue
                other = m.tri_edge[t, k]
                a, b = m.V[m.edge_vertices[other]]
                P = m.V[m.T[t]]
                mid = 0.5 * (a + b)
                f = m.tri_sign[t, i] * (mid - P[i]) / (2 * m.area[t])
                nu = np.cross(b - a, m.normal[t])
                assert abs(np.dot(f, nu)) < 1e-12 * np.linalg.norm(nu) * np.linalg.norm(f) + 1e-30


def test_gram_closed_form_matches_quadrature():
    """Closed-form Gram blocks = degree-4-exact conical Gauss quadrature of
    f_i . f_j (a quadratic integrand) on random triangles."""
    rng = np.random.default_rng(7)
    V = rng.standard_normal((30, 3))
    T = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8]])
    class Mini:
        pass
    m = Mini()
    m.V, m.T = V, T
    P = V[T]
    m.area = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    m.centroid = P.mean(axis=1)
    m.tri_sign = np.array([[1, -1, 1], [1, 1, -1], [-1, -1, 1]], float)
    m.local_scale = lambda: m.tri_sign / (2 * m.area[:, None])
    G = gram_local(m)
    lam, w = integrals.conical_rule(4)
    for t in range(3):
        r = lam @ P[t]
        f = [m.tri_sign[t, i] * (r - P[t, i]) / (2 * m.area[t]) for i in range(3)]
        ref = np.array([[m.area[t] * np.sum(w * np.einsum('qd,qd->q', f[i], f[j]))
                         for j in range(3)] for i in range(3)])
        assert np.allclose(G[t], ref, rtol=1e-13, atol=0)


def lateral_uniform_coefficients(m, s, direction):
    """Edge coefficients whose RWG expansion equals the uniform field
    ``direction`` on every lateral triangle of a box bar: the coefficient is
    the current through the edge from T+ to T-, i.e. the flux of the field
    out of a lateral triangle on either side (sign flipped for T-)."""
    contact = np.zeros(m.ntri, bool)
    contact[s.ports[0][0]] = True
    contact[s.ports[0][1]] = True
    coef = np.zeros(m.nedge)
    for e in range(m.nedge):
        t, sign = (m.tplus[e], 1.0) if not contact[m.tplus[e]] else (m.tminus[e], -1.0)
        a, b = m.V[m.edge_vertices[e]]
        nu = np.cross(b - a, m.normal[t])          # length x in-plane normal
        if np.dot(nu, 0.5 * (a + b) - m.centroid[t]) < 0:
            nu = -nu
        coef[e] = sign * np.dot(direction, nu)
    return coef


def test_gram_uniform_axial_current_gives_dc_resistance_factor():
    """Uniform axial surface current x/P on the lateral faces of a bar lies in
    the basis span; its Gram energy over the lateral faces is exactly l/P, so
    r_s l/P is the resistance of the tube (the rho l / A limit)."""
    s = W.config1_bar()
    m = RWGMesh(s.V, s.T)
    P = 2 * (20e-6 + 10e-6)
    ell = 1e-3
    coef = lateral_uniform_coefficients(m, s, np.array([1.0, 0, 0])) / P
    lateral = np.ones(m.ntri, bool)
    lateral[s.ports[0][0]] = False
    lateral[s.ports[0][1]] = False
    G = gram_matrix(m, weight=lateral.astype(float))
    assert coef @ (G @ coef) == pytest.approx(ell / P, rel=1e-12)
