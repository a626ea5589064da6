"""Pins for the oracle's post-processing (Sec. V-A: branch currents, branch
voltages, panel potentials with the sink faces at 0 V, centroid current)."""
import numpy as np
import pytest

import workloads as W
from oracle.mesh import RWGMesh, gram_matrix
from oracle.circuit import Circuit
from oracle import solve as S, post as PO

SIGMA = 5.8e7


def _solve(mesh, circ, K, om, zs):
    wt = S.triangle_impedance(mesh, circ, zs)
    G = gram_matrix(mesh, weight=wt).toarray()
    Zb = S.branch_impedance(G, K, om, 1.0, circ.nport)
    A = circ.loop_matrix()
    Zl = S.loop_impedance(A, Zb)
    _, I = S.port_admittance(Zl, circ.port_loop)
    return A, Zb, I


def test_resistive_bar_linear_potential(c1):
    """Constant real surface resistance at 15 Hz: the resistive solution
    (uniform axial current, potential falling linearly from 1 V at the source
    face to 0 V at the sink face) lies in the discrete space, and the
    inductive term changes real parts only at second order in omega L / R
    (about 1e-12 here).  So every lateral panel's potential has real part
    1 - x_c / L at its centroid, the centroid current has real part
    x / (r_s L), and the imaginary parts are first-order small."""
    m, c, K = c1["mesh"], c1["circ"], c1["K"]
    s = c1["s"]
    L, w, t = 1e-3, 20e-6, 10e-6
    rs = 2 * (w + t) / (SIGMA * w * t)
    A, Zb, I = _solve(m, c, K, 2 * np.pi * 15.0, rs)
    Ib = PO.branch_currents(A, I[:, 0])
    Vb = PO.branch_voltages(Zb, Ib)
    phi = PO.panel_potentials(c, Vb)
    J = PO.centroid_current(m, Ib[:m.nedge])
    fo = s.params["face_of"]
    lat = ~np.isin(fo, ["x0", "x1"])
    xc = m.centroid[:, 0]
    assert np.abs(phi[lat].real - (1.0 - xc[lat] / L)).max() <= 1e-9
    assert np.abs(phi.imag).max() <= 1e-4
    src = phi[fo == "x0"]
    assert np.all(src == src[0]) and abs(src[0] - 1.0) <= 1e-12
    assert np.all(phi[fo == "x1"] == 0.0)
    J0 = 1.0 / (rs * L)
    assert np.abs(J[lat].real - np.array([J0, 0.0, 0.0])).max() <= 1e-8 * J0
    # the port current is the perimeter times the surface current density
    assert I[c.port_loop[0], 0].real == pytest.approx(2 * (w + t) * J0, rel=1e-9)


def test_full_model_source_to_sink_is_one_volt(c1):
    """At 1 GHz (skin effect and inductance): the source face is 1 V above
    the sink face, the branch voltages are consistent with node potentials
    (every loop equation holds), and the branch currents obey Kirchhoff's
    current law at every node that is not a port terminal."""
    m, c, K = c1["mesh"], c1["circ"], c1["K"]
    om = 2 * np.pi * 1e9
    A, Zb, I = _solve(m, c, K, om, S.surface_impedance(om, SIGMA))
    Ib = PO.branch_currents(A, I[:, 0])
    Vb = PO.branch_voltages(Zb, Ib)
    phi = PO.node_potentials(c, Vb)
    src, snk = c.port_src_node[0], c.port_snk_node[0]
    assert phi[snk] == 0.0
    assert abs(phi[src] - 1.0) <= 1e-10
    res = max(abs(phi[int(c.branch_u[e])] - phi[int(c.branch_v[e])] - Vb[e])
              for e in range(m.nedge) if c.branch_u[e] != c.branch_v[e])
    assert res <= 1e-10 * np.abs(Vb).max()
    N = c.incidence().toarray()
    kcl = N @ Ib
    idx = {int(x): i for i, x in enumerate(c.nodes)}
    term = {idx[src], idx[snk]}
    inner = [i for i in range(len(c.nodes)) if i not in term]
    assert np.abs(kcl[inner]).max() <= 1e-12 * np.abs(Ib).max()
    # the source branch (sink -> source) carries the port current into the source face
    assert Ib[m.nedge] == I[c.port_loop[0], 0]


def test_shorted_ports_are_equipotential():
    """One bar, three ports (x, y, z face pairs), port 0 driven: its source
    sits 1 V above its sink (the reference), the shorted ports' faces are at
    equal potentials."""
    from workloads.geometry import box_bar
    from oracle import integrals
    s = box_bar(np.linspace(0.0, 100e-6, 13), np.linspace(0.0, 6e-6, 3), np.linspace(0.0, 4e-6, 3))
    fo = s.params["face_of"]
    ports = [(np.nonzero(fo == a)[0], np.nonzero(fo == b)[0]) for a, b in (("x0", "x1"), ("y0", "y1"), ("z0", "z1"))]
    m = RWGMesh(s.V, s.T)
    c = Circuit(m, ports)
    K = integrals.kernel_dense(m)
    om = 2 * np.pi * 5e9
    A, Zb, I = _solve(m, c, K, om, S.surface_impedance(om, SIGMA))
    phi = PO.node_potentials(c, PO.branch_voltages(Zb, PO.branch_currents(A, I[:, 0])))
    assert phi[c.port_snk_node[0]] == 0.0
    assert abs(phi[c.port_src_node[0]] - 1.0) <= 1e-10
    for k in (1, 2):
        assert abs(phi[c.port_src_node[k]] - phi[c.port_snk_node[k]]) <= 1e-10
