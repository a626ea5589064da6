"""Pins for the oracle's circuit graph and loop basis (Sec. III)."""
import numpy as np
import pytest

import workloads as W
from oracle.mesh import RWGMesh
from oracle.circuit import Circuit


def _circ(s, ports=None):
    m = RWGMesh(s.V, s.T)
    return m, Circuit(m, s.ports if ports is None else ports)


def test_prism_loops_without_and_with_source():
    """Fig. 1 prism: 8 nodes, 12 branches, one conductor -> b - n + s = 5
    fundamental loops; a voltage source between two nodes adds one link
    (Sec. III-C) -> 6."""
    s = W.prism()
    m, c0 = _circ(s, ports=[])
    assert c0.nloop == 12 - 8 + 1 == 5
    m, c1 = _circ(s)
    assert c1.nloop == 6


def test_paper_bar_428_triangles_230_loops():
    """Sec. V-A: 428 triangles give 230 loops.  With each 8-triangle end face
    merged into one contact node: n' = 428 - 16 + 2 = 414, b = 642,
    l = b - n' + s + p = 642 - 414 + 1 + 1 = 230."""
    s = W.paper_bar_e1()
    assert s.n == 428
    m, c = _circ(s)
    assert m.nedge == 642 and len(c.nodes) == 414 and c.ncomp == 1
    assert c.nloop == 230


def test_config1_and_wire_loop_counts():
    m, c = _circ(W.config1_bar())
    assert c.nloop == 3000 - 1970 + 1 + 1 == 1032
    m, c = _circ(W.config2_wires())
    assert c.ncomp == 8 and c.nport == 8
    assert c.nloop == 59904 - (39936 - 8 * 22) + 8 + 8 == 20160


def test_loop_matrix_rows_are_cycles_and_independent():
    """Every fundamental loop is a closed cycle (N A^T = 0, with N the
    node-branch incidence), the loops are independent (rank l) and complete
    (l = b - n' + s + p)."""
    s = W.paper_bar_e1()
    m, c = _circ(s)
    A = c.loop_matrix()
    N = c.incidence()
    assert abs(N @ A.T).max() == 0
    assert np.linalg.matrix_rank(A.toarray()) == c.nloop
    assert c.nloop == c.nbranch - len(c.nodes) + c.ncomp


def test_loop_dimension_is_about_20_percent_of_mna():
    """Sec. III-B: for closed surfaces the loop system is ~20% of MNA (b + n)."""
    s = W.config2_wires()
    m, c = _circ(s)
    ratio = c.nloop / (m.nedge + m.ntri)
    assert 0.19 < ratio < 0.21


def test_source_links_are_never_twigs():
    m, c = _circ(W.config2_wires())
    assert not c.twig[m.nedge:].any()
    assert np.all(c.links[c.port_loop] == m.nedge + np.arange(8))


def test_invalid_topologies_raise():
    s = W.config1_bar()
    src, snk = s.ports[0]
    m = RWGMesh(s.V, s.T)
    with pytest.raises(ValueError):
        Circuit(m, [(src, np.concatenate([snk, src[:1]]))])      # overlapping contacts
    w = W.bond_wires(nwire=2, nseg=6)
    mw = RWGMesh(w.V, w.T)
    with pytest.raises(ValueError):
        Circuit(mw, [(w.ports[0][0], w.ports[1][1])])            # different conductors
    with pytest.raises(ValueError):
        RWGMesh(s.V, s.T[:-1])                                    # open surface
