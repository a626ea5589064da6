"""Post-processing of solved loop currents (oracle, FP64; test infrastructure).

Sec. V-A: once the loop currents are known, the branch currents follow from
Eq. CurT and the branch voltages from Eq. BranchVandI; with the potential of
the sink faces set to zero, the potential of every triangular panel follows
from the branch voltages.

* Eq. CurT: I_b = A^T I_l (mesh branches, then the port source branches).
* Eq. BranchVandI: V_b = Z_b I_b.
* Eq. Vb: a mesh branch's voltage is the potential of its T+ node minus the
  potential of its T- node.  Where the loop equations hold these
  differences are consistent, so the node potentials are the least-squares
  solution of (phi_u - phi_v = V_b(e)) over all mesh branches, written here
  without any spanning tree.  Reading: each conductor's reference node (0 V)
  is the sink face of its lowest-numbered port, or its lowest node when it
  carries no port.
* Eqs. ExpandJ and RWG: the surface current density at the centroid of a
  triangle is the sum over its three edges of I_e f_e(centroid).
"""
import numpy as np


def branch_currents(A, I_l):
    """Eq. CurT."""
    return A.T @ I_l


def branch_voltages(Zb, I_b):
    """Eq. BranchVandI."""
    return Zb @ I_b


def reference_nodes(circuit):
    """Reference node of every conductor (component id -> node id)."""
    ref = {}
    for k in range(circuit.nport):
        c = circuit.comp[circuit.port_snk_node[k]]
        ref.setdefault(c, circuit.port_snk_node[k])
    for x in circuit.nodes:
        c = circuit.comp[int(x)]
        if c not in ref:
            ref[c] = int(x)
    return ref


def node_potentials(circuit, V_b):
    """Node id -> potential, from the mesh-branch voltages by least squares
    per conductor with its reference node at 0 V."""
    ref = reference_nodes(circuit)
    phi = {}
    for c in range(circuit.ncomp):
        nodes = [int(x) for x in circuit.nodes if circuit.comp[int(x)] == c]
        free = [x for x in nodes if x != ref[c]]
        col = {x: i for i, x in enumerate(free)}
        rows, rhs = [], []
        for e in range(circuit.nmesh_branch):
            u, v = int(circuit.branch_u[e]), int(circuit.branch_v[e])
            if u == v or circuit.comp[u] != c:
                continue
            r = np.zeros(len(free), dtype=np.complex128)
            if u in col:
                r[col[u]] += 1.0
            if v in col:
                r[col[v]] -= 1.0
            rows.append(r)
            rhs.append(V_b[e])
        phi[ref[c]] = 0.0 + 0.0j
        if free:
            sol = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)[0]
            for x, i in col.items():
                phi[x] = sol[i]
    return phi


def panel_potentials(circuit, V_b):
    """Potential of every triangle (its node's potential)."""
    phi = node_potentials(circuit, V_b)
    return np.array([phi[int(x)] for x in circuit.node_of_tri])


def centroid_current(mesh, I_mesh):
    """Surface current density (complex, A/m) at each triangle's centroid
    from the mesh-branch currents: f_e is (r - v+)/(2A+) on T+ and
    (v- - r)/(2A-) on T- (Eq. RWG), v+- the vertex opposite the edge."""
    J = np.zeros((mesh.ntri, 3), dtype=np.complex128)
    for t in range(mesh.ntri):
        c = mesh.centroid[t]
        for i in range(3):
            e = int(mesh.tri_edge[t, i])
            if mesh.tplus[e] == t:
                f = (c - mesh.V[mesh.vplus[e]]) / (2.0 * mesh.area[t])
            else:
                f = (mesh.V[mesh.vminus[e]] - c) / (2.0 * mesh.area[t])
            J[t] += I_mesh[e] * f
    return J
