"""Oracle systems shared by the GPU solver tests: mesh, circuit, kernel matrix,
loop matrix and the branch impedance Z_b(omega) (Eq. Zb) of a structure."""
import numpy as np


def oracle_system(s, K=None):
    from oracle.mesh import RWGMesh, gram_matrix
    from oracle.circuit import Circuit
    from oracle import integrals as I, solve as S
    m = RWGMesh(s.V, s.T)
    c = Circuit(m, s.ports)
    if K is None:
        K = I.kernel_dense(m)
    A = c.loop_matrix().toarray()
    G = gram_matrix(m, weight=S.triangle_impedance(m, c, 1.0).real).toarray()

    def Zb(omega):
        zs = S.surface_impedance(omega, 5.8e7)
        Z = np.zeros((m.nedge + c.nport,) * 2, complex)
        Z[:m.nedge, :m.nedge] = zs * G + 1j * omega * S.MU0 / (4 * np.pi) * K
        return Z
    return m, c, K, A, Zb
