"""Dense loop-space system, direct solve and R/L extraction (oracle, FP64).

* Eq. Zb: Z_b = Z_s G + (j omega mu / 4 pi) K, with G the Gram matrix of the
  basis and K the dense 1/|r - r'| matrix (the sparse term is the one with
  Z_s, the dense term the inductive one).
* Eq. ImpedanceOp: Z_s = sqrt(j omega mu / sigma), principal root
  (1 + j) sqrt(omega mu / (2 sigma)), e^{j omega t} convention, mu = mu0.
* Eq. LoopVandI / FinalME: Z_l = A Z_b A^T, V_l = e_(loop of port k) x 1 V.
* Sec. V: ports excited in turn (others shorted) give the admittance matrix
  Y[j, k] = I_l[loop of port j]; Z = Y^-1, R = Re Z, L = Im Z / omega; loop
  quantities R_o = R11 - 2 R12 + R22 (and likewise L_o).
* Eq. Precond: P = A Z_b^N A^T with Z_b^N the diagonal of Z_b (source
  branches: 0), applied as a dense inverse here.
"""
import numpy as np
import scipy.linalg as sla

MU0 = 4e-7 * np.pi


def surface_impedance(omega, sigma, mu_r=1.0):
    return (1.0 + 1.0j) * np.sqrt(omega * MU0 * mu_r / (2.0 * sigma))


def triangle_impedance(mesh, circuit, zs, contact_zs=False):
    """Per-triangle surface impedance: zs everywhere, 0 on contact faces
    unless ``contact_zs`` (ideal terminals by default)."""
    w = np.full(mesh.ntri, zs, dtype=np.complex128)
    if not contact_zs:
        w[circuit.contact] = 0.0
    return w


def branch_impedance(G_tri_weighted, K, omega, mu_r, nport):
    """Dense (b + p) x (b + p) Z_b; source branches have zero rows/cols."""
    b = K.shape[0]
    Z = np.zeros((b + nport, b + nport), dtype=np.complex128)
    Z[:b, :b] = G_tri_weighted + 1j * omega * MU0 * mu_r / (4.0 * np.pi) * K
    return Z


def loop_impedance(A, Zb):
    A = A.toarray() if hasattr(A, "toarray") else A
    return A @ Zb @ A.T


def port_admittance(Zl, port_loop):
    p = len(port_loop)
    V = np.zeros((Zl.shape[0], p), dtype=np.complex128)
    V[port_loop, np.arange(p)] = 1.0
    lu = sla.lu_factor(Zl)
    I = sla.lu_solve(lu, V)
    return I[port_loop, :], I


def extract_rl(Y, omega):
    Z = np.linalg.inv(Y)
    return Z.real, Z.imag / omega, Z


def loop_rl(R, L):
    return (R[0, 0] - 2 * R[0, 1] + R[1, 1]), (L[0, 0] - 2 * L[0, 1] + L[1, 1])


def precond_dense(A, Zb):
    """P = A diag(Z_b) A^T as a dense matrix."""
    A = A.toarray() if hasattr(A, "toarray") else A
    return (A * np.diag(Zb)[None, :]) @ A.T


def gmres(matvec, b, M=None, tol=1e-6, restart=60, maxit=1000, right=True):
    """Plain restarted GMRES with modified Gram-Schmidt and Givens rotations.
    ``M`` is the preconditioner application (right-preconditioned by default,
    so the monitored residual is the true residual; ``right=False`` gives the
    left-preconditioned form of Eq. LoopWithP, monitoring |M r|/|M b|).
    Returns (x, iterations, history of relative residuals)."""
    n = b.shape[0]
    M = M or (lambda v: v)
    x = np.zeros(n, dtype=np.complex128)
    bnorm = np.linalg.norm(b if right else M(b))
    hist = []
    it = 0
    while it < maxit:
        r = b - matvec(x)
        if not right:
            r = M(r)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol:
            break
        V = np.zeros((n, restart + 1), dtype=np.complex128)
        Z = np.zeros((n, restart), dtype=np.complex128)
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart, dtype=np.complex128)
        sn = np.zeros(restart, dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        g[0] = beta
        V[:, 0] = r / beta
        k_done = 0
        for k in range(restart):
            if right:
                Z[:, k] = M(V[:, k])
                w = matvec(Z[:, k])
            else:
                w = M(matvec(V[:, k]))
            for j in range(k + 1):
                H[j, k] = np.vdot(V[:, j], w)
                w = w - H[j, k] * V[:, j]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] != 0:
                V[:, k + 1] = w / H[k + 1, k]
            # rotation (x, y) -> (conj(c) x + conj(s) y, -s x + c y)
            for j in range(k):
                t = np.conj(cs[j]) * H[j, k] + np.conj(sn[j]) * H[j + 1, k]
                H[j + 1, k] = -sn[j] * H[j, k] + cs[j] * H[j + 1, k]
                H[j, k] = t
            den = np.sqrt(abs(H[k, k]) ** 2 + abs(H[k + 1, k]) ** 2)
            cs[k] = H[k, k] / den
            sn[k] = H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = np.conj(cs[k]) * g[k]
            it += 1
            k_done = k + 1
            hist.append(abs(g[k + 1]) / bnorm)
            if hist[-1] <= tol or it >= maxit:
                break
        y = sla.solve_triangular(H[:k_done, :k_done], g[:k_done])
        if right:
            x = x + Z[:, :k_done] @ y
        else:
            x = x + V[:, :k_done] @ y
        if hist and hist[-1] <= tol:
            break
    return x, it, hist
