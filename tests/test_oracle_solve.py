"""Pins for the oracle's dense solve and R/L extraction (Sec. II-C, III, IV-A, V)."""
import numpy as np
import pytest

import workloads as W
from oracle.mesh import RWGMesh, gram_matrix
from oracle.circuit import Circuit
from oracle import integrals as I, solve as S
from test_oracle_integrals import tube_kernel_energy

SIGMA = 5.8e7


def solve_rl(mesh, circ, K, f, zs, contact_zs=False):
    om = 2 * np.pi * f
    wt = S.triangle_impedance(mesh, circ, zs, contact_zs)
    G = gram_matrix(mesh, weight=wt).toarray()
    Zb = S.branch_impedance(G, K, om, 1.0, circ.nport)
    Zl = S.loop_impedance(circ.loop_matrix(), Zb)
    Y, _ = S.port_admittance(Zl, circ.port_loop)
    R, L, Z = S.extract_rl(Y, om)
    return R, L, Z, Zl, Zb


def test_dc_resistance_limit(c1):
    """Real constant surface resistance r_s = rho P / A_cs with ideal
    contacts, omega -> 0: uniform axial current is in the basis span and the
    Galerkin solution is exact, so Re Z = r_s l / P = rho l / A = 0.0862069 Ohm
    (1 mm x 20 um x 10 um copper)."""
    w, t, ell = 20e-6, 10e-6, 1e-3
    P = 2 * (w + t)
    rs = P / (SIGMA * w * t)
    R, L, *_ = solve_rl(c1["mesh"], c1["circ"], c1["K"], 150.0, rs)
    assert R[0, 0] == pytest.approx(ell / (SIGMA * w * t), rel=1e-10)
    assert R[0, 0] == pytest.approx(0.0862069, rel=1e-6)


def test_low_frequency_inductance_matches_tube_closed_form(c1):
    """With the resistive (uniform) current, Im Z / omega equals the partial
    self-inductance of a uniform-surface-current tube, (mu0/4 pi P^2) times
    the strip integrals, up to the end-face currents (well below 0.5%)."""
    w, t, ell = 20e-6, 10e-6, 1e-3
    P = 2 * (w + t)
    rs = P / (SIGMA * w * t)
    R, L, *_ = solve_rl(c1["mesh"], c1["circ"], c1["K"], 150.0, rs)
    L_tube = 1e-7 * tube_kernel_energy(ell, w, t)
    assert L[0, 0] == pytest.approx(L_tube, rel=5e-3)
    assert L[0, 0] == pytest.approx(L_tube, rel=1e-4)


def test_high_frequency_resistance_bound_and_passivity(c1):
    """Re Z >= Re(Z_s) l / P (Cauchy-Schwarz on the Gram energy under the
    unit-current constraint), Re Z > 0, Im Z > 0 at 1 GHz."""
    P, ell = 60e-6, 1e-3
    zs = S.surface_impedance(2 * np.pi * 1e9, SIGMA)
    R, L, Z, *_ = solve_rl(c1["mesh"], c1["circ"], c1["K"], 1e9, zs)
    assert R[0, 0] >= zs.real * ell / P
    assert R[0, 0] > 0 and L[0, 0] > 0


@pytest.fixture(scope="module")
def two_wires():
    s = W.bond_wires(nwire=2, nseg=20, span=0.3e-3, height=60e-6)
    m = RWGMesh(s.V, s.T)
    c = Circuit(m, s.ports)
    K = I.kernel_dense(m)
    return s, m, c, K


def test_reciprocity_and_passivity_two_ports(two_wires):
    """Z_l = A Z_b A^T is complex symmetric, so Z_12 = Z_21; the resistance
    and inductance matrices are positive definite."""
    s, m, c, K = two_wires
    zs = S.surface_impedance(2 * np.pi * 5e9, SIGMA)
    R, L, Z, Zl, _ = solve_rl(m, c, K, 5e9, zs)
    assert abs(Z[0, 1] - Z[1, 0]) <= 1e-12 * abs(Z).max()
    assert np.all(np.linalg.eigvalsh(0.5 * (R + R.T)) > 0)
    assert np.all(np.linalg.eigvalsh(0.5 * (L + L.T)) > 0)
    assert abs(Z[0, 1]) < abs(Z[0, 0])


def test_invariance_to_relabelling():
    """R and L do not depend on the triangle numbering, which changes the
    edge orientations (T+ = lower index), the spanning tree and the loops."""
    s = W.paper_bar_e1()
    rng = np.random.default_rng(4)
    perm = rng.permutation(s.n)
    inv = np.argsort(perm)
    out = []
    for T, ports in ((s.T, s.ports), (s.T[perm], [(inv[a], inv[b]) for a, b in s.ports])):
        m = RWGMesh(s.V, T)
        c = Circuit(m, ports)
        K = I.kernel_dense(m)
        zs = S.surface_impedance(2 * np.pi * 50e9, SIGMA)
        R, L, *_ = solve_rl(m, c, K, 50e9, zs)
        out.append((R[0, 0], L[0, 0]))
    assert out[0][0] == pytest.approx(out[1][0], rel=1e-10)
    assert out[0][1] == pytest.approx(out[1][1], rel=1e-10)


def test_preconditioner_cuts_iterations(c1):
    """Eq. Precond with left preconditioning (Eq. LoopWithP) at tol 1e-3:
    several times fewer GMRES iterations than without it (Sec. V-A reports
    about one order of magnitude for large meshes)."""
    zs = S.surface_impedance(2 * np.pi * 1e9, SIGMA)
    R, L, Z, Zl, Zb = solve_rl(c1["mesh"], c1["circ"], c1["K"], 1e9, zs)
    V = np.zeros(Zl.shape[0], complex)
    V[c1["circ"].port_loop[0]] = 1.0
    Pinv = np.linalg.inv(S.precond_dense(c1["circ"].loop_matrix(), Zb))
    _, it0, _ = S.gmres(lambda v: Zl @ v, V, None, tol=1e-3, restart=200, right=False)
    _, it1, _ = S.gmres(lambda v: Zl @ v, V, lambda v: Pinv @ v, tol=1e-3, restart=200, right=False)
    assert it1 * 3 <= it0


def test_gmres_reaches_direct_solution(c1):
    zs = S.surface_impedance(2 * np.pi * 1e9, SIGMA)
    *_, Zl, Zb = solve_rl(c1["mesh"], c1["circ"], c1["K"], 1e9, zs)
    V = np.zeros(Zl.shape[0], complex)
    V[c1["circ"].port_loop[0]] = 1.0
    Pinv = np.linalg.inv(S.precond_dense(c1["circ"].loop_matrix(), Zb))
    x, it, hist = S.gmres(lambda v: Zl @ v, V, lambda v: Pinv @ v, tol=1e-10, restart=15)
    assert np.linalg.norm(Zl @ x - V) <= 1e-9 * np.linalg.norm(V)
    assert np.linalg.norm(x - np.linalg.solve(Zl, V)) <= 1e-6 * np.linalg.norm(x)


def test_surface_impedance_principal_root():
    """Eq. ImpedanceOp: Z_s^2 = j omega mu / sigma, principal root (Re > 0)."""
    om = 2 * np.pi * 1e9
    zs = S.surface_impedance(om, SIGMA)
    assert zs * zs == pytest.approx(1j * om * S.MU0 / SIGMA, rel=1e-14)
    assert zs.real > 0 and zs.imag == pytest.approx(zs.real)


@pytest.mark.parametrize("right", [True, False])
def test_gmres_terminates_on_distinct_eigenvalues(right):
    """A diagonalisable matrix with k distinct eigenvalues has a minimal
    polynomial of degree k, so (full) GMRES reaches the exact solution in k
    steps whatever b is; the residual history never increases."""
    rng = np.random.default_rng(3)
    n, k = 40, 5
    lam = np.array([1.0, 2.0 + 1j, -3.0, 0.5j, 4.0 - 2j])
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)))
    D = lam[np.arange(n) % k]
    Am = (Q * D) @ Q.conj().T
    b = rng.normal(size=n) + 1j * rng.normal(size=n)
    x, it, hist = S.gmres(lambda v: Am @ v, b, None, tol=1e-12, restart=n, right=right)
    assert it == k
    assert np.all(np.diff(hist) <= 1e-14)
    assert np.linalg.norm(Am @ x - b) <= 1e-10 * np.linalg.norm(b)


def test_left_gmres_monitors_preconditioned_residual():
    """Left preconditioning (Eq. LoopWithP): the stopping quantity is
    |M (b - A x)| / |M b|, recomputed here from the returned iterate; with M
    the exact inverse the first step solves the system."""
    rng = np.random.default_rng(5)
    n = 30
    Am = np.eye(n) * 4 + rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    Md = np.diag(1.0 / np.diag(Am))
    b = rng.normal(size=n) + 0j
    x, it, hist = S.gmres(lambda v: Am @ v, b, lambda v: Md @ v, tol=1e-3, restart=n, right=False)
    pres = np.linalg.norm(Md @ (b - Am @ x)) / np.linalg.norm(Md @ b)
    assert hist[-1] <= 1e-3 and pres == pytest.approx(hist[-1], rel=1e-8)
    assert len(hist) == it and (it == 1 or hist[-2] > 1e-3)
    Ainv = np.linalg.inv(Am)
    x1, it1, _ = S.gmres(lambda v: Am @ v, b, lambda v: Ainv @ v, tol=1e-10, restart=n, right=False)
    assert it1 == 1 and np.linalg.norm(x1 - Ainv @ b) <= 1e-10 * np.linalg.norm(x1)
