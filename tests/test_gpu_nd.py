"""The preconditioner's nested-dissection path (Sec. IV-A, Eq. Precond; the
paper factors P with a sparse direct solver): supernodal LDL^T of the nodal
matrix on the host, forward and backward sweeps over the supernode levels on
the device.  It is chosen by itself when a conductor's band would be wider
than 256 (the PDN-like planes); here it is also forced (nd_plan 1) on
structures the band path handles, and the two must give the same P^-1 to
rounding; R and L with it match the dense oracle within 0.5%."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu


def _pdn_reduced():
    return W.pdn(nx=10, ny=10, cell=100e-6, vias=[(2, 2), (6, 6)], block=2, ports=[(1, 6), (6, 1)], patch=2)


@gpu
@pytest.mark.parametrize("case", ["bar", "wires", "pdn"])
def test_nd_solve_matches_band_solve(case):
    import paper_2210_04891_amd as P
    if case == "bar":
        s, grid = W.config1_bar(), (64, 8, 8)
    elif case == "wires":
        s, grid = W.bond_wires(nwire=3, nseg=30), (64, 32, 16)
    else:
        s, grid = _pdn_reduced(), (32, 32, 16)
    ctx = P.Context(s, grid, near_kappa=1.5, grid_fp64=False)
    l = ctx.sizes["l"]
    om = 2 * np.pi * np.repeat(np.array([1e8, 3e9, 2e10]), 3)
    Y = torch.from_numpy(W.complex_normal(51, (om.size, l))).cuda()
    assert ctx.get_option("nd_plan") == 0
    zb = ctx.matvec(Y, omega=om, space=1, flags=P.PFFT_PRECOND_ONLY).cpu().numpy()
    ctx.set_option("nd_plan", 1)
    zn = ctx.matvec(Y, omega=om, space=1, flags=P.PFFT_PRECOND_ONLY).cpu().numpy()
    for r in range(om.size):
        assert np.linalg.norm(zn[r] - zb[r]) <= 1e-11 * np.linalg.norm(zb[r]), r


@gpu
def test_nd_reduced_pdn_rl_match_oracle():
    import paper_2210_04891_amd as P
    from oracle.mesh import RWGMesh
    from oracle import integrals, solve as S
    from systems import oracle_system
    s = _pdn_reduced()
    m = RWGMesh(s.V, s.T)
    K = integrals.kernel_dense(m)
    _, c, _, A, Zb = oracle_system(s, K)
    f = np.array([1e9, 1e10])
    ctx = P.Context(s, (32, 32, 16), near_kappa=1.5, grid_fp64=False)
    ctx.set_option("nd_plan", 1)
    Y, it, rr, code = ctx.solve_ports(f, tol=1e-7, maxit=300, restart=60, precond=1)
    assert code == 0 and np.all(rr <= 1e-7)
    R, L = P.extract_RL(f, Y)
    for k in range(f.size):
        om = 2 * np.pi * f[k]
        Yo, _ = S.port_admittance(S.loop_impedance(A, Zb(om)), c.port_loop)
        Ro, Lo, _ = S.extract_rl(Yo, om)
        for i in range(2):
            for j in range(2):
                assert abs(R[k, i, j] - Ro[i, j]) <= 5e-3 * Ro[i, i], (k, i, j)
                assert abs(L[k, i, j] - Lo[i, j]) <= 5e-3 * Lo[i, i], (k, i, j)
