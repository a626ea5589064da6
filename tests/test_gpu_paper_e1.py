"""The Section V-A interconnect (5 um x 7.5 um x 200 um bar, 428 triangles,
230 loops) swept over 10-150 GHz, and the paper's solver form.

* Left-preconditioned GMRES (Eq. LoopWithP) at tol 1e-3: the GPU's iteration
  counts with and without P equal those of the oracle's textbook GMRES on
  the same pFFT operator (dense, FP64), and the GPU's iterate equals the
  oracle's iterate after that many steps.
* The sweep in one batched call: R and L within 0.5% of the dense oracle
  (exact kernel, direct solve); R rises and L falls with frequency (skin
  effect); P cuts the iteration count at every frequency (Fig. Case1_It).
"""
import numpy as np
import pytest

import workloads as W
from systems import oracle_system

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu

GRID = (32, 8, 8)
FREQS = np.linspace(10e9, 150e9, 8)


@pytest.fixture(scope="module")
def e1():
    from oracle import pfft as PF
    s = W.paper_bar_e1()
    m, c, K, A, Zb = oracle_system(s)
    op = PF.PFFTOperator(m, GRID, 4, 1.5)
    Kp = np.stack([op.apply(col) for col in np.eye(m.nedge)], axis=1).real
    Zbp = oracle_system(s, Kp)[4]
    return dict(s=s, m=m, c=c, A=A, Zb=Zb, Zbp=Zbp)


def _oracle_left_gmres(e1, f, precond, tol, restart, maxit):
    from oracle import solve as S
    om = 2 * np.pi * f
    Zl = S.loop_impedance(e1["A"], e1["Zbp"](om))
    b = np.zeros(Zl.shape[0], complex)
    b[e1["c"].port_loop[0]] = 1.0
    M = None
    if precond:
        Pinv = np.linalg.inv(S.precond_dense(e1["A"], e1["Zbp"](om)))
        M = lambda v: Pinv @ v      # noqa: E731
    return S.gmres(lambda v: Zl @ v, b, M, tol=tol, restart=restart, maxit=maxit, right=False)


@gpu
def test_e1_sizes():
    import paper_2210_04891_amd as P
    s = W.paper_bar_e1()
    ctx = P.Context(s, GRID, near_kappa=1.5, grid_fp64=True)
    assert s.T.shape[0] == 428 and ctx.sizes["l"] == 230 and ctx.nport == 1


@gpu
@pytest.mark.parametrize("precond", [1, 0])
def test_left_gmres_matches_oracle_iterations(e1, precond):
    """Same operator, same Krylov process: the GPU stops at the first step
    whose residual estimate is at most 0.9 tol (its margin for rounding in
    the product), so its count is the oracle's first step below 0.9 tol."""
    import paper_2210_04891_amd as P
    ctx = P.Context(e1["s"], GRID, near_kappa=1.5, grid_fp64=True)
    l = ctx.sizes["l"]
    tol = 1e-3
    Y, it, rr, code = ctx.solve_ports_lgmres(FREQS, tol=tol, maxit=l, restart=l, precond=precond)
    assert code == 0 and np.all(rr <= tol)
    for k, f in enumerate(FREQS):
        _, _, hist = _oracle_left_gmres(e1, f, precond, 1e-2 * tol, l, l)
        want = 1 + int(np.argmax(np.asarray(hist) <= 0.9 * tol))
        assert abs(int(it[k, 0]) - want) <= 1, (f, it[k, 0], want)
        x, itx, _ = _oracle_left_gmres(e1, f, precond, 1e-300, l, int(it[k, 0]))
        assert itx == it[k, 0]
        y0 = x[e1["c"].port_loop[0]]
        assert abs(Y[k, 0, 0] - y0) <= 1e-4 * abs(y0), f


@gpu
def test_left_gmres_reaches_tight_tolerance(e1):
    """At a tight tolerance the left form gives the same admittance as the
    right-preconditioned solver."""
    import paper_2210_04891_amd as P
    ctx = P.Context(e1["s"], GRID, near_kappa=1.5, grid_fp64=True)
    f = FREQS[[0, 7]]
    Yl, itl, rrl, cl = ctx.solve_ports_lgmres(f, tol=1e-9, maxit=300, restart=60, precond=1)
    Yr, itr, rrr, cr = ctx.solve_ports(f, tol=1e-9, maxit=300, restart=60, precond=1)
    assert cl == 0 and cr == 0
    assert np.abs(Yl - Yr).max() <= 1e-7 * np.abs(Yr).max()


@gpu
def test_e1_sweep_rl_matches_oracle(e1):
    """R and L over 10-150 GHz from one batched solve against the dense
    oracle with the exact kernel; skin effect: R up, L down with f."""
    import paper_2210_04891_amd as P
    from oracle import solve as S
    ctx = P.Context(e1["s"], GRID, near_kappa=1.5, grid_fp64=True)
    Y, it, rr, code = ctx.solve_ports(FREQS, tol=1e-6, maxit=300, restart=60, precond=1)
    assert code == 0 and np.all(rr <= 1e-6)
    R, L = P.extract_RL(FREQS, Y)
    for k, f in enumerate(FREQS):
        om = 2 * np.pi * f
        Zl = S.loop_impedance(e1["A"], e1["Zb"](om))
        Yo, _ = S.port_admittance(Zl, e1["c"].port_loop)
        Ro, Lo, _ = S.extract_rl(Yo, om)
        assert R[k, 0, 0] == pytest.approx(Ro[0, 0], rel=5e-3), f
        assert L[k, 0, 0] == pytest.approx(Lo[0, 0], rel=5e-3), f
    assert np.all(np.diff(R[:, 0, 0]) > 0)
    assert np.all(np.diff(L[:, 0, 0]) < 0)


@gpu
def test_e1_preconditioner_cuts_iterations_at_every_frequency(e1):
    """Fig. Case1_It, bottom: at tol 1e-3 the left-preconditioned solve
    needs fewer iterations than plain GMRES at every frequency."""
    import paper_2210_04891_amd as P
    ctx = P.Context(e1["s"], GRID, near_kappa=1.5, grid_fp64=True)
    l = ctx.sizes["l"]
    _, it1, _, c1 = ctx.solve_ports_lgmres(FREQS, tol=1e-3, maxit=l, restart=l, precond=1)
    _, it0, _, c0 = ctx.solve_ports_lgmres(FREQS, tol=1e-3, maxit=l, restart=l, precond=0)
    assert c1 == 0 and c0 == 0
    assert np.all(it1 < it0)


@gpu
def test_left_gmres_rejects_learned(e1):
    import paper_2210_04891_amd as P
    ctx = P.Context(e1["s"], GRID, near_kappa=1.5, grid_fp64=True)
    with pytest.raises(P.PfftError):
        ctx.solve_ports_lgmres([1e10], precond=2)
    with pytest.raises(P.PfftError):
        ctx.solve_ports_lgmres([1e10], tol=-1.0)
