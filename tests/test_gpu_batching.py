"""Batched execution: multi-RHS solves, HIP-graph replay and the autotuner.

* One solve_ports call over several frequencies gives the same admittances as
  one call per frequency (each right-hand side has its own Krylov space).
* FGMRES with the product and P^-1 replayed as HIP graphs reproduces the eager
  solve bit for bit (every replay is checked, with eager Gram-Schmidt work
  and host synchronisation between replays).
* Every plan value gives the same product to FP32 accuracy, and the
  autotuner keeps valid choices.
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu


@pytest.fixture(scope="module")
def wires():
    return W.bond_wires(nwire=2, nseg=24, span=0.4e-3, height=80e-6)


def _ctx(s, **kw):
    import paper_2210_04891_amd as P
    return P.Context(s, (32, 32, 16), near_kappa=1.5, grid_fp64=False, **kw)


@gpu
def test_graph_replay_matches_eager(wires):
    f = np.array([1e8, 2e9, 1.5e10])
    ctx = _ctx(wires)
    assert ctx.get_option("graphs") == 1
    Yg, itg, rrg, cg = ctx.solve_ports(f, tol=1e-6, maxit=200, restart=30, precond=1)
    ctx.set_option("graphs", 0)
    Ye, ite, rre, ce = ctx.solve_ports(f, tol=1e-6, maxit=200, restart=30, precond=1)
    assert cg == 0 and ce == 0
    assert itg.min() >= 5                      # several replays of each graph
    assert np.array_equal(itg, ite) and np.array_equal(Yg, Ye) and np.array_equal(rrg, rre)
    # a second graph solve in the same context (fresh capture) agrees too
    ctx.set_option("graphs", 1)
    Y2, it2, rr2, c2 = ctx.solve_ports(f, tol=1e-6, maxit=200, restart=30, precond=1)
    assert np.array_equal(Y2, Ye) and np.array_equal(it2, ite)


@gpu
def test_batched_sweep_matches_per_frequency(wires):
    f = np.array([3e8, 4e9, 2e10])
    ctx = _ctx(wires)
    Yb, itb, _, cb = ctx.solve_ports(f, tol=1e-7, maxit=200, restart=60, precond=1)
    assert cb == 0
    for k, fk in enumerate(f):
        Y1, it1, _, c1 = ctx.solve_ports([fk], tol=1e-7, maxit=200, restart=60, precond=1)
        assert c1 == 0
        assert np.abs(Y1[0] - Yb[k]).max() <= 1e-12 * np.abs(Yb[k]).max()


@gpu
def test_plans_agree_and_autotune(wires):
    import paper_2210_04891_amd as P
    ctx = _ctx(wires)
    l = ctx.sizes["l"]
    # 20 right-hand sides: the tiled near-field product runs (two chunks,
    # the second ragged)
    om = 2 * np.pi * np.repeat(np.array([1e9, 1e10]), 10)
    x = torch.from_numpy(W.complex_normal(31, (om.size, l))).cuda()
    ref = ctx.matvec(x, omega=om, flags=P.PFFT_PRECOND).cpu().numpy()
    for name in ("fft_plan", "ldl_plan", "project_plan", "project_rhs", "combine_plan", "stream_split",
                 "near_dense"):
        ctx.set_option(name, 1 - ctx.get_option(name))
        y = ctx.matvec(x, omega=om, flags=P.PFFT_PRECOND).cpu().numpy()
        ctx.set_option(name, 1 - ctx.get_option(name))
        assert np.linalg.norm(y - ref) <= 2e-6 * np.linalg.norm(ref), name
    rep = ctx.autotune(om, reps=2)
    for name in ("fft_plan", "ldl_plan", "project_plan", "project_rhs", "combine_plan", "stream_split",
                 "near_dense"):
        assert rep[name]["chosen"] in (0, 1)
        assert ctx.get_option(name) == rep[name]["chosen"]
        assert rep[name]["0"] > 0 and rep[name]["1"] > 0
    y = ctx.matvec(x, omega=om, flags=P.PFFT_PRECOND).cpu().numpy()
    assert np.linalg.norm(y - ref) <= 2e-6 * np.linalg.norm(ref)


@gpu
def test_stream_split_matches_one_stream(wires):
    """The right-hand sides of a product split over two streams give the same
    result bit for bit (every kernel treats right-hand sides independently)."""
    import paper_2210_04891_amd as P
    ctx = _ctx(wires)
    l = ctx.sizes["l"]
    om = 2 * np.pi * np.repeat(np.array([1e8, 1e9, 1e10, 3e10]), 3)
    x = torch.from_numpy(W.complex_normal(41, (om.size, l))).cuda()
    assert ctx.get_option("stream_split") == 0
    ctx.set_option("stream_split", 1)
    a = ctx.matvec(x, omega=om, flags=P.PFFT_PRECOND).cpu().numpy()
    ctx.set_option("stream_split", 0)
    b = ctx.matvec(x, omega=om, flags=P.PFFT_PRECOND).cpu().numpy()
    assert np.array_equal(a, b)
    f = np.array([2e9, 2e10])
    Y0, it0, _, _ = ctx.solve_ports(f, tol=1e-7, maxit=200, restart=60)
    ctx.set_option("stream_split", 1)
    Y1, it1, _, _ = ctx.solve_ports(f, tol=1e-7, maxit=200, restart=60)
    assert np.array_equal(Y0, Y1) and np.array_equal(it0, it1)


@gpu
def test_pruned_fft_matches_dense(wires):
    """The pruned FFT passes (only stencil nodes read and written) give the
    dense passes' product bit for bit: the nodes they skip hold exact zeros on
    the way in and are never read on the way out.  Checked on the far-field
    product alone and on the preconditioned loop product, with a dense call
    between two pruned ones (the pruned path must not depend on what the
    dense one left in the grid buffers, nor the other way round)."""
    import paper_2210_04891_amd as P
    ctx = _ctx(wires)
    assert ctx.get_option("fft_prune") == 1
    b, l = ctx.sizes["b"], ctx.sizes["l"]
    xb = torch.from_numpy(W.complex_normal(51, (12, b))).cuda()
    om = 2 * np.pi * np.repeat(np.array([1e8, 1e9, 1e10, 3e10]), 3)
    xl = torch.from_numpy(W.complex_normal(52, (om.size, l))).cuda()
    far1 = ctx.matvec(xb, space=0, flags=P.PFFT_FAR_ONLY).cpu().numpy()
    loop1 = ctx.matvec(xl, omega=om, flags=P.PFFT_PRECOND).cpu().numpy()
    ctx.set_option("fft_prune", 0)
    far0 = ctx.matvec(xb, space=0, flags=P.PFFT_FAR_ONLY).cpu().numpy()
    loop0 = ctx.matvec(xl, omega=om, flags=P.PFFT_PRECOND).cpu().numpy()
    ctx.set_option("fft_prune", 1)
    far2 = ctx.matvec(xb, space=0, flags=P.PFFT_FAR_ONLY).cpu().numpy()
    assert np.abs(far0).max() > 0
    assert np.array_equal(far1, far0) and np.array_equal(far2, far0)
    assert np.array_equal(loop1, loop0)


@gpu
def test_option_errors(wires):
    import paper_2210_04891_amd as P
    ctx = _ctx(wires)
    with pytest.raises(P.PfftError):
        ctx.set_option("no_such_plan", 1)
    with pytest.raises(P.PfftError):
        ctx.set_option("fft_plan", 2)
    with pytest.raises(P.PfftError):
        ctx.get_option("no_such_plan")


@gpu
def test_projection_rhs_groups_same_bits(wires):
    """The tiled projection with 16 or 8 right-hand sides per workgroup sums
    every node in the same order: the far field is the same bit for bit."""
    import paper_2210_04891_amd as P
    ctx = _ctx(wires)
    b = ctx.sizes["b"]
    x = torch.from_numpy(W.complex_normal(33, (21, b))).cuda()
    ref = ctx.matvec(x, space=0, flags=P.PFFT_FAR_ONLY).cpu().numpy()
    ctx.set_option("project_rhs", 1 - ctx.get_option("project_rhs"))
    y = ctx.matvec(x, space=0, flags=P.PFFT_FAR_ONLY).cpu().numpy()
    assert np.array_equal(y, ref)
