"""pfft_matvec_noalloc: the product with the library's fixed scratch in place
of allocated workspaces, against pfft_matvec (same kernels, so the results
agree to rounding, here exactly), on two calls in a row with the second one
smaller, in branch and loop space; and the rejection of a problem whose one
right-hand side needs more than the scratch holds.  Run last: collection
order puts this module at the end."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu


def _check_pair(ctx, space, nrhs, seed, omega=None):
    dim = ctx.sizes["l"] if space == 1 else ctx.sizes["b"]
    X = torch.from_numpy(W.complex_normal(seed, (nrhs, dim))).cuda()
    ref = ctx.matvec(X, omega, space=space).cpu().numpy()
    got = ctx.matvec_noalloc(X, omega, space=space).cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err <= 1e-13, (space, nrhs, err)


@gpu
@pytest.mark.parametrize("fp64", [True, False])
def test_noalloc_matches_matvec(fp64):
    import paper_2210_04891_amd as P
    s = W.config1_bar()
    ctx = P.Context(s, (64, 8, 8), near_kappa=1.5, grid_fp64=fp64)
    for nrhs, seed in ((40, 3), (7, 4)):           # the second call smaller
        _check_pair(ctx, 0, nrhs, seed)
        om = 2 * np.pi * np.logspace(8, 10, nrhs)
        _check_pair(ctx, 1, nrhs, seed + 10, om)


@gpu
def test_noalloc_two_contexts_share_scratch():
    """Two contexts on one GPU, called alternately on one stream: each call
    rewrites the shared scratch (per-RHS coefficients included)."""
    import paper_2210_04891_amd as P
    a = P.Context(W.config1_bar(), (64, 8, 8), near_kappa=1.5, grid_fp64=False)
    b = P.Context(W.paper_bar_e1(), (32, 8, 8), near_kappa=1.5, grid_fp64=False)
    for k in range(2):
        om = 2 * np.pi * np.array([1e9, 3e9, 5e9][: 3 - k])
        _check_pair(a, 1, om.size, 30 + k, om)
        _check_pair(b, 1, om.size, 40 + k, om * 7)


@gpu
def test_noalloc_rejects_oversized_problem():
    import paper_2210_04891_amd as P
    s = W.paper_bar_e1()
    ctx = P.Context(s, (256, 64, 64), near_kappa=1.5, grid_fp64=True)   # one RHS: ~150 MB of grid scratch
    X = torch.from_numpy(W.complex_normal(5, (1, ctx.sizes["b"]))).cuda()
    with pytest.raises(P.PfftError) as ei:
        ctx.matvec_noalloc(X, space=0)
    assert ei.value.code == -3 and "scratch" in str(ei.value)
    with pytest.raises(P.PfftError) as ei:
        ctx.matvec_noalloc(torch.from_numpy(W.complex_normal(6, (1, ctx.sizes["l"]))).cuda(), [1e9],
                           space=1, flags=P.PFFT_PRECOND)
    assert ei.value.code == -1
