"""FFT-convolution plans against the oracle's FP64 grid product.

The plane stage (Y, Z with the spectrum, inverse Z, inverse Y) has these
implementations: register-resident lines with even/odd half transforms
(planes up to 64 x 32), the big-plane kernel for 256 x 32 and 512 x 16
planes (the package-trace and PDN shapes: four-step y transforms, one
workgroup half per even/odd y half), unfused passes, and LDS Stockham passes
(option fft_plan = 1).  Each must reproduce the oracle's explicit
B^T (H * (B alpha)) to FP32 accuracy, on small grids and on the bench grid
(256 x 64 x 32, 39,936 triangles), and agree with the Stockham plan, as a
whole-vector 2-norm and entry by entry (relative to the largest entry).
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu


def _far(ctx, X, plan):
    import paper_2210_04891_amd as P
    ctx.set_option("fft_plan", 1 if plan == "lds" else 0)
    return ctx.matvec(torch.from_numpy(X).cuda(), space=0, flags=P.PFFT_FAR_ONLY).cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@gpu
@pytest.mark.parametrize("case", ["two_wires_32x32x16", "two_wires_64x32x16", "two_wires_128x16x16",
                                  "two_wires_64x16x8", "two_wires_32x256x32", "two_wires_16x512x16",
                                  "bond_wires_256x64x32"])
def test_plane_plans_match_oracle(case):
    import paper_2210_04891_amd as P
    from oracle.mesh import RWGMesh
    from oracle import pfft as PF
    if case.startswith("two"):
        grid = tuple(int(v) for v in case.split("_")[-1].split("x"))
        s, nrhs, tol = W.bond_wires(nwire=2, nseg=24, span=0.4e-3, height=80e-6), 3, 2e-6
    else:
        s, grid, nrhs, tol = W.config2_wires(), (256, 64, 32), 2, 5e-6
    m = RWGMesh(s.V, s.T)
    op = PF.PFFTOperator(m, grid, 4, 1.5, with_near=False)
    ctx = P.Context(s, grid, near_kappa=1.5, grid_fp64=False)
    X = W.complex_normal(21, (nrhs, m.nedge))
    y_reg = _far(ctx, X, "register")
    ctx.set_option("fft_prune", 0)
    y_dense = _far(ctx, X, "register")
    ctx.set_option("fft_prune", 1)
    # the pruned passes skip only zeros: same bits
    assert np.array_equal(y_reg, y_dense)
    y_lds = _far(ctx, X, "lds")
    for r in range(nrhs):
        ref = op.far(X[r])
        assert _rel(y_reg[r], ref) < tol
        assert _rel(y_lds[r], ref) < tol
        assert np.abs(y_reg[r] - ref).max() < 10 * tol * np.abs(ref).max()
    assert _rel(y_reg, y_lds) < tol
