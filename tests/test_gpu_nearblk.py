"""Near-field pair blocks computed on the device (Sec. IV-B step 4, Eq. Lb).

pfft_setup computes every near pair's scaled (direct - grid) block on the
GPU, one thread per pair; the host-only model runs the same pair routine in
a host loop.  The two near-field matrices (and the diagonal of the direct K)
must agree to 1e-12 of their largest entry, on the bar and on the bond-wire
array (39,936 triangles, grid 256 x 64 x 32), with the same sparsity.
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
gpu = pytest.mark.gpu


def _compare(s, grid, kappa=1.5):
    import paper_2210_04891_amd as P
    h = P.HostModel(s, grid, stencil=4, near_kappa=kappa)
    ctx = P.Context(s, grid, stencil=4, near_kappa=kappa, grid_fp64=False)
    try:
        for name, dt in (("near_rowptr", np.int64), ("near_col", np.int32)):
            assert np.array_equal(h.get(name, dt), ctx.model_array(name, dt)), name
        for name in ("near_val", "kdiag"):
            a, b = h.get(name, np.float64), ctx.model_array(name, np.float64)
            assert a.shape == b.shape and a.size > 0
            assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max(), name
        ms = ctx.model_array("setup_ms", np.float64)
        assert ms.shape == (8,) and np.all(ms >= 0)
        print("setup ms (device context):", np.round(ms, 1).tolist(),
              "host-only model:", np.round(h.get("setup_ms", np.float64), 1).tolist())
    finally:
        h.close()
        ctx.close()


@gpu
def test_device_pair_blocks_match_host_bar():
    _compare(W.config1_bar(), (64, 8, 8))


@gpu
def test_device_pair_blocks_match_host_wires():
    _compare(W.config2_wires(), (256, 64, 32))
