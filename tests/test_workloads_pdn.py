"""The plane-and-via generator: closed, consistently outward-oriented
2-manifold surfaces whose genus is the via count minus one (two slabs joined
by k tubes), with the enclosed volume of two slabs plus k prism barrels, and
port patches of the stated size on the outer faces."""
import numpy as np

import workloads as W


def _check(s, nvia):
    V, T = s.V, s.T
    e = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]])
    und, cnt = np.unique(np.sort(e, axis=1), axis=0, return_counts=True)
    assert np.all(cnt == 2)                                   # closed 2-manifold
    assert np.unique(e, axis=0).shape[0] == e.shape[0]        # each directed edge once: consistent orientation
    chi = V.shape[0] - und.shape[0] + T.shape[0]
    assert chi == 2 - 2 * (nvia - 1)
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    assert np.all(0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1) > 0)
    vol = np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0   # > 0 for outward triangles
    p = s.params
    L = p["nx"] * p["cell"]
    ngon = 0.5 * p["nfacet"] * p["radius"] ** 2 * np.sin(2 * np.pi / p["nfacet"])
    assert abs(vol - (2 * L * L * p["thick"] + nvia * ngon * p["gap"])) <= 1e-9 * vol


def test_small_pdn_is_a_closed_oriented_surface_of_genus_one():
    s = W.pdn(nx=10, ny=10, cell=100e-6, vias=[(2, 2), (6, 6)], block=2, ports=[(1, 6), (6, 1)], patch=2)
    _check(s, 2)
    for src, snk in s.ports:
        assert len(src) == len(snk) == 8                      # 2 x 2 cells, two triangles each
        assert np.all(s.V[s.T[src]][:, :, 2] == s.V[:, 2].max())
        assert np.all(s.V[s.T[snk]][:, :, 2] == 0.0)


def test_config4_pdn_size_and_genus():
    s = W.config4_pdn()
    assert s.n == 995_200
    _check(s, 100)
    assert len(s.ports) == 16 and all(len(a) == len(b) == 32 for a, b in s.ports)
