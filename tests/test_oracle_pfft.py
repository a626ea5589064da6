"""Pins for the oracle's pFFT steps (Sec. IV-B, Eqs. Projection, FFTCal,
interpolation, Lb)."""
import numpy as np
import pytest

import workloads as W
from oracle.mesh import RWGMesh
from oracle import pfft as PF, integrals as I


def test_fft_convolution_equals_direct_toeplitz_sum():
    """Eq. FFTCal: the zero-padded circulant FFT product equals the direct
    O(N^2) three-level Toeplitz sum on a small anisotropic grid."""
    V = np.array([[0, 0, 0], [7e-6, 3e-6, 2e-6]])
    g = PF.Grid(V, (9, 7, 6), 4)
    Q = np.random.default_rng(2).standard_normal((3, 9, 7, 6)) + 0j
    a = PF.convolve(g, Q)
    b = PF.convolve_direct(g, Q)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_grid_fits_every_stencil():
    s = W.config1_bar()
    m = RWGMesh(s.V, s.T)
    g = PF.Grid(m.V, (64, 8, 8), 4)
    a = g.anchor(m.centroid)
    u = (m.centroid - g.x0) / g.h
    assert np.all(a >= 0) and np.all(a + 4 <= g.dims)
    # the centroid sits between the 2nd and 3rd stencil nodes in every dimension
    assert np.all(u - a >= 1.0) and np.all(u - a < 2.0)


def test_projection_reproduces_low_moments():
    """Lagrange stencils reproduce polynomials up to degree 3 per dimension,
    so the grid currents of f_e carry the exact zeroth and first moments:
    sum_g B[(c,g),e] = int f_e,c and sum_g B[(c,g),e] x_g,d = int f_e,c r_d
    (integrands of degree <= 2, exact under the 7-point rule)."""
    s = W.config1_bar()
    m = RWGMesh(s.V, s.T)
    g = PF.Grid(m.V, (64, 8, 8), 4)
    B = PF.projection_matrix(m, g).toarray().reshape(3, -1, m.nedge)
    idx = np.stack(np.meshgrid(*[np.arange(d) for d in g.dims], indexing="ij"), -1).reshape(-1, 3)
    xg = g.x0 + idx * g.h
    lam, w = I.conical_rule(4)
    rng = np.random.default_rng(0)
    for e in rng.choice(m.nedge, 20, replace=False):
        m0 = np.zeros(3)
        m1 = np.zeros((3, 3))
        for t, sgn, v in ((m.tplus[e], 1, m.vplus[e]), (m.tminus[e], -1, m.vminus[e])):
            r = lam @ m.V[m.T[t]]
            f = sgn * (r - m.V[v]) / (2 * m.area[t])
            m0 += m.area[t] * (w @ f)
            m1 += m.area[t] * np.einsum('q,qc,qd->cd', w, f, r)
        assert np.allclose(B[:, :, e].sum(axis=1), m0, rtol=1e-10, atol=1e-20)
        assert np.allclose(B[:, :, e] @ xg, m1, rtol=1e-9, atol=1e-9 * np.abs(m1).max())


@pytest.fixture(scope="module")
def c1_pfft(c1):
    return PF.PFFTOperator(c1["mesh"], (64, 8, 8), 4, 1.5)


def test_pfft_matches_dense_kernel(c1, c1_pfft):
    """Eq. Lb at the config-1 grid (64 x 8 x 8, O_s = 4, kappa = 1.5):
    relative matvec error below 1e-3 against the dense FP64 kernel."""
    alpha = W.complex_normal(0, c1["mesh"].nedge)
    yd = c1["K"] @ alpha
    y = c1_pfft.apply(alpha)
    assert np.linalg.norm(y - yd) / np.linalg.norm(yd) < 1e-3


def test_pfft_error_falls_with_near_radius(c1):
    """Larger near-field radius -> more exact entries -> smaller error."""
    m, K = c1["mesh"], c1["K"]
    alpha = W.complex_normal(1, m.nedge)
    yd = K @ alpha
    errs = []
    for kappa in (0.75, 1.5):
        op = PF.PFFTOperator(m, (64, 8, 8), 4, kappa)
        errs.append(np.linalg.norm(op.apply(alpha) - yd) / np.linalg.norm(yd))
    assert errs[1] < errs[0]


def test_zero_offset_value_never_reaches_far_pairs():
    """H(0) is singular; every pair whose stencils share a node is near, so
    the value given to H(0) cancels between the grid and the pre-correction."""
    s = W.paper_bar_e1()
    m = RWGMesh(s.V, s.T)
    a = PF.PFFTOperator(m, (24, 6, 6), 4, 1.0, h0=0.0)
    b = PF.PFFTOperator(m, (24, 6, 6), 4, 1.0, h0=3.0 / 1e-6)
    x = W.complex_normal(3, m.nedge)
    ya, yb = a.apply(x), b.apply(x)
    assert np.linalg.norm(ya - yb) <= 1e-10 * np.linalg.norm(ya)


def test_near_pairs_are_exact():
    """For alpha supported on one edge e, rows e' whose triangle pairs with
    e's triangles are all near receive the exact kernel entries."""
    s = W.paper_bar_e1()
    m = RWGMesh(s.V, s.T)
    op = PF.PFFTOperator(m, (24, 6, 6), 4, 1.0)
    ti, tj = PF.near_pairs(m, op.grid, 1.0)
    near = set(zip(ti.tolist(), tj.tolist()))
    e = 100
    x = np.zeros(m.nedge, complex)
    x[e] = 1.0
    y = op.apply(x)
    Krow = I.kernel_rows(m, [e])[0]
    te = (m.tplus[e], m.tminus[e])
    checked = 0
    for e2 in range(m.nedge):
        t2 = (m.tplus[e2], m.tminus[e2])
        if all((a, b) in near for a in te for b in t2):
            assert y[e2].real == pytest.approx(Krow[e2], rel=1e-7, abs=1e-9 * abs(Krow).max())
            checked += 1
    assert checked > 20
