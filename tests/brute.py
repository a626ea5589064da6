"""Brute-force reference for triangle-pair integrals of 1/|r - r'| (tests
only; independent of the oracle's Sauter-Schwab cubature).

    M[i, j] = int_t int_t' (r - p_i).(r' - q_j) / |r - r'| dS' dS

The inner integral over t' is the classical closed form for a flat triangle
(the potentials V0 = int 1/R and V1 = int (r' - r)/R, from the surface
divergence theorem: each edge contributes a log and an arctangent term); the
outer integral over t is scipy's adaptive cubature on the unit square, mapped
onto t by the collapse (u, v) -> p0 + u (p1 - p0) + u v (p2 - p1), Jacobian
2 A u.  The places where the outer integrand is not smooth (the shared edge
or vertex, the edges of t itself for the same triangle) then lie on the
boundary of the square, where adaptive subdivision resolves them.
"""
import numpy as np
from scipy import integrate


def flat_triangle_potentials(r, Q):
    """V0 (m,) and V1 (m, 3) at points r (m, 3) for one triangle Q (3, 3)."""
    r = np.atleast_2d(r)
    e = np.roll(Q, -1, axis=0) - Q                       # edge i: Q[i] -> Q[i+1]
    nrm = np.cross(e[0], -e[2])
    nrm /= np.linalg.norm(nrm)
    elen = np.linalg.norm(e, axis=1)
    lhat = e / elen[:, None]
    uhat = np.cross(lhat, nrm)                           # in-plane normal of each edge
    h = (r - Q[0]) @ nrm                                 # signed height above the plane
    rho = r - h[:, None] * nrm[None, :]
    ah = np.abs(h)
    V0 = np.zeros(r.shape[0])
    W = np.zeros((r.shape[0], 3))
    for i in range(3):
        d = Q[i][None, :] - rho
        t0 = d @ uhat[i]
        s1 = d @ lhat[i]
        s2 = s1 + elen[i]
        R02 = t0 * t0 + h * h
        R1 = np.sqrt(R02 + s1 * s1)
        R2 = np.sqrt(R02 + s2 * s2)
        # log((R2 + s2)/(R1 + s1)); for negative s use R + s = R0^2/(R - s)
        with np.errstate(divide="ignore", invalid="ignore"):
            A2 = np.where(s2 > 0, R2 + s2, R02 / (R2 - s2))
            A1 = np.where(s1 > 0, R1 + s1, R02 / (R1 - s1))
            lg = np.log(A2 / A1)
            at = np.arctan2(t0 * s2, R02 + ah * R2) - np.arctan2(t0 * s1, R02 + ah * R1)
        on_line = R02 <= (1e-13 * elen[i]) ** 2
        lg = np.where(on_line, 0.0, lg)
        at = np.where(on_line, 0.0, at)
        V0 += t0 * lg - ah * at
        W += (0.5 * (R02 * lg + s2 * R2 - s1 * R1))[:, None] * uhat[i][None, :]
    V1 = W - (h * V0)[:, None] * nrm[None, :]
    return V0, V1


def pair_block(P, Q, rtol=1e-12):
    """3 x 3 raw block of the triangle pair (P outer, Q inner), vertex rows.
    The shared vertices must be P[0] (vertex) or P[0], P[1] (edge)."""
    A = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))

    def f(x):
        u, v = x[:, 0], x[:, 1]
        r = P[0] + u[:, None] * (P[1] - P[0]) + (u * v)[:, None] * (P[2] - P[1])
        V0, V1 = flat_triangle_potentials(r, Q)
        out = np.empty((r.shape[0], 9))
        for i in range(3):
            a = r - P[i]
            for j in range(3):
                inner = V1 + (r - Q[j]) * V0[:, None]
                out[:, 3 * i + j] = np.einsum("kd,kd->k", a, inner)
        return out * (2 * A * u)[:, None]

    res = integrate.cubature(f, [0.0, 0.0], [1.0, 1.0], rtol=rtol, atol=0.0, max_subdivisions=200000)
    assert res.status == "converged", res.status
    return res.estimate.reshape(3, 3)
