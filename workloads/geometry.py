"""Seeded, deterministic surface-mesh generators for the synthetic workloads.

Every generator returns a :class:`Structure`: vertex coordinates in metres,
outward-oriented (counter-clockwise seen from outside) triangles, and one
(source, sink) pair of triangle-index sets per port.  The meshes are closed
2-manifolds, so every edge is shared by exactly two triangles.

The structures stand in for the paper's examples (Section V), whose exact
geometries are only shown in figures:

* ``config1_bar``   -- straight Cu bar 1 mm x 20 um x 10 um, 2,000 triangles.
* ``paper_bar_e1``  -- the Section V-A bar, 5 x 7.5 x 200 um, 428 triangles.
* ``prism``         -- the 8-triangle prism of Fig. 1.
* ``config2_wires`` -- 8 parabolic bond wires, 12-gon section, ~40k triangles.
* ``config3_traces``-- 32 Manhattan meander traces in 156.25 um lanes.
* ``config4_pdn``   -- two 10 x 10 mm planes joined by 100 vias, ~1 M triangles.
"""
from dataclasses import dataclass, field
import numpy as np


@dataclass
class Structure:
    name: str
    V: np.ndarray                 # (nv, 3) float64, metres
    T: np.ndarray                 # (n, 3) int32, outward CCW
    ports: list = field(default_factory=list)   # [(src_tris, snk_tris)] int32 arrays
    params: dict = field(default_factory=dict)

    @property
    def n(self):
        return int(self.T.shape[0])


class _VertexPool:
    """Assigns one vertex id per distinct integer key."""

    def __init__(self):
        self.ids = {}
        self.xyz = []

    def get(self, key, xyz):
        i = self.ids.get(key)
        if i is None:
            i = len(self.xyz)
            self.ids[key] = i
            self.xyz.append(np.asarray(xyz, dtype=np.float64))
        return i

    def array(self):
        return np.array(self.xyz, dtype=np.float64).reshape(-1, 3)


def _orient(V, tri, outward):
    a, b, c = (V[i] for i in tri)
    if np.dot(np.cross(b - a, c - a), outward) < 0.0:
        return (tri[0], tri[2], tri[1])
    return tuple(tri)


def box_bar(xs, ys, zs, split4=(), name="bar"):
    """Structured surface mesh of the box spanned by the node coordinates
    ``xs``, ``ys``, ``zs`` (1-D increasing arrays).  Each face cell is cut into
    two right triangles along its (low, low) -> (high, high) diagonal, except
    the cells listed in ``split4`` as (face, i, j), which get a centre vertex
    and four triangles.  Port 0 has the x = xs[0] face as source and the
    x = xs[-1] face as sink."""
    xs, ys, zs = (np.asarray(a, dtype=np.float64) for a in (xs, ys, zs))
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    pool = _VertexPool()
    tris, face_of = [], []
    split4 = set(split4)

    def P(i, j, k):
        return pool.get(("L", i, j, k), (xs[i], ys[j], zs[k]))

    # faces: (name, fixed axis, fixed index, outward normal, free axes)
    faces = [("y0", 1, 0, (0, -1, 0)), ("y1", 1, ny, (0, 1, 0)),
             ("z0", 2, 0, (0, 0, -1)), ("z1", 2, nz, (0, 0, 1)),
             ("x0", 0, 0, (-1, 0, 0)), ("x1", 0, nx, (1, 0, 0))]
    counts = (nx, ny, nz)
    for fname, ax, fix, nrm in faces:
        a1, a2 = [d for d in range(3) if d != ax]
        for i in range(counts[a1]):
            for j in range(counts[a2]):
                def idx(di, dj):
                    ijk = [0, 0, 0]
                    ijk[ax] = fix
                    ijk[a1] = i + di
                    ijk[a2] = j + dj
                    return P(*ijk)
                p00, p10, p01, p11 = idx(0, 0), idx(1, 0), idx(0, 1), idx(1, 1)
                V = pool.xyz      # coordinates so far (a list: no copy per cell)
                if (fname, i, j) in split4:
                    cen = 0.25 * (V[p00] + V[p10] + V[p01] + V[p11])
                    pc = pool.get(("C", fname, i, j), cen)
                    quad = [(p00, p10), (p10, p11), (p11, p01), (p01, p00)]
                    cand = [(pc, u, v) for u, v in quad]
                else:
                    cand = [(p00, p10, p11), (p00, p11, p01)]
                V = pool.xyz
                for t in cand:
                    tris.append(_orient(V, t, np.array(nrm, float)))
                    face_of.append(fname)
    V = pool.array()
    T = np.array(tris, dtype=np.int32)
    face_of = np.array(face_of)
    src = np.nonzero(face_of == "x0")[0].astype(np.int32)
    snk = np.nonzero(face_of == "x1")[0].astype(np.int32)
    return Structure(name, V, T, [(src, snk)],
                     dict(nx=nx, ny=ny, nz=nz, face_of=face_of))


def config1_bar():
    """Straight copper bar of length 1 mm along x and cross-section
    20 um (y) x 10 um (z): 82 x 4 x 2 cells, 2,000 right triangles,
    1,002 vertices; source end face at x = 0, sink at x = 1 mm."""
    s = box_bar(np.linspace(0.0, 1e-3, 83), np.linspace(-10e-6, 10e-6, 5),
                np.linspace(-5e-6, 5e-6, 3), name="config1_bar")
    s.params.update(length=1e-3, width=20e-6, thick=10e-6)
    return s


def paper_bar_e1():
    """The Section V-A interconnect, 5 um x 7.5 um x 200 um, as a closed mesh
    of 428 triangles with 8-triangle end faces (the counts the paper states).
    25 axial cells x 8 perimeter cells give 400 lateral triangles; six top
    cells carry a centre vertex (4 triangles each) to reach 428."""
    split = [("z1", i, j) for i in range(3) for j in range(2)]
    s = box_bar(np.linspace(0.0, 200e-6, 26), np.linspace(0.0, 5e-6, 3),
                np.linspace(0.0, 7.5e-6, 3), split4=split, name="paper_bar_e1")
    s.params.update(length=200e-6, width=5e-6, thick=7.5e-6)
    return s


def prism():
    """The triangular-prism interconnect of Fig. 1: 8 triangles, 12 edges,
    6 vertices (two triangular ends and three rectangular sides)."""
    L = 10e-6
    base = np.array([[0.0, 0.0], [2e-6, 0.0], [1e-6, 1.5e-6]])
    V = np.array([[0.0, y, z] for y, z in base] + [[L, y, z] for y, z in base])
    cen = V.mean(axis=0)
    raw = [(0, 1, 2), (3, 4, 5)]
    for k in range(3):
        a, b = k, (k + 1) % 3
        raw += [(a, b, b + 3), (a, b + 3, a + 3)]
    tris = []
    for t in raw:
        c = V[list(t)].mean(axis=0)
        out = c - cen
        if t == (0, 1, 2):
            out = np.array([-1.0, 0, 0])
        elif t == (3, 4, 5):
            out = np.array([1.0, 0, 0])
        else:
            out[0] = 0.0
        tris.append(_orient(V, t, out))
    T = np.array(tris, dtype=np.int32)
    return Structure("prism", V, T, [(np.array([0], np.int32), np.array([1], np.int32))])


def _arc_uniform_parabola(S, H, nseg):
    """x positions giving equal arc-length steps along z = 4H(x/S)(1-x/S)."""
    xf = np.linspace(0.0, S, 20001)
    dz = 4.0 * H / S * (1.0 - 2.0 * xf / S)
    ds = np.sqrt(1.0 + dz * dz)
    s = np.concatenate([[0.0], np.cumsum(0.5 * (ds[1:] + ds[:-1]) * np.diff(xf))])
    return np.interp(np.linspace(0.0, s[-1], nseg + 1), s, xf)


def bond_wires(nwire=8, pitch=100e-6, span=2e-3, height=300e-6, radius=12.5e-6,
               nfacet=12, nseg=207, name="bond_wires"):
    """Parallel parabolic-arch bond wires along x at y = k * pitch.

    The centreline is z = 4 H (x/S)(1 - x/S).  Each wire is a regular
    ``nfacet``-gon tube (circumradius ``radius``) of ``nseg`` arc-length-uniform
    segments, closed by fanned end caps.  Port k: source = start cap of wire k,
    sink = end cap of wire k."""
    verts, tris, ports = [], [], []
    nv = 0
    xk = _arc_uniform_parabola(span, height, nseg)
    th = 2.0 * np.pi * np.arange(nfacet) / nfacet
    yhat = np.array([0.0, 1.0, 0.0])
    for w in range(nwire):
        y0 = w * pitch
        zc = 4.0 * height * (xk / span) * (1.0 - xk / span)
        dz = 4.0 * height / span * (1.0 - 2.0 * xk / span)
        C = np.stack([xk, np.full_like(xk, y0), zc], axis=1)
        Tg = np.stack([np.ones_like(xk), np.zeros_like(xk), dz], axis=1)
        Tg /= np.linalg.norm(Tg, axis=1)[:, None]
        Nh = np.cross(yhat[None, :], Tg)
        ring = (C[:, None, :] + radius * (np.cos(th)[None, :, None] * Nh[:, None, :]
                                          + np.sin(th)[None, :, None] * yhat[None, None, :]))
        nr = nseg + 1
        V = np.concatenate([ring.reshape(-1, 3), C[[0]], C[[-1]]], axis=0)
        c0, c1 = nr * nfacet, nr * nfacet + 1

        def vid(k, j):
            return k * nfacet + (j % nfacet)
        wt = []
        for k in range(nseg):
            mid = 0.5 * (C[k] + C[k + 1])
            for j in range(nfacet):
                a, b, c, d = vid(k, j), vid(k, j + 1), vid(k + 1, j + 1), vid(k + 1, j)
                for t in ((a, b, c), (a, c, d)):
                    cen = V[list(t)].mean(axis=0)
                    wt.append(_orient(V, t, cen - mid))
        src, snk = [], []
        for j in range(nfacet):
            src.append(len(wt))
            wt.append(_orient(V, (c0, vid(0, j), vid(0, j + 1)), -Tg[0]))
        for j in range(nfacet):
            snk.append(len(wt))
            wt.append(_orient(V, (c1, vid(nseg, j), vid(nseg, j + 1)), Tg[-1]))
        base = len(tris)
        tris.extend([(a + nv, b + nv, c + nv) for a, b, c in wt])
        verts.append(V)
        nv += V.shape[0]
        ports.append((np.array(src, np.int32) + base, np.array(snk, np.int32) + base))
    return Structure(name, np.concatenate(verts, axis=0),
                     np.array(tris, dtype=np.int32), ports,
                     dict(nwire=nwire, pitch=pitch, span=span, height=height,
                          radius=radius, nfacet=nfacet, nseg=nseg))


def config2_wires():
    """8 parabolic-arch wires, 25 um diameter (12 facets), span 2 mm, arch
    height 300 um, pitch 100 um: 39,936 triangles, 8 ports."""
    return bond_wires(name="config2_wires")


# ---------------------------------------------------------------------------
# Manhattan meander traces
# ---------------------------------------------------------------------------

def _section(nw, nt, width, thick):
    """Perimeter points (u, v) of a width x thick rectangle with nw cells along
    the width and nt along the thickness, counter-clockwise in (u, v)."""
    us = np.linspace(-width / 2, width / 2, nw + 1)
    vs = np.linspace(-thick / 2, thick / 2, nt + 1)
    pts = [(u, vs[0]) for u in us[:-1]]
    pts += [(us[-1], v) for v in vs[:-1]]
    pts += [(u, vs[-1]) for u in us[::-1][:-1]]
    pts += [(us[0], v) for v in vs[::-1][:-1]]
    return np.array(pts), us, vs


def _trace_mesh(path, width, thick, nw, nt, step):
    """Tube of rectangular section along a planar Manhattan polyline ``path``
    (k x 2 points in the z = 0 plane), mitred at the corners, with structured
    end caps.  Returns (V, T, src_tris, snk_tris)."""
    per, us, vs = _section(nw, nt, width, thick)
    m = per.shape[0]
    path = np.asarray(path, dtype=np.float64)
    d = np.diff(path, axis=0)
    L = np.linalg.norm(d, axis=1)
    D = d / L[:, None]
    Nl = np.stack([-D[:, 1], D[:, 0]], axis=1)          # left normal of each segment
    # stations: (centre point, in-plane offset direction for u)
    rings = []
    for s in range(len(L)):
        if s == 0:
            rings.append(path[0][None, :] + per[:, :1] * Nl[0][None, :])
        nstep = max(1, int(round(L[s] / step)))
        for k in range(1, nstep):
            c = path[s] + D[s] * (L[s] * k / nstep)
            rings.append(c[None, :] + per[:, :1] * Nl[s][None, :])
        c = path[s + 1]
        if s + 1 < len(L):
            # mitre: offset u maps to c + u * (n_s + n_{s+1}) (90-degree turn)
            rings.append(c[None, :] + per[:, :1] * (Nl[s] + Nl[s + 1])[None, :])
        else:
            rings.append(c[None, :] + per[:, :1] * Nl[s][None, :])
    R = np.stack(rings, axis=0)                          # (nr, m, 2)
    nr = R.shape[0]
    V = np.concatenate([R, np.broadcast_to(per[None, :, 1:], (nr, m, 1))], axis=2).reshape(-1, 3)
    tris = []

    def vid(k, j):
        return k * m + (j % m)
    for k in range(nr - 1):
        ck = R[k].mean(axis=0)
        ck1 = R[k + 1].mean(axis=0)
        axis3 = np.array([ck1[0] - ck[0], ck1[1] - ck[1], 0.0])
        mid3 = np.array([(ck[0] + ck1[0]) / 2, (ck[1] + ck1[1]) / 2, 0.0])
        for j in range(m):
            a, b, c, dd = vid(k, j), vid(k, j + 1), vid(k + 1, j + 1), vid(k + 1, j)
            for t in ((a, b, c), (a, c, dd)):
                cen = V[list(t)].mean(axis=0)
                out = cen - mid3
                out = out - axis3 * np.dot(out, axis3) / np.dot(axis3, axis3)
                tris.append(_orient(V, t, out))
    # end caps: structured nw x nt grid in (u, v); perimeter nodes reuse ring vertices
    Vl = [V]
    nv = V.shape[0]
    caps = []
    for end, (k, nrm2) in enumerate(((0, -D[0]), (nr - 1, D[-1]))):
        nl = Nl[0] if end == 0 else Nl[-1]
        ctr = path[0] if end == 0 else path[-1]
        key = {}
        for j, (u, v) in enumerate(per):
            key[(round(u * 1e12), round(v * 1e12))] = vid(k, j)
        extra = []
        grid = np.empty((nw + 1, nt + 1), dtype=np.int64)
        for i, u in enumerate(us):
            for jj, v in enumerate(vs):
                kk = (round(u * 1e12), round(v * 1e12))
                if kk in key:
                    grid[i, jj] = key[kk]
                else:
                    grid[i, jj] = nv + len(extra)
                    extra.append([ctr[0] + u * nl[0], ctr[1] + u * nl[1], v])
        Vl.append(np.array(extra).reshape(-1, 3))
        nv += len(extra)
        Vc = np.concatenate(Vl, axis=0)
        out = np.array([nrm2[0], nrm2[1], 0.0])
        start = len(tris)
        for i in range(nw):
            for jj in range(nt):
                p00, p10, p01, p11 = grid[i, jj], grid[i + 1, jj], grid[i, jj + 1], grid[i + 1, jj + 1]
                for t in ((p00, p10, p11), (p00, p11, p01)):
                    tris.append(_orient(Vc, t, out))
        caps.append(np.arange(start, len(tris), dtype=np.int32))
    V = np.concatenate(Vl, axis=0)
    return V, np.array(tris, dtype=np.int32), caps[0], caps[1]


def _meander_path(rng, x0, x1, ylo, yhi, turns, length):
    """Manhattan path from (x0, y) to the right, jogging between y levels
    inside [ylo, yhi]; ``turns`` corners in total."""
    njog = turns // 2
    ys = [ylo, yhi]
    ymid = 0.5 * (ylo + yhi)
    jog = yhi - ylo
    xrun = min(x1 - x0, max(length - njog * jog - (turns % 2) * 0.5 * jog, 0.2 * (x1 - x0)))
    cuts = np.sort(rng.uniform(0.1, 0.9, size=njog)) if njog else np.array([])
    xs = x0 + xrun * cuts
    cur = 0
    pts = [(x0, ys[cur])]
    for xc in xs:
        pts.append((xc, ys[cur]))
        cur ^= 1
        pts.append((xc, ys[cur]))
    xe = x0 + xrun
    pts.append((xe, ys[cur]))
    if turns % 2:
        pts.append((xe, ymid if cur == 0 else ymid))
    # drop zero-length segments
    out = [pts[0]]
    for p in pts[1:]:
        if abs(p[0] - out[-1][0]) + abs(p[1] - out[-1][1]) > 1e-12:
            out.append(p)
    return np.array(out)


def traces(ntrace=32, seed=0, area=5e-3, width=20e-6, thick=15e-6, nw=4, nt=3,
           step=None, target_tris=200_000, len_range=(2e-3, 6e-3), name="traces"):
    """``ntrace`` Manhattan meander traces, one per lane of width area/ntrace,
    width x thickness section meshed with nw x nt cells, seeded turn count in
    3..8 and seeded length in ``len_range`` (capped by what fits the lane).
    The axial step is chosen so the total triangle count is near
    ``target_tris``.  Port k: source = start cap, sink = end cap of trace k."""
    lane = area / ntrace
    plans = []
    for k in range(ntrace):
        rng = np.random.default_rng(k + 100 * seed)
        turns = int(rng.integers(3, 9))
        length = float(rng.uniform(*len_range))
        ylo = k * lane + 0.5 * width + 0.15 * lane
        yhi = (k + 1) * lane - 0.5 * width - 0.15 * lane
        plans.append(_meander_path(rng, 0.0, area, ylo, yhi, turns, length))
    total = sum(np.abs(np.diff(p, axis=0)).sum() for p in plans)
    m = 2 * (nw + nt)
    if step is None:
        step = max(total * 2 * m / max(target_tris - ntrace * 4 * nw * nt, 1), width / nw)
    Vs, Ts, ports = [], [], []
    nv = nt_ = 0
    for p in plans:
        V, T, s, e = _trace_mesh(p, width, thick, nw, nt, step)
        Vs.append(V)
        Ts.append(T + nv)
        ports.append((s + nt_, e + nt_))
        nv += V.shape[0]
        nt_ += T.shape[0]
    return Structure(name, np.concatenate(Vs), np.concatenate(Ts).astype(np.int32), ports,
                     dict(ntrace=ntrace, seed=seed, step=step, width=width, thick=thick))


def config3_traces(seed=0):
    """32 meander traces on a 5 x 5 mm area, ~200k triangles, 32 ports."""
    return traces(seed=seed, name="config3_traces")


def _zipper(inner, outer, ci, co):
    """Triangles between two closed vertex rings around a common centre, each
    listed counter-clockwise by angle (``ci``/``co``: their angles, increasing
    from the same start); both rings are star-shaped about the centre, so
    advancing along whichever ring has the next smaller angle never folds."""
    ni, no = len(inner), len(outer)
    ai = np.concatenate([ci, ci[:1] + 2 * np.pi])
    ao = np.concatenate([co, co[:1] + 2 * np.pi])
    tris = []
    i = j = 0
    while i < ni or j < no:
        if j < no and (i >= ni or ao[j + 1] <= ai[i + 1]):
            tris.append((inner[i % ni], outer[j % no], outer[(j + 1) % no]))
            j += 1
        else:
            tris.append((inner[i % ni], outer[j % no], inner[(i + 1) % ni]))
            i += 1
    return tris


def pdn(nx=350, ny=350, cell=10e-3 / 350, thick=35e-6, gap=200e-6, vias=(), block=6, radius=50e-6,
        nfacet=12, ports=(), patch=4, name="pdn"):
    """Two parallel copper planes joined by cylindrical vias, as one closed
    surface (genus = number of vias - 1).

    The planes span [0, nx cell] x [0, ny cell]; the lower one z in [0, thick],
    the upper one z in [thick + gap, 2 thick + gap].  Their large faces are
    lattices of cell x cell squares cut into two triangles.  A via joins the
    lower plane's top face to the upper plane's bottom face: it occupies a
    ``block`` x ``block`` cell block with lower corner ``vias[k]`` = (i, j),
    whose interior lattice points are replaced by an ``nfacet``-gon hole of
    the given radius at the block centre (the ring between the block's
    boundary points and the hole is triangulated by angle), and its barrel is
    an ``nfacet``-gon prism in about cell-high rings.  The side faces carry the
    lattice spacing along the edges and about cell-high layers across.
    Port k (``ports[k]`` = (i, j)): source = the ``patch`` x ``patch`` cells
    at (i, j) of the upper plane's top face, sink = the same cells of the
    lower plane's bottom face."""
    nzl = max(1, int(round(thick / cell)))
    nzb = max(1, int(round(gap / cell)))
    zlev = [[p * (thick + gap) + thick * k / nzl for k in range(nzl + 1)] for p in range(2)]
    xs = np.arange(nx + 1) * cell
    ys = np.arange(ny + 1) * cell
    inblock = np.zeros((nx, ny), dtype=bool)      # cells replaced by a via ring
    hidden = np.zeros((nx + 1, ny + 1), dtype=bool)
    for (bi, bj) in vias:
        assert 0 < bi and bi + block < nx and 0 < bj and bj + block < ny, "via block off the plane"
        assert not inblock[bi:bi + block, bj:bj + block].any(), "overlapping via blocks"
        inblock[bi:bi + block, bj:bj + block] = True
        hidden[bi + 1:bi + block, bj + 1:bj + block] = True
    V = []
    nv = 0

    def add(pts):
        nonlocal nv
        pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
        V.append(pts)
        ids = np.arange(nv, nv + pts.shape[0])
        nv += pts.shape[0]
        return ids

    X, Y = np.meshgrid(xs, ys, indexing="ij")
    # big-face lattices: face (p, top) for plane p, top = 0 lower face, 1 upper
    face = {}
    for p in range(2):
        for top in range(2):
            z = zlev[p][nzl if top else 0]
            holes = (p == 0 and top == 1) or (p == 1 and top == 0)
            ids = -np.ones((nx + 1, ny + 1), dtype=np.int64)
            keep = ~hidden if holes else np.ones_like(hidden)
            ids[keep] = add(np.stack([X[keep], Y[keep], np.full(int(keep.sum()), z)], axis=1))
            face[(p, top)] = ids
    # intermediate z levels of the side faces: perimeter points only
    per = [(i, 0) for i in range(nx)] + [(nx, j) for j in range(ny)] + \
          [(i, ny) for i in range(nx, 0, -1)] + [(0, j) for j in range(ny, 0, -1)]
    side = {}
    for p in range(2):
        for k in range(nzl + 1):
            if k == 0:
                side[(p, k)] = np.array([face[(p, 0)][i, j] for i, j in per])
            elif k == nzl:
                side[(p, k)] = np.array([face[(p, 1)][i, j] for i, j in per])
            else:
                side[(p, k)] = add([(xs[i], ys[j], zlev[p][k]) for i, j in per])
    tris, tag = [], []
    Vall = lambda: np.concatenate(V)   # noqa: E731
    # large faces
    for (p, top), ids in face.items():
        holes = (p == 0 and top == 1) or (p == 1 and top == 0)
        ii, jj = np.nonzero(~inblock) if holes else np.nonzero(np.ones((nx, ny), bool))
        a, b, c, d = ids[ii, jj], ids[ii + 1, jj], ids[ii + 1, jj + 1], ids[ii, jj + 1]
        if top:   # outward +z: counter-clockwise seen from above
            t1, t2 = np.stack([a, b, c], 1), np.stack([a, c, d], 1)
        else:
            t1, t2 = np.stack([a, c, b], 1), np.stack([a, d, c], 1)
        tt = np.empty((2 * len(ii), 3), dtype=np.int64)
        tt[0::2], tt[1::2] = t1, t2
        tris.append(tt)
        tg = np.empty((2 * len(ii), 3), dtype=np.int64)
        tg[:, 0], tg[:, 1], tg[:, 2] = (p * 2 + top), np.repeat(ii, 2), np.repeat(jj, 2)
        tag.append(tg)
    # side faces
    npr = len(per)
    for p in range(2):
        for k in range(nzl):
            lo, hi = side[(p, k)], side[(p, k + 1)]
            q = np.arange(npr)
            a, b, c, d = lo[q], lo[(q + 1) % npr], hi[(q + 1) % npr], hi[q]
            # the perimeter runs counter-clockwise seen from above, so
            # (a, b, c) winds outward
            tt = np.empty((2 * npr, 3), dtype=np.int64)
            tt[0::2], tt[1::2] = np.stack([a, b, c], 1), np.stack([a, c, d], 1)
            tris.append(tt)
            tag.append(np.full((2 * npr, 3), -1, dtype=np.int64))
    # via rings and barrels
    ang = 2 * np.pi * (np.arange(nfacet) + 0.5) / nfacet
    extra = []
    for (bi, bj) in vias:
        cx, cy = (bi + block / 2) * cell, (bj + block / 2) * cell
        bnd = [(bi + s, bj) for s in range(block)] + [(bi + block, bj + s) for s in range(block)] + \
              [(bi + block - s, bj + block) for s in range(block)] + [(bi, bj + block - s) for s in range(block)]
        bang = np.array([np.arctan2(ys[j] - cy, xs[i] - cx) for i, j in bnd])
        # start both rings at the smallest angle of the boundary (a corner)
        r0 = int(np.argmin(np.mod(bang, 2 * np.pi)))
        bnd = bnd[r0:] + bnd[:r0]
        bang = np.mod(np.concatenate([bang[r0:], bang[:r0]]) - 0.0, 2 * np.pi)
        start = bang[0]
        bang = np.mod(bang - start, 2 * np.pi)
        hang = np.mod(ang - start, 2 * np.pi)
        hord = np.argsort(hang)
        rings = []
        for s in range(nzb + 1):
            z = thick + gap * s / nzb
            rings.append(add(np.stack([cx + radius * np.cos(ang), cy + radius * np.sin(ang),
                                       np.full(nfacet, z)], axis=1)))
        for s, (p, top, outz) in ((0, (0, 1, 1.0)), (nzb, (1, 0, -1.0))):
            ids = face[(p, top)]
            outer = [ids[i, j] for i, j in bnd]
            inner = [rings[s][h] for h in hord]
            VV = Vall()
            for t in _zipper(inner, outer, hang[hord], bang):
                extra.append(_orient(VV, t, np.array([0.0, 0.0, outz])))
        VV = Vall()
        for s in range(nzb):
            for h in range(nfacet):
                h1 = (h + 1) % nfacet
                a, b, c, d = rings[s][h], rings[s][h1], rings[s + 1][h1], rings[s + 1][h]
                mid = 0.25 * (VV[a] + VV[b] + VV[c] + VV[d])
                out = np.array([mid[0] - cx, mid[1] - cy, 0.0])
                extra.append(_orient(VV, (a, b, c), out))
                extra.append(_orient(VV, (a, c, d), out))
    T = np.concatenate(tris + ([np.array(extra, dtype=np.int64)] if extra else []), axis=0).astype(np.int32)
    tags = np.concatenate(tag + ([np.full((len(extra), 3), -1, dtype=np.int64)] if extra else []), axis=0)
    Vc = Vall()
    plist = []
    for (pi, pj) in ports:
        sel = lambda f: np.nonzero((tags[:, 0] == f) & (tags[:, 1] >= pi) & (tags[:, 1] < pi + patch) &  # noqa: E731
                                   (tags[:, 2] >= pj) & (tags[:, 2] < pj + patch))[0].astype(np.int32)
        plist.append((sel(3), sel(0)))   # source: upper plane's top face; sink: lower plane's bottom face
    return Structure(name, Vc, T, plist, dict(nx=nx, ny=ny, cell=cell, thick=thick, gap=gap, vias=list(vias),
                                              block=block, radius=radius, nfacet=nfacet, patch=patch))


def _via_sites(rng, nx, ny, block, nvia, min_gap_cells, margin):
    """Rejection-sampled lower corners of nvia via blocks, block centres at
    least min_gap_cells apart and ``margin`` cells from the plane edge."""
    out = []
    tries = 0
    while len(out) < nvia:
        tries += 1
        assert tries < 100000, "cannot place the vias"
        i = int(rng.integers(margin, nx - margin - block))
        j = int(rng.integers(margin, ny - margin - block))
        if all((i - a) ** 2 + (j - b) ** 2 >= min_gap_cells ** 2 for a, b in out):
            out.append((i, j))
    return out


def config4_pdn(seed=0, nx=350, nvia=100, nport=16):
    """Two 10 x 10 mm planes, 35 um thick, 0.2 mm apart, joined by ``nvia``
    vias of 100 um diameter (12 facets) at seeded positions at least 300 um
    apart on the ~28.6 um lattice; ``nport`` ports as a square array of
    ~114 um patches, source on the top face, sink directly below on the
    bottom face.  ~1 M triangles at the default size."""
    cell = 10e-3 / 350
    rng = np.random.default_rng(1000 + seed)
    block = 6
    vias = _via_sites(rng, nx, nx, block, nvia, int(np.ceil(300e-6 / cell)), 2)
    k = int(round(np.sqrt(nport)))
    assert k * k == nport
    step = nx // (k + 1)
    ports = [(step * (a + 1) - 2, step * (b + 1) - 2) for a in range(k) for b in range(k)]
    return pdn(nx=nx, ny=nx, cell=cell, vias=vias, block=block, ports=ports, name="config4_pdn")
