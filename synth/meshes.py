"""Closed triangulated surfaces used as synthetic workloads.

Every mesh is returned as ``(verts, tris)``: ``verts`` float64 (n_v, 3),
``tris`` int32 (n_t, 3), counter-clockwise seen from outside (so the winding
normal points out of the enclosed volume, the orientation the boundary
formulation assumes for its outward normal).  All generators are
deterministic; none of them draws random numbers.
"""
import numpy as np

_PHI = (1.0 + 5.0 ** 0.5) / 2.0


def _orient_outward(verts, tris, centre=(0.0, 0.0, 0.0)):
    """Flip triangles whose winding normal points towards ``centre``.

    Valid for surfaces that are star-shaped about ``centre`` (all generators
    here produce convex surfaces)."""
    v = verts[tris]
    n = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    c = v.mean(axis=1) - np.asarray(centre)
    flip = (n * c).sum(axis=1) < 0
    out = tris.copy()
    out[flip, 1], out[flip, 2] = tris[flip, 2], tris[flip, 1]
    return out


def _base_icosahedron():
    v = np.array([(-1, _PHI, 0), (1, _PHI, 0), (-1, -_PHI, 0), (1, -_PHI, 0),
                  (0, -1, _PHI), (0, 1, _PHI), (0, -1, -_PHI), (0, 1, -_PHI),
                  (_PHI, 0, -1), (_PHI, 0, 1), (-_PHI, 0, -1), (-_PHI, 0, 1)],
                 dtype=np.float64)
    f = np.array([(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
                  (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
                  (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
                  (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)],
                 dtype=np.int32)
    return v, _orient_outward(v, f)


def icosphere(m, radius=1.0):
    """Geodesic sphere: each icosahedron face split into m*m triangles, points
    projected radially onto the sphere.  20*m*m triangles, 10*m*m+2 vertices.
    Shared edge points are computed from the lower-numbered corner so the two
    faces that own an edge produce bit-identical vertices."""
    m = int(m)
    if m < 1:
        raise ValueError("frequency must be >= 1")
    base_v, base_f = _base_icosahedron()
    index = {}
    pts = []

    def vid(key, xyz):
        i = index.get(key)
        if i is None:
            i = len(pts)
            index[key] = i
            pts.append(xyz)
        return i

    def point(face, i, j):
        a, b, c = (int(t) for t in base_f[face])
        # barycentric weights (m-i-j, i, j)/m on corners (a, b, c)
        wa, wb, wc = m - i - j, i, j
        nz = [(w, corner) for w, corner in ((wa, a), (wb, b), (wc, c)) if w > 0]
        if len(nz) == 1:
            corner = nz[0][1]
            return vid(("v", corner), base_v[corner])
        if len(nz) == 2:
            (w0, p0), (w1, p1) = nz
            lo, hi = (p0, p1) if p0 < p1 else (p1, p0)
            t = w1 if hi == p1 else w0          # weight of the higher corner
            xyz = base_v[lo] + (t / m) * (base_v[hi] - base_v[lo])
            return vid(("e", lo, hi, t), xyz)
        xyz = (wa * base_v[a] + wb * base_v[b] + wc * base_v[c]) / m
        return vid(("f", face, i, j), xyz)

    tris = []
    for f in range(20):
        grid = {}
        for i in range(m + 1):
            for j in range(m + 1 - i):
                grid[i, j] = point(f, i, j)
        for i in range(m):
            for j in range(m - i):
                tris.append((grid[i, j], grid[i + 1, j], grid[i, j + 1]))
                if i + j + 1 < m:
                    tris.append((grid[i + 1, j], grid[i + 1, j + 1], grid[i, j + 1]))
    v = np.array(pts, dtype=np.float64)
    v *= radius / np.linalg.norm(v, axis=1, keepdims=True)
    t = np.array(tris, dtype=np.int32)
    return v, _orient_outward(v, t)


def ellipsoid(m, semi_axes):
    """Icosphere of frequency m mapped onto an ellipsoid with the given
    semi-axes (x, y, z)."""
    v, t = icosphere(m, 1.0)
    return v * np.asarray(semi_axes, dtype=np.float64)[None, :], t


def rounded_box(dims, rho, spacing):
    """Sphere-swept box with outer dimensions ``dims`` and edge/corner
    rounding radius ``rho``, meshed from a lattice of the given spacing.

    The outer box surface is covered by a structured lattice (each face split
    into quads, each quad into two triangles); every lattice point q is then
    moved to c + rho*(q - c)/|q - c| with c the closest point of the inner box
    (the outer box shrunk by rho).  rho = 0 gives the sharp box."""
    dims = np.asarray(dims, dtype=np.float64)
    n = np.maximum(1, np.rint(dims / spacing).astype(int))
    half = dims / 2.0
    index = {}
    pts = []

    def vid(ijk):
        i = index.get(ijk)
        if i is None:
            i = len(pts)
            index[ijk] = i
            pts.append(ijk)
        return i

    tris = []
    for axis in range(3):
        a1, a2 = [a for a in range(3) if a != axis]
        for side in (0, n[axis]):
            for u in range(n[a1]):
                for w in range(n[a2]):
                    quad = []
                    for du, dw in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        ijk = [0, 0, 0]
                        ijk[axis] = side
                        ijk[a1] = u + du
                        ijk[a2] = w + dw
                        quad.append(vid(tuple(ijk)))
                    # alternate the diagonal to avoid a directional bias
                    if (u + w) % 2 == 0:
                        tris.append((quad[0], quad[1], quad[2]))
                        tris.append((quad[0], quad[2], quad[3]))
                    else:
                        tris.append((quad[0], quad[1], quad[3]))
                        tris.append((quad[1], quad[2], quad[3]))
    ijk = np.array(pts, dtype=np.float64)
    q = -half + ijk * (dims / n)
    if rho > 0:
        inner = half - rho
        c = np.clip(q, -inner, inner)
        d = q - c
        q = c + rho * d / np.linalg.norm(d, axis=1, keepdims=True)
    t = np.array(tris, dtype=np.int32)
    return q, _orient_outward(q, t)


def tetrahedron(scale=0.1):
    v = scale * np.array([(1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)], dtype=np.float64)
    t = np.array([(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)], dtype=np.int32)
    return v, _orient_outward(v, t)


def octahedron(scale=0.1):
    v = scale * np.array([(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)],
                         dtype=np.float64)
    t = np.array([(0, 2, 4), (2, 1, 4), (1, 3, 4), (3, 0, 4),
                  (2, 0, 5), (1, 2, 5), (3, 1, 5), (0, 3, 5)], dtype=np.int32)
    return v, _orient_outward(v, t)


def icosahedron(scale=0.1):
    v, t = _base_icosahedron()
    return v * scale / np.linalg.norm(v[0]), t


def flat_plate(size, n):
    """Open square plate in the z = 0 plane (n x n quads); used only for
    pair-level checks on coplanar triangles, never as a closed workload."""
    x = np.linspace(-size / 2, size / 2, n + 1)
    X, Y = np.meshgrid(x, x, indexing="ij")
    v = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    t = []
    for i in range(n):
        for j in range(n):
            a, b, c, d = i * (n + 1) + j, (i + 1) * (n + 1) + j, (i + 1) * (n + 1) + j + 1, i * (n + 1) + j + 1
            t.append((a, b, c))
            t.append((a, c, d))
    return v, np.array(t, dtype=np.int32)


def scene(*parts):
    """Several closed surfaces in one mesh: parts are (verts, tris, offset)
    with offset a translation (3,); vertex indices are renumbered."""
    vs, ts, base = [], [], 0
    for v, t, off in parts:
        vs.append(np.asarray(v, np.float64) + np.asarray(off, np.float64))
        ts.append(np.asarray(t, np.int32) + base)
        base += len(v)
    return np.concatenate(vs), np.concatenate(ts).astype(np.int32)


def mesh_stats(verts, tris):
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    L = np.linalg.norm(verts[e[:, 0]] - verts[e[:, 1]], axis=1)
    return {"n_tris": int(len(tris)), "n_verts": int(len(verts)), "n_edges": int(len(e)),
            "mean_edge": float(L.mean()), "min_edge": float(L.min()), "max_edge": float(L.max())}
