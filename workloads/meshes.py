"""Triangle meshes for PEC scatterers (closed spheres/ellipsoids, open plates).

Every mesh is returned as ``(xyz, tri)``: ``xyz`` float64 (nv, 3) in metres and
``tri`` int32 (nt, 3) with each triangle counter-clockwise when seen from the
outside (outward normal by the right-hand rule).
"""

import numpy as np


def _icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    return v, f


def _orient_outward(xyz, tri):
    """Flip any triangle whose right-hand normal points towards the origin
    (valid for star-shaped bodies centred at the origin)."""
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    n = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", n, (a + b + c) / 3.0) < 0
    tri = tri.copy()
    tri[flip] = tri[flip][:, [0, 2, 1]]
    return tri


def icosphere(subdiv, radius=1.0):
    """Icosahedron refined ``subdiv`` times by 4-way midpoint splitting, with
    every new vertex projected to the unit sphere after each level, then
    scaled to ``radius``.  subdiv s gives 20*4**s triangles and 30*4**s edges."""
    v, f = _icosahedron()
    verts = [tuple(p) for p in v]
    for _ in range(subdiv):
        cache = {}
        vlist = verts

        def mid(i, j):
            key = (i, j) if i < j else (j, i)
            k = cache.get(key)
            if k is None:
                p = np.array(vlist[i]) + np.array(vlist[j])
                p /= np.linalg.norm(p)
                vlist.append(tuple(p))
                k = len(vlist) - 1
                cache[key] = k
            return k

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        f = np.array(nf, dtype=np.int64)
        verts = vlist
    xyz = np.array(verts, dtype=np.float64) * radius
    tri = _orient_outward(xyz, f)
    return xyz, tri.astype(np.int32)


def geodesic_sphere(freq, radius=1.0):
    """Class-I geodesic icosahedron of frequency ``freq``: every face of the
    icosahedron is split into freq**2 triangles on a barycentric grid, and the
    grid points are projected once to the sphere.  20*freq**2 triangles."""
    v, f = _icosahedron()
    key_to_idx = {}
    pts = []

    def vid(face, i, j):
        # barycentric grid point (i, j) of face: a + (b-a) i/n + (c-a) j/n
        a, b, c = f[face]
        n = freq
        # canonical key for points shared between faces: integer barycentrics
        # over the global vertex ids.
        w = {a: n - i - j, b: i, c: j}
        key = tuple(sorted((g, wt) for g, wt in w.items() if wt > 0))
        k = key_to_idx.get(key)
        if k is None:
            p = (v[a] * (n - i - j) + v[b] * i + v[c] * j) / n
            p = p / np.linalg.norm(p)
            pts.append(p)
            k = len(pts) - 1
            key_to_idx[key] = k
        return k

    tris = []
    n = freq
    for face in range(len(f)):
        for i in range(n):
            for j in range(n - i):
                p0 = vid(face, i, j)
                p1 = vid(face, i + 1, j)
                p2 = vid(face, i, j + 1)
                tris.append([p0, p1, p2])
                if i + j < n - 1:
                    p3 = vid(face, i + 1, j + 1)
                    tris.append([p1, p3, p2])
    xyz = np.array(pts, dtype=np.float64) * radius
    tri = _orient_outward(xyz, np.array(tris, dtype=np.int64))
    return xyz, tri.astype(np.int32)


def ellipsoid_mesh(xyz_unit, tri, semi_axes):
    """Affine image of a unit-sphere mesh: (x, y, z) -> (a x, b y, c z).
    Orientation is preserved because all three factors are positive."""
    s = np.asarray(semi_axes, dtype=np.float64)
    return xyz_unit * s[None, :], tri.copy()


def flat_plate(side, n):
    """Open square plate in the z=0 plane, side ``side`` metres, centred at the
    origin, split into n x n squares of two triangles each (normal +z)."""
    g = np.linspace(-side / 2.0, side / 2.0, n + 1)
    X, Y = np.meshgrid(g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)

    def idx(i, j):
        return i * (n + 1) + j

    tris = []
    for i in range(n):
        for j in range(n):
            a, b, c, d = idx(i, j), idx(i + 1, j), idx(i + 1, j + 1), idx(i, j + 1)
            tris.append([a, b, c])
            tris.append([a, c, d])
    return xyz, np.array(tris, dtype=np.int32)
