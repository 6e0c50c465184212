"""RWG basis functions (Rao-Wilton-Glisson) on a triangle mesh.

The paper discretises the surface current with RWG functions and tests them
by Galerkin's method (Sec. II, the paragraph before eq. 9).  One unknown per
interior edge.  Conventions fixed here (the paper is silent on them):

* unknowns are the interior edges sorted lexicographically by
  (min vertex id, max vertex id);
* T+ is the triangle that traverses the edge from the smaller to the larger
  vertex id in its own counter-clockwise order, T- the other one;
* on T+:  f(r) = +(l / 2A+) (r - v+),  div f = +l / A+;
  on T-:  f(r) = -(l / 2A-) (r - v-),  div f = -l / A-;
  where v+- is the vertex of T+- opposite the edge and l the edge length.
  The normal component of f across the edge is 1 (flux continuity).
"""

import numpy as np


class MeshError(ValueError):
    pass


def triangle_geometry(xyz, tri):
    """Centroids (v0+v1+v2)/3, areas, unit normals (right-hand rule)."""
    v0, v1, v2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    cen = (v0 + v1 + v2) / 3.0
    nrm = np.cross(v1 - v0, v2 - v0)
    twice_area = np.linalg.norm(nrm, axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        unit = nrm / twice_area[:, None]
    return cen, 0.5 * twice_area, unit


def max_edge_length(xyz, tri):
    v = xyz[tri]
    e = np.concatenate([v[:, 1] - v[:, 0], v[:, 2] - v[:, 1], v[:, 0] - v[:, 2]])
    return float(np.sqrt((e[:, 0] * e[:, 0] + e[:, 1] * e[:, 1]) + e[:, 2] * e[:, 2]).max())


def build_rwg(xyz, tri, allow_open=False):
    """Return a dict describing the RWG functions of the mesh.

    Raises MeshError for out-of-range indices, degenerate triangles, edges with
    more than two triangles, inconsistent orientation, or (unless
    ``allow_open``) boundary edges.
    """
    xyz = np.asarray(xyz, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    if tri.ndim != 2 or tri.shape[1] != 3 or xyz.ndim != 2 or xyz.shape[1] != 3:
        raise MeshError("bad array shapes")
    if tri.min() < 0 or tri.max() >= len(xyz):
        raise MeshError("triangle vertex index out of range")
    _, area, _ = triangle_geometry(xyz, tri)
    h = max_edge_length(xyz, tri)
    if np.any(area <= 1e-12 * h * h):
        raise MeshError("degenerate triangle")
    if np.any(tri[:, 0] == tri[:, 1]) or np.any(tri[:, 1] == tri[:, 2]) or np.any(tri[:, 0] == tri[:, 2]):
        raise MeshError("degenerate triangle")

    edges = {}
    for t in range(len(tri)):
        for e in range(3):
            a, b = int(tri[t, e]), int(tri[t, (e + 1) % 3])
            key = (a, b) if a < b else (b, a)
            edges.setdefault(key, []).append((t, a < b))
    keys = sorted(edges)
    ev, tp, tm = [], [], []
    for key in keys:
        inc = edges[key]
        if len(inc) > 2:
            raise MeshError("non-manifold edge %s" % (key,))
        if len(inc) == 1:
            if not allow_open:
                raise MeshError("open boundary edge %s" % (key,))
            continue
        (t1, fwd1), (t2, fwd2) = inc
        if fwd1 == fwd2:
            raise MeshError("inconsistent orientation at edge %s" % (key,))
        plus, minus = (t1, t2) if fwd1 else (t2, t1)
        ev.append(key)
        tp.append(plus)
        tm.append(minus)
    ev = np.array(ev, dtype=np.int64).reshape(-1, 2)
    tp = np.array(tp, dtype=np.int64)
    tm = np.array(tm, dtype=np.int64)

    def free_vertex(t):
        tv = tri[t]
        m = (tv != ev[:, :1]) & (tv != ev[:, 1:2])
        return tv[np.arange(len(t)), np.argmax(m, axis=1)]

    vp, vm = free_vertex(tp), free_vertex(tm)
    d = xyz[ev[:, 1]] - xyz[ev[:, 0]]
    length = np.sqrt((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
    return dict(edges=ev, tplus=tp, tminus=tm, vplus=vp, vminus=vm, length=length,
                N=len(ev), xyz=xyz, tri=tri)


def edge_midpoints(rwg):
    xyz, ev = rwg["xyz"], rwg["edges"]
    return 0.5 * (xyz[ev[:, 0]] + xyz[ev[:, 1]])


def rwg_value(rwg, n, side, r):
    """f_n(r) for points r (K, 3) on triangle T+ (side=+1) or T- (side=-1)."""
    xyz, tri = rwg["xyz"], rwg["tri"]
    t = rwg["tplus"][n] if side > 0 else rwg["tminus"][n]
    v = xyz[rwg["vplus"][n] if side > 0 else rwg["vminus"][n]]
    _, area, _ = triangle_geometry(xyz, tri[t:t + 1])
    return side * rwg["length"][n] / (2.0 * area[0]) * (np.asarray(r) - v)
