"""Seeded mesh generators for closed star-shaped surfaces centred at the origin.

All meshes are returned as ``(xyz, tri)``: ``xyz`` is ``float64[nv, 3]`` and
``tri`` is ``int32[nt, 3]`` with 0-based vertex indices, counter-clockwise when
seen from outside (outward normal by the right-hand rule).  Every vertex is used
by at least one triangle.

Generators:
  * icosphere(level)       -- recursive 4-way split of the icosahedron,
                              nt = 20*4**level, nv = 10*4**level + 2.
  * fibonacci_sphere(n)    -- n Fibonacci-lattice points, convex hull,
                              nt = 2n - 4 (an independent, nonconforming grid).
  * random_rotation(rng)   -- rotation from a normalised Gaussian quaternion.
  * jitter_on_sphere       -- tangential Gaussian vertex noise, re-projected
                              onto the unit sphere.
  * scale_to_ellipsoid     -- linear map (x, y, z) -> (a x, b y, c z).
  * planar_square          -- structured triangulation of the unit square with
                              optional in-plane node perturbation (boundary
                              nodes move along the boundary, corners fixed).
"""
import numpy as np


def _normalise(v):
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def orient_outward(xyz, tri):
    """Flip triangles whose right-hand normal points towards the origin."""
    tri = np.array(tri, dtype=np.int32, copy=True)
    p0, p1, p2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    n = np.cross(p1 - p0, p2 - p0)
    c = (p0 + p1 + p2) / 3.0
    flip = np.einsum("ij,ij->i", n, c) < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    return tri


def icosphere(level):
    """Icosahedron refined ``level`` times by edge midpoints, on the unit sphere."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    f = [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
         [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
         [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
         [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]]
    verts = list(_normalise(v))
    faces = [tuple(x) for x in f]
    for _ in range(level):
        cache = {}
        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]
        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    xyz = np.array(verts, dtype=np.float64)
    tri = orient_outward(xyz, np.array(faces, dtype=np.int32))
    return xyz, tri


def fibonacci_sphere(n):
    """Convex hull of ``n`` Fibonacci-lattice points on the unit sphere."""
    from scipy.spatial import ConvexHull
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * np.pi * (3.0 - 5.0 ** 0.5)
    xyz = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
    hull = ConvexHull(xyz)
    tri = orient_outward(xyz, hull.simplices.astype(np.int32))
    return xyz, tri


def random_rotation(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def mean_edge_length(xyz, tri):
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    return float(np.mean(np.linalg.norm(xyz[e[:, 0]] - xyz[e[:, 1]], axis=1)))


def jitter_on_sphere(xyz, tri, frac, rng):
    """Move each vertex by tangential Gaussian noise of standard deviation
    ``frac`` times the mean edge length, then project back onto the sphere."""
    if frac <= 0:
        return xyz.copy()
    s = frac * mean_edge_length(xyz, tri)
    u = _normalise(xyz)
    g = rng.standard_normal(xyz.shape) * s
    g -= np.einsum("ij,ij->i", g, u)[:, None] * u
    return _normalise(xyz + g)


def scale_to_ellipsoid(xyz, axes):
    return xyz * np.asarray(axes, dtype=np.float64)[None, :]


def mesh_check(xyz, tri):
    """Closed, consistently oriented 2-manifold with positive enclosed volume,
    no degenerate triangle and no unused vertex.  Returns the signed volume."""
    tri = np.asarray(tri)
    nv = xyz.shape[0]
    assert tri.min() >= 0 and tri.max() < nv
    assert np.unique(tri).size == nv, "unused vertex"
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    key = e[:, 0].astype(np.int64) * nv + e[:, 1]
    assert np.unique(key).size == key.size, "edge used twice in one direction"
    rkey = e[:, 1].astype(np.int64) * nv + e[:, 0]
    assert np.all(np.isin(rkey, key)), "open or inconsistently oriented edge"
    p0, p1, p2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    a = 0.5 * np.linalg.norm(np.cross(p1 - p0, p2 - p0), axis=1)
    assert a.min() > 1e-12 * a.max(), "degenerate triangle"
    vol = np.sum(np.einsum("ij,ij->i", p0, np.cross(p1, p2))) / 6.0
    assert vol > 0, "inward orientation"
    return vol


def planar_square(m, sigma=0.0, rng=None):
    """Structured triangulation of [0,1]^2 (z = 0) with (m+1)^2 nodes.
    With ``sigma > 0`` interior nodes get 2-D Gaussian noise, boundary nodes
    move along their edge and the four corners stay fixed; noise is clipped to
    a third of the grid spacing so that the triangulation stays valid."""
    h = 1.0 / m
    g = np.linspace(0.0, 1.0, m + 1)
    X, Y = np.meshgrid(g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    if sigma > 0:
        d = np.clip(rng.standard_normal((xyz.shape[0], 2)) * sigma, -h / 3, h / 3)
        ix, iy = np.divmod(np.arange(xyz.shape[0]), m + 1)
        bx = (ix == 0) | (ix == m)
        by = (iy == 0) | (iy == m)
        d[bx, 0] = 0.0
        d[by, 1] = 0.0
        xyz[:, :2] += d
    tri = []
    for i in range(m):
        for j in range(m):
            a = i * (m + 1) + j
            b = (i + 1) * (m + 1) + j
            tri.append([a, b, b + 1])
            tri.append([a, b + 1, a + 1])
    return xyz, np.array(tri, dtype=np.int32)
