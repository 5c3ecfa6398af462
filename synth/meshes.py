"""Synthetic surfaces and point clouds (geometry and connectivity only)."""
import numpy as np

from .rng import uniform, normal


def edges_from_faces(faces):
    """Unique undirected edges (u < v), sorted, of a triangle list; int32 (m, 2)."""
    f = np.asarray(faces, dtype=np.int64)
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=0)
    e.sort(axis=1)
    n = int(f.max()) + 1 if f.size else 0
    keys = np.unique(e[:, 0] * n + e[:, 1])
    return np.stack([keys // n, keys % n], 1).astype(np.int32)


def icosphere(subdivisions):
    """Unit icosphere: icosahedron, then `subdivisions` 4-to-1 splits.

    Vertex order: the 12 icosahedron vertices, then edge midpoints in creation
    order (each projected to the unit sphere).  Returns (points (n,3), faces (F,3)).
    """
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdivisions):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                p = verts[a] + verts[b]
                verts.append(p / np.linalg.norm(p))
                idx = len(verts) - 1
                cache[key] = idx
            return idx

        nf = []
        for (a, b, c) in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.array(verts, dtype=np.float64), np.array(faces, dtype=np.int32)


def torus_grid(nu, nv, R=1.0, r=0.4):
    """Torus as an nu x nv periodic (u, v) grid; vertex (i, j) has index i*nv + j.

    Each quad (i,j),(i+1,j),(i+1,j+1),(i,j+1) is split along its
    (i,j)-(i+1,j+1) diagonal.  Returns (points, faces).
    """
    i = np.arange(nu)[:, None]
    j = np.arange(nv)[None, :]
    u = 2.0 * np.pi * i / nu
    v = 2.0 * np.pi * j / nv
    x = (R + r * np.cos(v)) * np.cos(u)
    y = (R + r * np.cos(v)) * np.sin(u)
    z = np.broadcast_to(r * np.sin(v), x.shape)
    pts = np.stack([x, y, z], axis=-1).reshape(-1, 3).astype(np.float64)
    ii, jj = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    a = ii * nv + jj
    b = ((ii + 1) % nu) * nv + jj
    c = ((ii + 1) % nu) * nv + (jj + 1) % nv
    d = ii * nv + (jj + 1) % nv
    f1 = np.stack([a, b, c], axis=-1).reshape(-1, 3)
    f2 = np.stack([a, c, d], axis=-1).reshape(-1, 3)
    faces = np.empty((2 * f1.shape[0], 3), dtype=np.int32)
    faces[0::2] = f1
    faces[1::2] = f2
    return pts, faces


def flat_grid(nx, ny, h=1.0):
    """Planar (z = 0) nx x ny grid with spacing h, quads split along the (i,j)-(i+1,j+1) diagonal."""
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    pts = np.stack([ii * h, jj * h, np.zeros_like(ii, dtype=np.float64)], axis=-1)
    pts = pts.reshape(-1, 3).astype(np.float64)
    a = (ii[:-1, :-1] * ny + jj[:-1, :-1]).ravel()
    b = ((ii[:-1, :-1] + 1) * ny + jj[:-1, :-1]).ravel()
    c = ((ii[:-1, :-1] + 1) * ny + jj[:-1, :-1] + 1).ravel()
    d = (ii[:-1, :-1] * ny + jj[:-1, :-1] + 1).ravel()
    faces = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)], 0).astype(np.int32)
    return pts, faces


def mean_edge_length(points, edges):
    d = points[edges[:, 0]] - points[edges[:, 1]]
    return float(np.sqrt((d * d).sum(1)).mean())


def radial_noise(points, seed, amplitude):
    """x <- x * (1 + amplitude * U[-1, 1]) per vertex."""
    u = uniform(seed, "geom", points.shape[0], -1.0, 1.0)
    return points * (1.0 + amplitude * u)[:, None]


def gaussian_jitter(points, seed, sigma):
    """Isotropic 3-D Gaussian displacement with standard deviation sigma."""
    g = normal(seed, "jitter", 3 * points.shape[0]).reshape(-1, 3)
    return points + sigma * g


def bumpy_sphere_points(n, seed=0, bump=0.05, noise=1e-3, kmax=8):
    """n points on r(theta, phi) = 1 + bump * sum_k sin(k theta) cos(k phi), plus normal noise."""
    g = normal(seed, "dirs", 3 * n).reshape(n, 3)
    d = g / np.linalg.norm(g, axis=1, keepdims=True)
    theta = np.arccos(np.clip(d[:, 2], -1.0, 1.0))
    phi = np.arctan2(d[:, 1], d[:, 0])
    rad = np.ones(n)
    for k in range(1, kmax + 1):
        rad += bump * np.sin(k * theta) * np.cos(k * phi)
    pts = d * rad[:, None]
    pts += noise * normal(seed, "noise", 3 * n).reshape(n, 3)
    return pts.astype(np.float64)


def knn_edges(points, k):
    """Exact kNN graph (self excluded), symmetrised by union.

    Returns (edges (m,2) int32 with u < v, knn_idx (n,k), knn_dist (n,k)).
    """
    from scipy.spatial import cKDTree
    tree = cKDTree(points)
    dist, idx = tree.query(points, k=k + 1, workers=-1)
    n = points.shape[0]
    own = idx == np.arange(n)[:, None]
    # drop self (normally column 0; duplicates may move it), keep the first k others
    keep = ~own
    first = np.cumsum(keep, axis=1) <= k
    sel = keep & first
    idx_k = idx[sel].reshape(n, k)
    dist_k = dist[sel].reshape(n, k)
    u = np.repeat(np.arange(n), k)
    v = idx_k.ravel()
    keys = np.unique(np.minimum(u, v).astype(np.int64) * n + np.maximum(u, v))
    e = np.stack([keys // n, keys % n], 1).astype(np.int32)
    return e, idx_k, dist_k
