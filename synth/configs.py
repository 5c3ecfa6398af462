"""The workloads: named, seeded problems of the sizes the method is measured on.

The paper measures on scanned meshes and point clouds (data smoothing,
(M + alpha S) x = M y); those datasets are not available, so these seeded
synthetic surfaces of the same size range and the same system class stand in
for them.
"""
import numpy as np

from .meshes import (icosphere, torus_grid, flat_grid, bumpy_sphere_points, edges_from_faces,
                     knn_edges, mean_edge_length, radial_noise, gaussian_jitter)
from .operators import cotan_laplacian, lumped_mass, gaussian_knn_laplacian, assemble, Problem
from .rng import uniform, normal


def _mesh_problem(name, pts, faces, alpha, seed, eta=None):
    edges = edges_from_faces(faces)
    off, diag = cotan_laplacian(pts, faces)
    mass = lumped_mass(pts, faces)
    if eta is None:                                   # data smoothing (M + alpha L) x = M y
        indptr, indices, data = assemble(off, diag, mass, alpha, edges)
    else:                                             # Poisson (L + eta M) x = M y
        indptr, indices, data = assemble(off, diag, mass, 1.0, edges, mass_weight=eta)
    y = uniform(seed, "rhs", pts.shape[0], -1.0, 1.0)
    return Problem(name, np.ascontiguousarray(pts), edges, indptr, indices, data, mass * y, mass)


def config_icosphere(subdivisions=5, seed=0, noise=0.01, alpha=1e-3):
    """Icosphere (5 subdivisions: 10,242 vertices), radial noise +-1%, (M + 1e-3 L) x = M b."""
    pts, faces = icosphere(subdivisions)
    pts = radial_noise(pts, seed, noise)
    return _mesh_problem(f"icosphere{subdivisions}", pts, faces, alpha, seed)


def config_torus(nu=1024, nv=1024, seed=0, alpha=1e-3, jitter=0.1):
    """Torus R=1, r=0.4 on an nu x nv grid, Gaussian jitter sigma = 0.1 * mean edge length."""
    pts, faces = torus_grid(nu, nv)
    sigma = jitter * mean_edge_length(pts, edges_from_faces(faces))
    pts = gaussian_jitter(pts, seed, sigma)
    return _mesh_problem(f"torus{nu}x{nv}", pts, faces, alpha, seed)


def config_bumpy_sphere(n=2_000_000, k=8, seed=0, alpha=1e-2):
    """Bumpy-sphere point cloud, symmetrised kNN graph, Gaussian graph Laplacian, (M + 1e-2 L)."""
    pts = bumpy_sphere_points(n, seed)
    edges, _, kd = knn_edges(pts, k)
    off, diag, mass = gaussian_knn_laplacian(pts, edges, kd)
    indptr, indices, data = assemble(off, diag, mass, alpha, edges)
    y = uniform(seed, "rhs", n, -1.0, 1.0)
    return Problem(f"bumpysphere{n}k{k}", pts, edges, indptr, indices, data, mass * y, mass)


def config_poisson(nu=96, nv=80, seed=0, eta=1e-6, jitter=0.1):
    """The Poisson problem of the paper's comparisons, (L + eta M) x = M y with eta = 1e-6,
    y ~ U[-1, 1], on the jittered torus."""
    pts, faces = torus_grid(nu, nv)
    sigma = jitter * mean_edge_length(pts, edges_from_faces(faces))
    pts = gaussian_jitter(pts, seed, sigma)
    return _mesh_problem(f"poisson_torus{nu}x{nv}", pts, faces, None, seed, eta=eta)


def config_adjoint(nu=707, nv=707, seed=0, alpha=1e-3):
    """Differentiation workload: the jittered torus (707 x 707 = 499,849 vertices),
    (M + 1e-3 L) x = M b, loss ||x - x*||^2 with target x* ~ U[-1, 1].  Returns the
    problem, x* and a seeded choice of 32 stored entries of A and 8 entries of b
    (indices) for finite-difference checks."""
    prob = config_torus(nu, nv, seed, alpha)
    target = uniform(seed, "target", prob.n, -1.0, 1.0)
    u = uniform(seed, "entries", 40, 0.0, 1.0)
    a_idx = np.minimum((u[:32] * prob.nnz).astype(np.int64), prob.nnz - 1)
    b_idx = np.minimum((u[32:] * prob.n).astype(np.int64), prob.n - 1)
    return prob, target, a_idx, b_idx


def config_batched(count=64, nrhs=8, lo=5_000, hi=200_000, seed=0):
    """Many meshes of uneven size, several right-hand sides each: vertex counts
    log-uniform in [lo, hi] (seeded); even entries are jittered tori whose grid
    is chosen to hit the count, odd entries jittered icospheres with the
    subdivision level nearest to it (in log scale).  (M + 1e-3 L) systems;
    returns a list of (Problem, B) with B of shape (nrhs, n), B_q = M y_q,
    y_q ~ U[-1, 1]."""
    u = uniform(seed, "sizes", count, 0.0, 1.0)
    sizes = np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))
    out = []
    for i, target in enumerate(sizes):
        if i % 2 == 0:
            nu = max(8, int(round(np.sqrt(target * 1.6))))
            nv = max(8, int(round(target / nu)))
            prob = config_torus(nu, nv, seed=seed + i)
        else:
            sub = int(np.argmin([abs(np.log((10 * 4 ** k + 2) / target)) for k in range(2, 8)])) + 2
            prob = config_icosphere(sub, seed=seed + i)
        ys = uniform(seed + i, "noise", nrhs * prob.n, -1.0, 1.0).reshape(nrhs, prob.n)
        out.append((prob, prob.mass[None, :] * ys))
    return out


def small_icosphere(subdivisions=3, seed=0):
    return config_icosphere(subdivisions, seed)


def small_torus(nu=48, nv=40, seed=0):
    return config_torus(nu, nv, seed)


def small_flat_grid(nx=24, ny=20, seed=0, jitter=0.2, alpha=1e-3):
    """Planar jittered grid (z stays exactly 0)."""
    pts, faces = flat_grid(nx, ny)
    j = uniform(seed, "jitter", 2 * pts.shape[0], -jitter, jitter).reshape(-1, 2)
    pts = pts.copy()
    pts[:, :2] += j
    return _mesh_problem(f"flat{nx}x{ny}", pts, faces, alpha, seed)


def small_pointcloud(n=4000, k=8, seed=0):
    return config_bumpy_sphere(n, k, seed)


def small_hubs(nu=96, nv=80, hubs=3, spokes=150, seed=0):
    """The small torus with a few hub points, each joined to `spokes` points drawn
    at random: long rows in every operator of the hierarchy.  A = L + I with L
    the unit-weight Laplacian of the edge graph (symmetric, diagonally
    dominant); rhs standard normal."""
    import scipy.sparse as sp
    base = config_torus(nu, nv, seed)
    n = base.n
    draws = uniform(seed, "hubs", hubs * (spokes + 1))
    idx = np.minimum((draws * n).astype(np.int64), n - 1).reshape(hubs, spokes + 1)
    extra = [(min(r[0], o), max(r[0], o)) for r in idx for o in r[1:] if o != r[0]]
    e = np.sort(base.edges.astype(np.int64), axis=1)
    e = np.unique(np.concatenate([e, np.array(extra, dtype=np.int64)]), axis=0)
    w = sp.coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n, n)).tocsr()
    w = (w + w.T).tocsr()
    w.data[:] = 1.0
    deg = np.asarray(w.sum(axis=1)).ravel()
    a = (sp.diags(deg + 1.0) - w).tocsr()
    a.sort_indices()
    return Problem(f"hubs{nu}x{nv}", base.points, e.astype(np.int32), a.indptr.astype(np.int32),
                   a.indices.astype(np.int32), a.data.astype(np.float64), normal(seed, "rhs", n))


CONFIGS = {
    "icosphere5": config_icosphere,
    "torus1024": config_torus,
    "bumpysphere2m": config_bumpy_sphere,
    "adjoint_torus707": config_adjoint,
    "batched64": config_batched,
}
