"""System matrices of the test problems (inputs to the solver, not part of it).

Cotan Laplacian and barycentric lumped mass follow the standard discrete
differential-geometry definitions (Wardetzky et al. 2007); the point-cloud
operator is a Gaussian-weighted kNN graph Laplacian with a kNN-disc mass.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class Problem:
    """One linear system on one geometry.

    points (n,3) f64, edges (m,2) int32, A as CSR (indptr, indices int32, data f64,
    sorted columns, symmetric pattern containing the diagonal), rhs (n,) f64.
    """
    name: str
    points: np.ndarray
    edges: np.ndarray
    indptr: np.ndarray
    indices: np.ndarray
    data: np.ndarray
    rhs: np.ndarray
    mass: np.ndarray = None       # the lumped mass diagonal M (right-hand sides are M y)

    @property
    def n(self):
        return int(self.points.shape[0])

    @property
    def m(self):
        return int(self.edges.shape[0])

    @property
    def nnz(self):
        return int(self.indices.shape[0])

    def matrix(self):
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.n, self.n))


def cotan_laplacian(points, faces):
    """Positive semi-definite cotan Laplacian L (L_ij = -(cot a + cot b)/2, L_ii = -sum_j L_ij)."""
    p = points
    f = np.asarray(faces, dtype=np.int64)
    n = p.shape[0]
    rows, cols, vals = [], [], []
    for k in range(3):
        i, j, o = f[:, (k + 1) % 3], f[:, (k + 2) % 3], f[:, k]
        e1 = p[i] - p[o]
        e2 = p[j] - p[o]
        cr = np.cross(e1, e2)
        cot = (e1 * e2).sum(1) / np.linalg.norm(cr, axis=1)
        w = -0.5 * cot
        rows += [i, j]
        cols += [j, i]
        vals += [w, w]
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    off = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    off.sum_duplicates()
    diag = -np.asarray(off.sum(axis=1)).ravel()
    return off, diag


def lumped_mass(points, faces):
    """Barycentric lumped mass: M_ii = sum of areas of incident triangles / 3."""
    p = points
    f = np.asarray(faces, dtype=np.int64)
    area = 0.5 * np.linalg.norm(np.cross(p[f[:, 1]] - p[f[:, 0]], p[f[:, 2]] - p[f[:, 0]]), axis=1)
    m = np.zeros(p.shape[0])
    for k in range(3):
        np.add.at(m, f[:, k], area / 3.0)
    return m


def gaussian_knn_laplacian(points, edges, knn_dist):
    """Graph Laplacian L = D - W with W_ij = exp(-|x_i - x_j|^2 / h^2), h = mean kNN distance,
    and mass M_ii = pi * d_(k)(i)^2 / (k + 1) with d_(k) the k-th neighbour distance."""
    n = points.shape[0]
    k = knn_dist.shape[1]
    h = float(knn_dist.mean())
    d = points[edges[:, 0]] - points[edges[:, 1]]
    w = np.exp(-(d * d).sum(1) / (h * h))
    r = np.concatenate([edges[:, 0], edges[:, 1]]).astype(np.int64)
    c = np.concatenate([edges[:, 1], edges[:, 0]]).astype(np.int64)
    off = sp.coo_matrix((np.concatenate([-w, -w]), (r, c)), shape=(n, n)).tocsr()
    off.sum_duplicates()
    diag = -np.asarray(off.sum(axis=1)).ravel()
    mass = np.pi * knn_dist[:, -1] ** 2 / (k + 1)
    return off, diag, mass


def assemble(off_lap, diag_lap, mass, alpha, edges, mass_weight=1.0):
    """A = mass_weight * M + alpha * L in CSR with sorted columns and pattern = edges U
    diagonal: the data-smoothing system (M + alpha L) by default, the Poisson system
    (L + eta M) with alpha = 1, mass_weight = eta.

    Structural zeros of the pattern are kept explicitly.
    """
    n = mass.shape[0]
    e = np.asarray(edges, dtype=np.int64)
    r = np.concatenate([e[:, 0], e[:, 1], np.arange(n)])
    c = np.concatenate([e[:, 1], e[:, 0], np.arange(n)])
    keys = np.unique(r * n + c)
    rows = keys // n
    indices = (keys % n).astype(np.int32)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=indptr[1:])
    coo = off_lap.tocoo()
    ko = coo.row.astype(np.int64) * n + coo.col.astype(np.int64)
    pos = np.searchsorted(keys, ko)
    if np.any(keys[np.minimum(pos, keys.size - 1)] != ko):
        raise ValueError("Laplacian entry outside the edge pattern")
    vals = np.bincount(pos, weights=alpha * coo.data, minlength=keys.size)
    dpos = np.searchsorted(keys, np.arange(n, dtype=np.int64) * n + np.arange(n))
    vals[dpos] += mass_weight * mass + alpha * diag_lap
    return indptr.astype(np.int32), indices, vals.astype(np.float64)
