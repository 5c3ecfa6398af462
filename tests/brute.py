"""Independent brute-force checkers for the oracle (NumPy / SciPy / plain Python).

These restate each property from its mathematical definition with different
machinery than the oracle (dense min-plus products, SciPy Dijkstra, exact
rationals, simplex enumeration), so that a mistake in the oracle shows up as
a disagreement.
"""
from fractions import Fraction

import numpy as np
import scipy.sparse as sp

M64 = (1 << 64) - 1


def mix64(z):
    """SplitMix64 finaliser written out on Python integers."""
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def sweep_keys(n, level, seed=0, order=0):
    if order == 1:
        return [(0, v) for v in range(n)]
    return [(mix64(seed ^ (level << 32) ^ v), v) for v in range(n)]


def color_keys(n, level, seed=0):
    salt = 0xC2B2AE3D27D4EB4F
    return [(mix64((seed ^ salt) ^ (level << 32) ^ v), v) for v in range(n)]


def csr_adjacency(erp, ecol):
    return [list(ecol[erp[i]:erp[i + 1]]) for i in range(len(erp) - 1)]


def edge_set(edges):
    s = set()
    for u, v in np.asarray(edges).tolist():
        if u != v:
            s.add((min(u, v), max(u, v)))
    return s


def conflict_matrix(X, edge_pairs, r):
    """Dense boolean conflict relation: q within path length r of p over paths of <= 2 edges.

    One-edge lengths D1 and two-edge lengths D2 = min_m (D1[p, m] + D1[m, q]) are
    formed as dense min-plus products (n <= a few thousand)."""
    n = X.shape[0]
    D1 = np.full((n, n), np.inf)
    for u, v in edge_pairs:
        d = X[u] - X[v]
        w = np.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])
        D1[u, v] = D1[v, u] = w
    C = D1 <= r
    for p in range(n):
        nb = np.nonzero(np.isfinite(D1[p]))[0]
        if nb.size == 0:
            continue
        two = (D1[p, nb][:, None] + D1[nb, :]).min(axis=0)
        C[p] |= two <= r
    np.fill_diagonal(C, False)
    return C


def exact_mean_edge(X, edge_pairs):
    s = Fraction(0)
    for u, v in edge_pairs:
        d = X[u] - X[v]
        w = float(np.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]))
        s += Fraction(w)
    return s / len(edge_pairs)


def closest_point_simplex(P, A, B, C):
    """Closest point of triangle ABC to P by enumerating the faces of the simplex.

    Candidates: the interior stationary point of |P - (A + s(B-A) + t(C-A))|^2
    (2x2 normal equations, accepted if inside), the clamped projection on each
    edge, and the three vertices.  Returns (weights, squared distance)."""
    P, A, B, C = (np.asarray(v, dtype=np.float64) for v in (P, A, B, C))
    cands = []
    E1, E2 = B - A, C - A
    G = np.array([[E1 @ E1, E1 @ E2], [E1 @ E2, E2 @ E2]])
    rhs = np.array([E1 @ (P - A), E2 @ (P - A)])
    try:
        s, t = np.linalg.solve(G, rhs)
        if s >= 0 and t >= 0 and s + t <= 1:
            cands.append(np.array([1 - s - t, s, t]))
    except np.linalg.LinAlgError:
        pass
    V = [A, B, C]
    for a, b in [(0, 1), (0, 2), (1, 2)]:
        d = V[b] - V[a]
        dd = d @ d
        t = 0.0 if dd == 0 else float(np.clip((P - V[a]) @ d / dd, 0.0, 1.0))
        w = np.zeros(3)
        w[a], w[b] = 1 - t, t
        cands.append(w)
    for a in range(3):
        w = np.zeros(3)
        w[a] = 1.0
        cands.append(w)
    best = None
    for w in cands:
        q = w[0] * A + w[1] * B + w[2] * C
        d2 = float((P - q) @ (P - q))
        if best is None or d2 < best[1]:
            best = (w, d2)
    return best


def sin2_angle(A, B, C):
    ab, ac = np.asarray(B) - A, np.asarray(C) - A
    c = np.cross(ab, ac)
    den = (ab @ ab) * (ac @ ac)
    return float(c @ c / den) if den > 0 else 0.0


def multi_source_dijkstra(X, erp, ecol, seeds):
    """SciPy Dijkstra from every seed: dense (len(seeds), n) distance table."""
    from scipy.sparse.csgraph import dijkstra
    n = X.shape[0]
    rows = np.repeat(np.arange(n), np.diff(erp))
    d = X[rows] - X[ecol]
    w = np.sqrt((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
    G = sp.csr_matrix((w, ecol, erp), shape=(n, n))
    return dijkstra(G, directed=True, indices=np.asarray(seeds))


def dense(rp, ci, va, shape):
    return sp.csr_matrix((va, ci, rp), shape=shape).toarray()


def ell_to_dense(pcol, pval, pcnt, nc):
    n = pcnt.shape[0]
    P = np.zeros((n, nc))
    for i in range(n):
        for t in range(pcnt[i]):
            P[i, pcol[i, t]] += pval[i, t]
    return P
