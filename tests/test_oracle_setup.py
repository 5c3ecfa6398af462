"""Pins of the CPU oracle's hierarchy construction (Sec. 4) against independent checks.

Every test here runs on the CPU.  Each check is formulated differently from
the oracle's own code path: characterisations instead of the sweep, dense
min-plus products instead of adjacency walks, SciPy's Dijkstra, exact
rational arithmetic, simplex-face enumeration, dense matrix products.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from tests import brute
from tests.conftest import problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SMALL = ["ico3", "ico4", "torus48", "flat", "pc4k"]


def hier(name, **opt):
    p = problem(name)
    o = oracle.default_options(min_coarse_points=opt.pop("min_coarse", 100), **opt)
    return p, oracle.Hierarchy.from_problem(p, o)


def test_splitmix64_reference_values():
    # SplitMix64 with state 0 yields 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4 (Steele et al. 2014)
    g = 0x9E3779B97F4A7C15
    assert oracle.mix64(g) == 0xE220A8397B1DCDAF
    assert oracle.mix64(2 * g) == 0x6E789E6AA1B965F4
    assert brute.mix64(g) == 0xE220A8397B1DCDAF
    for z in [0, 1, 12345, 2**63 + 5, 2**64 - 1]:
        assert oracle.mix64(z) == brute.mix64(z)


@pytest.mark.parametrize("name", SMALL)
def test_edges_canonical_and_weights(name):
    p, h = hier(name)
    lv = h.level(0)
    erp, ecol = lv["erp"], lv["ecol"]
    got = set()
    for i in range(p.n):
        row = ecol[erp[i]:erp[i + 1]]
        assert np.all(np.diff(row) > 0), "rows sorted, no duplicates"
        assert i not in row
        for j in row:
            got.add((min(i, j), max(i, j)))
    assert got == brute.edge_set(p.edges)
    rows = np.repeat(np.arange(p.n), np.diff(erp))
    d = p.points[rows] - p.points[ecol]
    w = np.sqrt((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
    assert np.array_equal(w, lv["ew"])


@pytest.mark.parametrize("name", SMALL)
def test_mean_edge_length_exact(name):
    """e_hat equals the exact rational mean of the edge lengths up to the fixed-point bound;
    r = 2 e_hat exactly for phi = 1/8 (Eq. 1)."""
    p, h = hier(name)
    X = h.export(0, oracle.POSITIONS)
    pairs = sorted(brute.edge_set(p.edges))
    exact = brute.exact_mean_edge(X, pairs)
    ehat, r = h.export(0, oracle.SCALARS)
    wmax = max(np.linalg.norm(X[u] - X[v]) for u, v in pairs)
    e = np.frexp(wmax)[1]
    lg = int(np.ceil(np.log2(len(pairs))))
    F = 62 - e - lg
    bound = 2.0 ** (-F - 1) + 4 * 2.0 ** -53 * float(exact)
    assert abs(float(exact) - ehat) <= bound
    assert r == 2.0 * ehat
    # coarser levels use the coarse points and coarse edges
    for l in range(1, h.num_levels - 1):
        lv = h.level(l)
        pr = [(i, j) for i in range(lv["n"]) for j in lv["ecol"][lv["erp"][i]:lv["erp"][i + 1]] if i < j]
        ex = brute.exact_mean_edge(lv["X"], pr)
        assert abs(float(ex) - lv["scalars"][0]) <= 1e-15 * float(ex) + 1e-300


def _check_lfmis(X, erp, ecol, r, samples, level, order=0, seed=0):
    n = X.shape[0]
    pairs = [(i, j) for i in range(n) for j in ecol[erp[i]:erp[i + 1]] if i < j]
    C = brute.conflict_matrix(X, pairs, r)
    assert np.array_equal(C, C.T)
    keys = brute.sweep_keys(n, level, seed, order)
    S = np.zeros(n, dtype=bool)
    S[samples] = True
    # independence
    assert not np.any(C[np.ix_(samples, samples)])
    # lexicographically first: every non-sample is blocked by an earlier sample
    for v in np.nonzero(~S)[0]:
        blockers = [u for u in np.nonzero(C[v] & S)[0] if keys[u] < keys[v]]
        assert blockers, f"point {v} is not blocked by an earlier sample"
    # and every sample had no earlier sample in conflict (implied by independence)
    return C


@pytest.mark.parametrize("name", SMALL)
def test_sampling_is_lexicographically_first_mis(name):
    p, h = hier(name)
    for l in range(h.num_levels - 1):
        lv = h.level(l)
        _check_lfmis(lv["X"], lv["erp"], lv["ecol"], lv["scalars"][1], lv["samples"], l)


def test_sampling_index_order_and_seed():
    p, h = hier("torus48", sample_order=1)
    lv = h.level(0)
    _check_lfmis(lv["X"], lv["erp"], lv["ecol"], lv["scalars"][1], lv["samples"], 0, order=1)
    p, h2 = hier("torus48", seed=77)
    lv2 = h2.level(0)
    _check_lfmis(lv2["X"], lv2["erp"], lv2["ecol"], lv2["scalars"][1], lv2["samples"], 0, seed=77)
    assert not np.array_equal(lv["samples"], lv2["samples"])


def test_sequential_sweep_brute_force():
    """Direct restatement on a tiny mesh: sweep in key order over the dense conflict matrix."""
    p, h = hier("ico3")
    lv = h.level(0)
    n = lv["n"]
    pairs = [(i, j) for i in range(n) for j in lv["ecol"][lv["erp"][i]:lv["erp"][i + 1]] if i < j]
    C = brute.conflict_matrix(lv["X"], pairs, lv["scalars"][1])
    elig = np.ones(n, dtype=bool)
    S = []
    for _, v in sorted(brute.sweep_keys(n, 0)):
        if elig[v]:
            S.append(v)
            elig[C[v]] = False
            elig[v] = False
    assert sorted(S) == lv["samples"].tolist()


def _voronoi_fixed_point(erp, ecol, w, samples, dist, labels):
    n = erp.shape[0] - 1
    sid = -np.ones(n, dtype=np.int64)
    sid[samples] = np.arange(samples.size)
    for v in range(n):
        if sid[v] >= 0:
            assert dist[v] == 0.0 and labels[v] == sid[v]
            continue
        nb = ecol[erp[v]:erp[v + 1]]
        cand = dist[nb] + w[erp[v]:erp[v + 1]]
        dmin = cand.min()
        lmin = labels[nb][cand == dmin].min()
        assert dist[v] == dmin and labels[v] == lmin, f"point {v} is not at the fixed point"


@pytest.mark.parametrize("name", SMALL)
def test_voronoi_fixed_point_and_dijkstra(name):
    p, h = hier(name)
    for l in range(h.num_levels - 1):
        lv = h.level(l)
        _voronoi_fixed_point(lv["erp"], lv["ecol"], lv["ew"], lv["samples"], lv["dist"], lv["labels"])
        D = brute.multi_source_dijkstra(lv["X"], lv["erp"], lv["ecol"], lv["samples"])
        best = D.min(axis=0)
        assert np.array_equal(best, lv["dist"]) or np.allclose(best, lv["dist"], rtol=1e-15, atol=0)
        arg = D.argmin(axis=0)
        tie = (D == best[None, :]).sum(axis=0) > 1
        ok = ~tie
        assert np.array_equal(arg[ok], lv["labels"][ok])


def path_hierarchy(n, phi, x=None):
    X = np.zeros((n, 3))
    X[:, 0] = np.arange(n, dtype=np.float64) if x is None else np.array(x, dtype=np.float64)
    edges = np.array([[i, i + 1] for i in range(n - 1)], dtype=np.int32)
    rp = [0]
    ci, va = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                ci.append(j)
                va.append(2.5 if i == j else -1.0)
        rp.append(len(ci))
    o = oracle.default_options(min_coarse_points=1, max_levels=2, sample_order=1, coarsening_ratio=phi)
    return oracle.Hierarchy(X, edges, np.array(rp), np.array(ci), np.array(va), o)


def test_sampling_and_voronoi_on_a_path():
    """Golden: unit paths where points sit exactly at the radius and exactly between two seeds."""
    g = json.load(open(os.path.join(GOLDEN, "path_ties.json")))
    for case in g["cases"]:
        h = path_hierarchy(case["n"], case["phi"], case.get("x"))
        lv = h.level(0)
        assert lv["scalars"][0] == (2.0 if "x" in case else 1.0)
        assert lv["samples"].tolist() == case["samples"], case["derivation"]
        assert lv["labels"].tolist() == case["labels"]
        assert lv["dist"].tolist() == case["dist"]


@pytest.mark.parametrize("name", SMALL)
def test_cells_shift_and_coarse_edges(name):
    p, h = hier(name)
    for l in range(h.num_levels - 1):
        lv, nx = h.level(l), h.level(l + 1)
        X, lab = lv["X"], lv["labels"]
        nc = nx["n"]
        assert nc == lv["samples"].size
        for I in range(nc):
            mem = np.nonzero(lab == I)[0]
            seq = np.cumsum(X[mem], axis=0)[-1] / mem.size      # sequential ascending sums
            assert np.array_equal(seq, nx["X"][I])
            exact = [sum(map(__import__("fractions").Fraction, X[mem, k])) / mem.size for k in range(3)]
            assert np.allclose(nx["X"][I], [float(e) for e in exact], rtol=0, atol=1e-14)
        want = set()
        for u in range(lv["n"]):
            for v in lv["ecol"][lv["erp"][u]:lv["erp"][u + 1]]:
                if lab[u] != lab[v]:
                    want.add((int(lab[u]), int(lab[v])))
        got = set()
        for I in range(nc):
            row = nx["ecol"][nx["erp"][I]:nx["erp"][I + 1]]
            assert np.all(np.diff(row) > 0)
            got |= {(I, int(J)) for J in row}
        assert got == want


def test_no_shift_keeps_sample_positions():
    p, h = hier("torus48", shift_coarse_points=0)
    lv, nx = h.level(0), h.level(1)
    assert np.array_equal(nx["X"], lv["X"][lv["samples"]])


def test_equal_distance_candidates_keep_the_first():
    """Without the shift a sample coincides with its coarse point, so every candidate triangle
    is at distance 0: the first non-degenerate candidate in (j, k) order must be chosen and the
    row must be the single entry {c: 1}."""
    for name in ["torus48", "ico4", "pc4k"]:
        p, h = hier(name, shift_coarse_points=0)
        lv, nx = h.level(0), h.level(1)
        Xc = nx["X"]
        checked = 0
        for I, s in enumerate(lv["samples"]):
            c = lv["labels"][s]
            assert c == I
            good = [(j, k) for j, k in _candidate_triangles(nx, c)
                    if brute.sin2_angle(Xc[c], Xc[j], Xc[k]) > 1e-12 * 1.01]
            if not good:
                continue
            assert tuple(lv["tri"][s]) == good[0]
            assert lv["pcnt"][s] == 1 and lv["pcol"][s, 0] == c and lv["pval"][s, 0] == 1.0
            checked += 1
        assert checked > 0


def test_closest_point_golden():
    g = json.load(open(os.path.join(GOLDEN, "closest_point.json")))
    A, B, C = (np.array(v, dtype=np.float64) for v in g["triangle"])
    for case in g["cases"]:
        w, region = oracle.closest_point(np.array(case["p"], dtype=np.float64), A, B, C)
        assert region == case["region"], case
        assert np.allclose(w, case["w"], rtol=0, atol=1e-15), case


def test_closest_point_vs_simplex_enumeration():
    rng = np.random.default_rng(0)
    regions = set()
    for trial in range(4000):
        A, B, C = rng.normal(size=(3, 3))
        if brute.sin2_angle(A, B, C) < 1e-6:
            continue
        P = (A + B + C) / 3 + rng.normal(size=3) * rng.choice([0.1, 1.0, 3.0])
        w, region = oracle.closest_point(P, A, B, C)
        regions.add(region)
        assert np.all(w >= 0) and abs(w.sum() - 1) <= 4e-16 * 4
        q = w[0] * A + w[1] * B + w[2] * C
        d2 = (P - q) @ (P - q)
        wb, d2b = brute.closest_point_simplex(P, A, B, C)
        scale = (P - A) @ (P - A) + (B - A) @ (B - A) + (C - A) @ (C - A)
        assert abs(d2 - d2b) <= 1e-12 * scale
        assert np.allclose(w, wb, atol=1e-7)
    assert regions == set(range(7)), "all seven regions exercised"


def test_degenerate_threshold():
    A = np.zeros(3)
    assert oracle.degenerate(A, np.array([1.0, 0, 0]), np.array([2.0, 0, 0]))
    assert not oracle.degenerate(A, np.array([1.0, 0, 0]), np.array([0.0, 1, 0]))
    # sin^2 of the angle at A: 1e-11 is kept, 1e-13 is rejected (tau = 1e-12)
    for s2, deg in [(1e-11, False), (1e-13, True)]:
        t = np.sqrt(s2 / (1 - s2))
        C = np.array([1.0, t, 0.0])
        assert oracle.degenerate(A, np.array([1.0, 0, 0]), C) == deg


def _candidate_triangles(nx, c):
    nb = set(nx["ecol"][nx["erp"][c]:nx["erp"][c + 1]].tolist())
    out = []
    for j in sorted(nb):
        nj = set(nx["ecol"][nx["erp"][j]:nx["erp"][j + 1]].tolist())
        for k in sorted(nb):
            if k > j and k in nj:
                out.append((j, k))
    return out


@pytest.mark.parametrize("name", SMALL)
def test_prolongation_rows(name):
    """Rows of P: 1..3 positive entries summing to 1; chosen triangle is the closest candidate."""
    p, h = hier(name)
    for l in range(h.num_levels - 1):
        lv, nx = h.level(l), h.level(l + 1)
        pcnt, pcol, pval, tri = lv["pcnt"], lv["pcol"], lv["pval"], lv["tri"]
        assert np.all((pcnt >= 1) & (pcnt <= 3))
        for i in range(lv["n"]):
            k = pcnt[i]
            assert np.all(pval[i, :k] > 0) and np.all(np.diff(pcol[i, :k]) > 0)
            assert np.all(pcol[i, k:] == -1) and np.all(pval[i, k:] == 0)
            assert abs(pval[i, :k].sum() - 1.0) <= 4 * 2.0 ** -52
        X, Xc, lab = lv["X"], nx["X"], lv["labels"]
        checked = 0
        for i in range(0, lv["n"], max(1, lv["n"] // 400)):
            c = lab[i]
            cands = _candidate_triangles(nx, c)
            good = [(j, k) for j, k in cands if brute.sin2_angle(Xc[c], Xc[j], Xc[k]) > 1e-12 * 1.01]
            if tri[i, 0] < 0:
                assert not good, f"fallback used although {good} exist"
                continue
            d2 = {(j, k): brute.closest_point_simplex(X[i], Xc[c], Xc[j], Xc[k])[1] for j, k in good}
            best = min(d2.values())
            scale = max((X[i] - Xc[c]) @ (X[i] - Xc[c]), 1e-300)
            assert abs(d2[(tri[i, 0], tri[i, 1])] - best) <= 1e-12 * scale
            checked += 1
        assert checked > 0


def test_linear_precision_on_flat_grid():
    """On a planar mesh, rows projected into a triangle's face reproduce the point exactly."""
    p, h = hier("flat", min_coarse=50)
    lv, nx = h.level(0), h.level(1)
    face = 0
    for i in range(lv["n"]):
        if lv["tri"][i, 0] < 0 or lv["pcnt"][i] != 3:
            continue
        q = sum(lv["pval"][i, t] * nx["X"][lv["pcol"][i, t]] for t in range(3))
        if np.abs(q - lv["X"][i]).max() <= 1e-12 * 40:
            face += 1
        else:
            # not in the face: the point lies outside every candidate triangle
            c = lv["labels"][i]
            cands = _candidate_triangles(nx, c)
            inside = False
            for j, k in cands:
                w, d2 = brute.closest_point_simplex(lv["X"][i], nx["X"][c], nx["X"][j], nx["X"][k])
                inside |= d2 <= 1e-20
            assert not inside
    assert face > 0.8 * lv["n"]


def test_fallback_inverse_distance_golden():
    """Golden: points on a line (all candidate triangles co-linear) use inverse-distance weights."""
    g = json.load(open(os.path.join(GOLDEN, "fallback_line.json")))
    n = g["n"]
    X = np.zeros((n, 3))
    X[:, 0] = np.array(g["x"], dtype=np.float64)
    edges = np.array([[i, i + 1] for i in range(n - 1)] + [[i, i + 2] for i in range(n - 2)],
                     dtype=np.int32)
    import scipy.sparse as sp
    r = np.concatenate([edges[:, 0], edges[:, 1], np.arange(n)])
    c = np.concatenate([edges[:, 1], edges[:, 0], np.arange(n)])
    v = np.concatenate([-np.ones(2 * len(edges)), 10 * np.ones(n)])
    A = sp.csr_matrix((v, (r, c)), shape=(n, n))
    A.sort_indices()
    o = oracle.default_options(min_coarse_points=1, max_levels=2, sample_order=1)
    h = oracle.Hierarchy(X, edges, A.indptr, A.indices, A.data, o)
    lv, nx = h.level(0), h.level(1)
    assert lv["samples"].tolist() == g["samples"]
    assert np.all(lv["tri"] == -1), "no non-degenerate triangle exists on a line"
    for i, row in enumerate(g["rows"]):
        k = lv["pcnt"][i]
        assert lv["pcol"][i, :k].tolist() == row["cols"], i
        assert np.allclose(lv["pval"][i, :k], row["w"], rtol=1e-14, atol=0), i
    assert h.sizes(0)["fallback"] == n


@pytest.mark.parametrize("name", SMALL)
def test_galerkin_against_dense_product(name):
    p, h = hier(name)
    for l in range(h.num_levels - 1):
        lv, nx = h.level(l), h.level(l + 1)
        n, nc = lv["n"], nx["n"]
        A = brute.dense(lv["arp"], lv["acol"], lv["aval"], (n, n))
        Apat = brute.dense(lv["arp"], lv["acol"], np.ones_like(lv["aval"]), (n, n))
        P = brute.ell_to_dense(lv["pcol"], lv["pval"], lv["pcnt"], nc)
        Ac = brute.dense(nx["arp"], nx["acol"], nx["aval"], (nc, nc))
        ref = P.T @ A @ P
        scale = np.abs(P).T @ np.abs(A) @ np.abs(P)
        assert np.all(np.abs(Ac - ref) <= 1e-12 * scale + 1e-300)
        pat = ((P != 0).astype(float).T @ Apat @ (P != 0).astype(float)) > 0
        got = brute.dense(nx["arp"], nx["acol"], np.ones_like(nx["aval"]), (nc, nc)) > 0
        assert np.array_equal(pat, got)
        assert np.all(np.abs(Ac - Ac.T) <= 1e-12 * scale + 1e-300)
        # P 1 = 1, so 1^T A_{l+1} 1 = 1^T A_l 1
        assert abs(Ac.sum() - A.sum()) <= 1e-10 * np.abs(A).sum()


def test_galerkin_keeps_constants_in_the_null_space():
    """For a Laplacian (A 1 = 0, shifted by 1e-9 I to stay SPD), P 1 = 1 keeps the coarse
    operators' row sums at the level of the shift."""
    import scipy.sparse as sp
    p = problem("torus48")
    M = p.matrix()
    off = M - sp.diags(M.diagonal())
    L = (off - sp.diags(np.asarray(off.sum(axis=1)).ravel() - 1e-9)).tocsr()
    L.sort_indices()
    h = oracle.Hierarchy(p.points, p.edges, L.indptr, L.indices, L.data,
                         oracle.default_options(min_coarse_points=100))
    assert h.num_levels >= 2
    for l in range(h.num_levels - 1):
        lv, nx = h.level(l), h.level(l + 1)
        A = brute.dense(lv["arp"], lv["acol"], lv["aval"], (lv["n"], lv["n"]))
        P = brute.ell_to_dense(lv["pcol"], lv["pval"], lv["pcnt"], nx["n"])
        Ac = brute.dense(nx["arp"], nx["acol"], nx["aval"], (nx["n"], nx["n"]))
        scale = (np.abs(P).T @ np.abs(A) @ np.abs(P)).sum(axis=1)
        # A_{l+1} 1 = P^T A P 1 = P^T (A 1) because P 1 = 1
        assert np.all(np.abs(Ac @ np.ones(nx["n"]) - P.T @ (A @ np.ones(lv["n"]))) <= 1e-12 * scale)
        # the row sums are the shift carried down by P^T, far below the diagonal
        assert np.all(np.abs(Ac @ np.ones(nx["n"])) <= 1e-3 * np.diag(Ac))


@pytest.mark.parametrize("name", SMALL)
def test_colouring_first_fit(name):
    """Without recolouring passes: first-fit in hashed key order (Jones-Plassmann)."""
    p, h = hier(name, color_passes=0)
    for l in range(h.num_levels - 1):
        lv = h.level(l)
        col = lv["colors"]
        keys = brute.color_keys(lv["n"], l)
        for v in range(lv["n"]):
            nb = [u for u in lv["acol"][lv["arp"][v]:lv["arp"][v + 1]] if u != v]
            assert all(col[u] != col[v] for u in nb)
            lower = {int(col[u]) for u in nb if keys[u] < keys[v]}
            mex = 0
            while mex in lower:
                mex += 1
            assert col[v] == mex


def _iterated_greedy(arp, acol, col, passes):
    """Culberson's iterated greedy colouring, written out: each pass colours the
    vertices first-fit, the classes of the previous colouring visited from the
    highest colour down and by index within a class."""
    n = len(col)
    nb = [[u for u in acol[arp[v]:arp[v + 1]] if u != v] for v in range(n)]
    for _ in range(passes):
        order = sorted(range(n), key=lambda v: (-col[v], v))
        new = [-1] * n
        for v in order:
            used = {new[u] for u in nb[v] if new[u] >= 0}
            c = 0
            while c in used:
                c += 1
            new[v] = c
        col = new
    return col


@pytest.mark.parametrize("name", SMALL)
def test_colouring_iterated_greedy(name):
    """The default colouring (3 recolouring passes): valid; first-fit (every vertex of
    colour c has neighbours of all colours below c); never more colours than the
    first colouring nor than the previous pass; equal to the passes written out from
    the pinned first colouring."""
    p, h0 = hier(name, color_passes=0)
    counts = [h0.sizes(l)["colors"] for l in range(h0.num_levels - 1)]
    for passes in (1, 2, 3):
        _, h = hier(name, color_passes=passes)
        assert h.num_levels == h0.num_levels
        for l in range(h.num_levels - 1):
            lv, l0 = h.level(l), h0.level(l)
            col = lv["colors"]
            nc = int(col.max()) + 1
            assert h.sizes(l)["colors"] == nc <= counts[l]
            counts[l] = nc
            for v in range(lv["n"]):
                nb = [u for u in lv["acol"][lv["arp"][v]:lv["arp"][v + 1]] if u != v]
                seen = {int(col[u]) for u in nb}
                assert col[v] not in seen
                assert all(c in seen for c in range(col[v]))
            if passes == 3:
                ref = _iterated_greedy(l0["arp"], l0["acol"], list(l0["colors"]), 3)
                assert list(col) == ref
    # the default options are these three passes
    _, hd = hier(name)
    for l in range(hd.num_levels - 1):
        assert np.array_equal(hd.level(l)["colors"], h.level(l)["colors"])


def test_colour_passes_out_of_range():
    p = problem("ico3")
    for k in (-1, 65):
        with pytest.raises(oracle.OracleError):
            oracle.Hierarchy.from_problem(p, oracle.default_options(color_passes=k))


@pytest.mark.parametrize("name", SMALL)
def test_levels_and_coarsest_factor(name):
    p, h = hier(name)
    sizes = [h.sizes(l)["n"] for l in range(h.num_levels)]
    assert sizes[-1] <= 100 < sizes[-2]
    for a, b in zip(sizes, sizes[1:]):
        assert b < a
    lv = h.level(h.num_levels - 1)
    Ac = brute.dense(lv["arp"], lv["acol"], lv["aval"], (lv["n"], lv["n"]))
    Lref = np.linalg.cholesky(Ac)
    assert np.allclose(h.chol(), Lref, rtol=0, atol=1e-12 * np.abs(Lref).max())


def test_coarsening_ratio_near_phi():
    """Roughly log_8(N / 1000) levels: each level keeps about 1/8 of the points (Sec. 4.2)."""
    p, h = hier("ico5", min_coarse=1000)
    sizes = [h.sizes(l)["n"] for l in range(h.num_levels)]
    for a, b in zip(sizes, sizes[1:]):
        assert 1 / 12 < b / a < 1 / 4


def test_invalid_inputs():
    p = problem("ico3")
    pts = p.points.copy()
    pts[3, 1] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.Hierarchy(pts, p.edges, p.indptr, p.indices, p.data)
    assert e.value.status == -1
    bad = p.edges.copy()
    bad[0, 0] = p.n
    with pytest.raises(oracle.OracleError) as e:
        oracle.Hierarchy(p.points, bad, p.indptr, p.indices, p.data)
    assert e.value.status == -1
    data = p.data.copy()
    data[p.indptr[5]:p.indptr[6]][p.indices[p.indptr[5]:p.indptr[6]] == 5] = 0.0
    with pytest.raises(oracle.OracleError) as e:
        oracle.Hierarchy(p.points, p.edges, p.indptr, p.indices, data)
    assert e.value.status == -4
