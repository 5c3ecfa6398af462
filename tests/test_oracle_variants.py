"""Pins of the oracle's prolongation variants (the weighting ablation of
Sec. 5.3, the fallback-trigger reading of Sec. 4.4) and of the Poisson system
of the comparisons (Sec. 5.4).

The variants change only the weights (or send vertex projections to the
fallback); the geometric hierarchy (samples, cells, coarse edges, triangle
choices) must stay the same.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.conftest import problem

GEOMETRIC = ["samples", "labels", "dist", "X", "erp", "ecol"]


def hier(name, **opt):
    p = problem(name)
    return p, oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=200, **opt))


@pytest.mark.parametrize("name", ["torus96", "pc4k", "flat"])
def test_uniform_weights(name):
    p, h0 = hier(name)
    _, h1 = hier(name, weighting=1)
    for l in range(h0.num_levels - 1):
        a, b = h0.level(l), h1.level(l)
        for k in GEOMETRIC + ["tri"]:
            assert np.array_equal(a[k], b[k]), (l, k)
        tri = b["tri"].reshape(-1, 2)
        has = tri[:, 0] >= 0
        assert np.all(b["pcnt"][has] == 3)
        assert np.all(b["pval"].reshape(-1, 3)[has] == 1.0 / 3.0)
        expect = np.sort(np.stack([b["labels"][has], tri[has, 0], tri[has, 1]], 1), axis=1)
        assert np.array_equal(b["pcol"].reshape(-1, 3)[has], expect)
        # fallback rows are the default's
        assert np.array_equal(a["pval"].reshape(-1, 3)[~has], b["pval"].reshape(-1, 3)[~has])


@pytest.mark.parametrize("name", ["torus96", "pc4k", "ico4"])
def test_inverse_distance_weights(name):
    p, h0 = hier(name)
    _, h2 = hier(name, weighting=2)
    for l in range(h0.num_levels - 1):
        a, b = h0.level(l), h2.level(l)
        for k in GEOMETRIC + ["tri"]:
            assert np.array_equal(a[k], b[k]), (l, k)
        Xf, Xc = b["X"].reshape(-1, 3), h2.level(l + 1)["X"].reshape(-1, 3)
        tri = b["tri"].reshape(-1, 2)
        has = tri[:, 0] >= 0
        cols, vals = b["pcol"].reshape(-1, 3), b["pval"].reshape(-1, 3)
        for i in np.nonzero(has)[0][:400]:
            verts = [b["labels"][i], tri[i, 0], tri[i, 1]]
            d = np.linalg.norm(Xc[verts] - Xf[i], axis=1)
            w = {int(c): v for c, v in zip(cols[i][:b["pcnt"][i]], vals[i][:b["pcnt"][i]])}
            wt = np.array([w.get(int(v), 0.0) for v in verts])
            assert abs(wt.sum() - 1.0) <= 4e-16
            if d.min() > 0:
                assert np.all(wt > 0)
                prod = wt * d                               # w proportional to 1/d
                assert np.ptp(prod) <= 1e-14 * prod.max(), (i, wt, d)
            else:
                assert wt[np.argmin(d)] == 1.0


@pytest.mark.parametrize("name", ["pc4k", "pc20k", "flat", "ico4"])
def test_fallback_on_vertex_projections(name):
    """Exactly the rows whose best projection is a triangle vertex (a one-entry
    row with a triangle) become fallback rows; every other row is unchanged."""
    p, h0 = hier(name)
    _, h3 = hier(name, fallback_on_vertex=1)
    moved = 0
    for l in range(h0.num_levels - 1):
        a, b = h0.level(l), h3.level(l)
        for k in GEOMETRIC:
            assert np.array_equal(a[k], b[k]), (l, k)
        ta, tb = a["tri"].reshape(-1, 2), b["tri"].reshape(-1, 2)
        vert = (ta[:, 0] >= 0) & (a["pcnt"] == 1)
        assert np.array_equal(tb[:, 0] < 0, (ta[:, 0] < 0) | vert)
        same = ~vert
        assert np.array_equal(a["pcol"].reshape(-1, 3)[same], b["pcol"].reshape(-1, 3)[same])
        assert np.array_equal(a["pval"].reshape(-1, 3)[same], b["pval"].reshape(-1, 3)[same])
        # the moved rows carry the inverse-distance fallback over {c} U N(c)
        Xf, Xc = b["X"].reshape(-1, 3), h3.level(l + 1)["X"].reshape(-1, 3)
        erp, ecol = h3.level(l + 1)["erp"], h3.level(l + 1)["ecol"]
        for i in np.nonzero(vert)[0]:
            c = b["labels"][i]
            nb = np.concatenate([[c], ecol[erp[c]:erp[c + 1]]])
            d2 = ((Xc[nb] - Xf[i]) ** 2).sum(1)
            order = np.lexsort((nb, d2))[:3]
            cnt = b["pcnt"][i]
            if d2[order[0]] == 0.0:
                assert cnt == 1 and b["pcol"].reshape(-1, 3)[i, 0] == nb[order[0]]
            else:
                assert set(b["pcol"].reshape(-1, 3)[i, :cnt]) == set(nb[order[:cnt]])
            moved += 1
        assert h3.sizes(l)["fallback"] == h0.sizes(l)["fallback"] + int(vert.sum())
    assert moved > 0


def test_variant_options_rejected_when_out_of_range():
    p = problem("ico3")
    for kw in (dict(weighting=3), dict(weighting=-1), dict(fallback_on_vertex=2)):
        with pytest.raises(oracle.OracleError):
            oracle.Hierarchy.from_problem(p, oracle.default_options(**kw))


def test_poisson_system():
    """(L + eta M) x = M y with eta = 1e-6: same pattern and geometry as the smoothing
    system, L's off-diagonal entries, a nearly singular SPD matrix; the solve converges
    to the direct solution."""
    ps = synth.config_poisson(48, 40)
    sm = synth.small_torus(48, 40)
    assert np.array_equal(ps.indptr, sm.indptr) and np.array_equal(ps.indices, sm.indices)
    rows = np.repeat(np.arange(ps.n), np.diff(ps.indptr))
    off = rows != ps.indices
    assert np.allclose(ps.data[off], (sm.data[off]) / 1e-3, rtol=1e-12)   # smoothing off-diagonals are alpha L
    assert abs(ps.matrix() @ np.ones(ps.n)).max() < 1e-4                   # L 1 = 0, eta M tiny
    h = oracle.Hierarchy.from_problem(ps, oracle.default_options(min_coarse_points=200))
    x, it, hist, st = h.solve(ps.rhs, tol=1e-8, max_iters=300)     # residual floor near 1e-10 (cond ~ 1/eta)
    assert st == 0
    import scipy.sparse.linalg as spla
    xs = spla.spsolve(ps.matrix().tocsc(), ps.rhs)
    assert np.linalg.norm(x - xs) <= 1e-4 * np.linalg.norm(xs)
