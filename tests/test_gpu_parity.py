"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Discrete outputs (samples, labels, coarse edges, triangle choices, P pattern,
A patterns, colours) must match bit for bit; so must every value produced
by a fixed operation sequence: positions, edge lengths, e_hat, Voronoi
distances, P weights, the Galerkin values of every A_l (each entry summed in
the oracle's pair order), the coarsest Cholesky factor and its inverse (the
substitutions of the oracle, entry by entry in its order).  The V-cycle then
performs the oracle's operations in its order on every level, so every
iterate x_k is bit-identical; only the residual norm of the convergence test
is summed in another order (a tree of partial sums instead of a sequential
sum).  Each of the two sums of n squares is within (n - 1) u of the exact sum
(u = 2^-53), so the two norms agree to about (n + 2) u relative; the
histories are compared to max(1e-12, (n + 2) u) and the V-cycle counts must
be equal (one more or less only if a residual lies within that bound of the
tolerance).
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.conftest import problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gmg():
    import paper_2307_04886_amd as g
    g.library()
    return g


def both(prob, **opt):
    g = gmg()
    from paper_2307_04886_amd.binding import from_problem
    o_orc = oracle.default_options(**opt)
    o_gpu = g.default_options(**opt)
    orc = oracle.Hierarchy.from_problem(prob, o_orc)
    gpu, tensors = from_problem(prob, o_gpu)
    return orc, gpu


BITWISE = ["positions", "edge_rowptr", "edge_col", "edge_w", "scalars", "samples", "labels", "dist",
           "p_col", "p_val", "p_cnt", "tri", "a_rowptr", "a_col", "a_val", "colors", "block_colors"]
ORC_CODE = {"positions": oracle.POSITIONS, "edge_rowptr": oracle.EDGE_ROWPTR, "edge_col": oracle.EDGE_COL,
            "edge_w": oracle.EDGE_W, "scalars": oracle.SCALARS, "samples": oracle.SAMPLES,
            "labels": oracle.LABELS, "dist": oracle.DIST, "p_col": oracle.P_COL, "p_val": oracle.P_VAL,
            "p_cnt": oracle.P_CNT, "tri": oracle.TRI, "a_rowptr": oracle.A_ROWPTR, "a_col": oracle.A_COL,
            "a_val": oracle.A_VAL, "colors": oracle.COLORS, "chol": oracle.CHOL,
            "coarse_inverse": oracle.CINV, "block_colors": oracle.BLOCK_COLORS}


def same_bits(a, b):
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
    return a.shape == b.shape and np.array_equal(a.view(np.int64), b.view(np.int64))


def assert_same_bits(a, b, what):
    if not same_bits(a, b):
        a, b = np.asarray(a).reshape(-1), np.asarray(b).reshape(-1)
        bad = np.nonzero(a.view(np.int64) != b.view(np.int64))[0] if a.shape == b.shape else []
        raise AssertionError(f"{what}: {len(bad)} of {a.size} differ, first {bad[:5]}, "
                             f"oracle {a[bad[:5]] if len(bad) else a.shape} gpu {b[bad[:5]] if len(bad) else b.shape}")


def compare_hierarchies(orc, gpu, name=""):
    assert gpu.num_levels == orc.num_levels, (gpu.num_levels, orc.num_levels)
    for l in range(orc.num_levels):
        so, sg = orc.sizes(l), gpu.sizes(l)
        assert so == sg, (name, l, so, sg)
        for what in BITWISE:
            a = orc.export(l, ORC_CODE[what]).reshape(-1)
            b = gpu.export(l, what).reshape(-1)
            assert a.shape == b.shape, (name, l, what, a.shape, b.shape)
            if a.dtype == np.float64:
                same = np.array_equal(a.view(np.int64), b.view(np.int64))
            else:
                same = np.array_equal(a, b)
            if not same:
                bad = np.nonzero(a != b)[0]
                raise AssertionError(f"{name} level {l} {what}: {bad.size} of {a.size} differ, "
                                     f"first {bad[:5]} oracle {a[bad[:5]]} gpu {b[bad[:5]]}")
    L = orc.num_levels - 1
    assert_same_bits(orc.chol(), gpu.export(L, "chol"), f"{name} Cholesky factor")
    assert_same_bits(orc.coarse_inverse(), gpu.export(L, "coarse_inverse"), f"{name} coarsest inverse")


def hist_rtol(n):
    """Residual norms of the same residual vector summed in two orders."""
    return max(1e-12, (n + 2) * 2.0 ** -53)


def oracle_solve(orc, rhs, tol, max_iters, chunk=None):
    """The oracle's plain solve; with `chunk`, run as consecutive solves of at
    most `chunk` V-cycles, each resumed from the previous iterate (the same
    iterates as one solve), printing progress between them."""
    if chunk is None:
        return orc.solve(rhs, tol=tol, max_iters=max_iters)
    x, hist, it = None, [], 0
    while it < max_iters:
        x, k, h, st = orc.solve(rhs, x0=x, tol=tol, max_iters=min(chunk, max_iters - it))
        hist.extend(h[:k])
        it += k
        _say(f"[gpu]   oracle: {it} V-cycles, rel. residual {hist[-1]:.3e}")
        if st == 0:
            return x, it, np.array(hist), 0
    return x, it, np.array(hist), 1


def compare_solves(orc, gpu, prob, tol=1e-8, max_iters=200, chunk=None):
    """Same V-cycle count, bit-identical solution, residual histories within
    hist_rtol(n); the returned solution meets the tolerance by its true residual."""
    x_o, it_o, hist_o, st_o = oracle_solve(orc, prob.rhs, tol, max_iters, chunk)
    b = torch.from_numpy(prob.rhs).cuda()
    x_g, info, st_g, hist_g = gpu.solve(b, tol=tol, max_iters=max_iters, history=True)
    torch.cuda.synchronize()
    x_g = x_g.cpu().numpy()
    bound = hist_rtol(prob.n) * hist_o
    near = abs(hist_o[-1] - tol) <= bound[-1] or (it_o > 1 and abs(hist_o[-2] - tol) <= bound[-2])
    assert info.iterations == it_o or (near and abs(info.iterations - it_o) == 1), (info.iterations, it_o)
    k = min(it_o, info.iterations)
    assert np.all(np.abs(hist_g[:k] - hist_o[:k]) <= bound[:k]), (hist_g[:k], hist_o[:k])
    if info.iterations == it_o:
        assert st_g == st_o
        assert_same_bits(x_o, x_g, "solution")
    else:                       # one more cycle on one side: compare the common iterate
        x_k, _, _, _ = orc.solve(prob.rhs, tol=0.0, max_iters=k)
        x_gk = gpu.solve(b, tol=0.0, max_iters=k)[0].cpu().numpy()
        assert_same_bits(x_k, x_gk, f"iterate {k}")
    A = prob.matrix()
    res = np.linalg.norm(prob.rhs - A @ x_g) / np.linalg.norm(prob.rhs)
    if st_g == 0:
        assert res <= tol * (1 + 1e-9)
    assert abs(res - info.rel_residual) <= 1e-9 * res
    err = np.linalg.norm(x_g - x_o) / np.linalg.norm(x_o)
    return info.iterations, err


SMALL = [("ico3", 100), ("ico4", 100), ("ico5", 1000), ("torus48", 100), ("torus96", 200), ("flat", 100),
         ("pc4k", 200), ("pc20k", 500), ("torus256", 1000), ("pc100k", 1000)]


@pytest.mark.parametrize("name,minc", SMALL)
def test_hierarchy_bitwise_small(name, minc):
    _say(f"[gpu] hierarchy parity {name} min_coarse={minc}")
    prob = problem(name)
    orc, gpu = both(prob, min_coarse_points=minc)
    compare_hierarchies(orc, gpu, name)


@pytest.mark.parametrize("name,minc", SMALL)
def test_solve_parity_small(name, minc):
    _say(f"[gpu] solve parity {name}")
    prob = problem(name)
    orc, gpu = both(prob, min_coarse_points=minc)
    compare_solves(orc, gpu, prob)


@pytest.mark.parametrize("opt", [dict(sample_order=1), dict(shift_coarse_points=0), dict(seed=12345),
                                 dict(coarsening_ratio=0.25), dict(nu_pre=1, nu_post=3), dict(block_min_rows=300),
                                 dict(block_min_rows=100, coarsening_ratio=0.25)])
def test_option_variants(opt):
    _say(f"[gpu] options {opt}")
    prob = problem("torus96")
    orc, gpu = both(prob, min_coarse_points=200, **opt)
    compare_hierarchies(orc, gpu, str(opt))
    compare_solves(orc, gpu, prob)


@pytest.mark.parametrize("name,opt", [("torus96", dict(weighting=1)), ("torus96", dict(weighting=2)),
                                      ("pc20k", dict(weighting=2)), ("pc20k", dict(fallback_on_vertex=1)),
                                      ("flat", dict(fallback_on_vertex=1, weighting=1))])
def test_prolongation_variants(name, opt):
    """The weighting-ablation variants and the fallback-trigger variant, bit for bit."""
    _say(f"[gpu] prolongation variant {name} {opt}")
    prob = problem(name)
    orc, gpu = both(prob, min_coarse_points=200, **opt)
    compare_hierarchies(orc, gpu, f"{name} {opt}")
    compare_solves(orc, gpu, prob, max_iters=300)


def test_poisson_problem():
    """The Poisson system of the comparisons, (L + 1e-6 M) x = M y."""
    _say("[gpu] Poisson system, torus 96 x 80")
    prob = synth.config_poisson(96, 80)
    orc, gpu = both(prob, min_coarse_points=200)
    compare_hierarchies(orc, gpu, "poisson")
    compare_solves(orc, gpu, prob, tol=1e-8, max_iters=300)


def test_config_icosphere_full():
    _say("[gpu] icosphere 5 subdivisions, full pipeline")
    prob = problem("ico5")
    orc, gpu = both(prob)
    compare_hierarchies(orc, gpu, "ico5")
    it, err = compare_solves(orc, gpu, prob)
    _say(f"[gpu] ico5 V-cycles {it} |x_gpu - x_orc| / |x_orc| = {err:.2e}")


def test_config_torus_full():
    _say("[gpu] torus 1024x1024, full pipeline (bench launch configuration)")
    prob = problem("torus1024")
    orc, gpu = both(prob)
    compare_hierarchies(orc, gpu, "torus1024")
    it, err = compare_solves(orc, gpu, prob, chunk=10)
    _say(f"[gpu] torus1024 V-cycles {it} |x_gpu - x_orc| / |x_orc| = {err:.2e}")


@pytest.mark.timeout(1100)
def test_config_bumpy_sphere_full():
    """2M-point bumpy sphere, kNN graph: the whole hierarchy bit for bit and
    the whole plain solve to 1e-8 against the oracle (V-cycle count, residual
    history, solution bits)."""
    _say("[gpu] bumpy sphere 2M points, kNN k=8, full pipeline")
    prob = problem("bumpy2m")
    orc, gpu = both(prob)
    compare_hierarchies(orc, gpu, "bumpy2m")
    _say("[gpu] bumpy2m hierarchy matches; full solve")
    it, err = compare_solves(orc, gpu, prob, chunk=10)
    _say(f"[gpu] bumpy2m V-cycles {it} |x_gpu - x_orc| / |x_orc| = {err:.2e}")


def test_golden_paths():
    """The hand-worked path cases (exact radius, equidistant seeds) through the C ABI."""
    import json
    import os
    _say("[gpu] golden path cases")
    g = gmg()
    from paper_2307_04886_amd.binding import build_hierarchy
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "path_ties.json")))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    for case in golden["cases"]:
        n = case["n"]
        X = np.zeros((n, 3))
        X[:, 0] = case.get("x", np.arange(n, dtype=np.float64))
        edges = np.array([[i, i + 1] for i in range(n - 1)], dtype=np.int32)
        rp, ci, va = [0], [], []
        for i in range(n):
            for j in (i - 1, i, i + 1):
                if 0 <= j < n:
                    ci.append(j)
                    va.append(2.5 if i == j else -1.0)
            rp.append(len(ci))
        o = g.default_options(min_coarse_points=1, max_levels=2, sample_order=1,
                              coarsening_ratio=case["phi"])
        h = build_hierarchy(dev(X), dev(edges), dev(np.array(rp, np.int32)), dev(np.array(ci, np.int32)),
                            dev(np.array(va)), o)
        assert h.export(0, "samples").tolist() == case["samples"]
        assert h.export(0, "labels").tolist() == case["labels"]
        assert h.export(0, "dist").tolist() == case["dist"]


def test_determinism():
    _say("[gpu] determinism")
    prob = problem("torus96")
    g = gmg()
    from paper_2307_04886_amd.binding import from_problem
    h1, _ = from_problem(prob, g.default_options(min_coarse_points=200))
    h2, _ = from_problem(prob, g.default_options(min_coarse_points=200))
    for l in range(h1.num_levels):
        for what in BITWISE + ["a_val"]:
            assert np.array_equal(h1.export(l, what), h2.export(l, what))
    b = torch.from_numpy(prob.rhs).cuda()
    x1 = h1.solve(b)[0].cpu().numpy()
    x2 = h1.solve(b)[0].cpu().numpy()
    assert np.array_equal(x1, x2)


@pytest.mark.parametrize("name,minc", [("hubs", 100), ("hubs_big", 1000)])
def test_hub_vertices(name, minc):
    """Hub points joined to 150 others each: rows longer than every fast path
    holds (SELL fill by slice, conflict and colouring lists, cell neighbours by
    lanes, candidate-triangle lists, the 64-slot Galerkin table, the tail's
    32-entry rounds), so the general forms run and must agree with the oracle.
    On the larger mesh the 5,920-row level with rows of up to 472 entries is
    swept by separate launches with 64 lanes per row."""
    _say(f"[gpu] hub vertices {name}")
    prob = problem(name)
    orc, gpu = both(prob, min_coarse_points=minc)
    compare_hierarchies(orc, gpu, name)
    compare_solves(orc, gpu, prob)


def test_edge_cases():
    _say("[gpu] edge cases")
    g = gmg()
    from paper_2307_04886_amd.binding import build_hierarchy
    prob = problem("ico3")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    # duplicate edges, reversed edges and self loops in the input are canonicalised
    e = np.concatenate([prob.edges, prob.edges[:, ::-1], np.stack([np.arange(5)] * 2, 1)]).astype(np.int32)
    o = dict(min_coarse_points=100)
    h = build_hierarchy(dev(prob.points), dev(e), dev(prob.indptr), dev(prob.indices), dev(prob.data),
                        g.default_options(**o))
    ho = oracle.Hierarchy(prob.points, e, prob.indptr, prob.indices, prob.data, oracle.default_options(**o))
    compare_hierarchies(ho, h, "messy edges")
    # no edges at all: every point is its own sample, the input level is solved directly
    n = prob.n
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    va = np.linspace(1.0, 2.0, n)
    h = build_hierarchy(dev(prob.points), dev(np.zeros((0, 2), np.int32)), dev(rp), dev(ci), dev(va),
                        g.default_options(**o))
    assert h.num_levels == 1
    b = torch.from_numpy(np.ones(n)).cuda()
    x, info, st = h.solve(b)
    assert st == 0 and info.iterations == 1
    assert np.allclose(x.cpu().numpy(), 1.0 / va, rtol=1e-14)
    # a single point
    h = build_hierarchy(dev(np.zeros((1, 3))), dev(np.zeros((0, 2), np.int32)), dev(np.array([0, 1], np.int32)),
                        dev(np.array([0], np.int32)), dev(np.array([4.0])), g.default_options())
    x, info, st = h.solve(torch.tensor([2.0], dtype=torch.float64).cuda())
    assert st == 0 and abs(x.item() - 0.5) < 1e-15
    # zero right-hand side
    from paper_2307_04886_amd.binding import from_problem
    hh, _ = from_problem(prob, g.default_options(**o))
    x, info, st = hh.solve(torch.zeros(n, dtype=torch.float64).cuda())
    assert st == 0 and info.iterations == 0 and not x.abs().sum().item()
    # iteration cap
    x, info, st = hh.solve(torch.from_numpy(prob.rhs).cuda(), max_iters=1, tol=1e-14)
    assert st == 1 and info.iterations == 1


def test_error_paths():
    _say("[gpu] error paths")
    g = gmg()
    from paper_2307_04886_amd.binding import build_hierarchy
    prob = problem("ico3")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    args = lambda **kw: [dev(kw.get(k, v)) for k, v in
                         [("points", prob.points), ("edges", prob.edges), ("rowptr", prob.indptr),
                          ("col", prob.indices), ("val", prob.data)]]
    pts = prob.points.copy()
    pts[7, 2] = np.nan
    with pytest.raises(g.GMGError) as e:
        build_hierarchy(*args(points=pts))
    assert e.value.status == -1
    bad = prob.edges.copy()
    bad[3, 1] = prob.n + 5
    with pytest.raises(g.GMGError) as e:
        build_hierarchy(*args(edges=bad))
    assert e.value.status == -1
    ci = prob.indices.copy()
    ci[prob.indptr[4]], ci[prob.indptr[4] + 1] = ci[prob.indptr[4] + 1], ci[prob.indptr[4]]
    with pytest.raises(g.GMGError) as e:
        build_hierarchy(*args(col=ci))
    assert e.value.status == -1
    va = prob.data.copy()
    row = 9
    va[prob.indptr[row]:prob.indptr[row + 1]][prob.indices[prob.indptr[row]:prob.indptr[row + 1]] == row] = -1.0
    with pytest.raises(g.GMGError) as e:
        build_hierarchy(*args(val=va))
    assert e.value.status == -4
    # indefinite matrix with a positive diagonal: the dense factorisation fails
    import scipy.sparse as sp
    M = prob.matrix()
    off = M - sp.diags(M.diagonal())
    Lp = off - sp.diags(np.asarray(off.sum(axis=1)).ravel())
    A = (Lp - 0.05 * Lp.diagonal().min() * sp.eye(prob.n)).tocsr()
    A.sort_indices()
    with pytest.raises(g.GMGError) as e:
        build_hierarchy(*args(rowptr=A.indptr.astype(np.int32), col=A.indices.astype(np.int32), val=A.data))
    assert e.value.status == -4
    h = build_hierarchy(*args())
    b = torch.from_numpy(prob.rhs).cuda()
    b[3] = float("inf")
    with pytest.raises(g.GMGError) as e:
        h.solve(b)
    assert e.value.status == -1


def test_autotuned_shapes_keep_the_bits():
    """The autotuner only changes how rows are spread over lanes and loads:
    solves on hierarchies with measured shapes and with the fixed rules give
    the same bits, and the chosen shapes are among the candidates."""
    _say("[gpu] autotuned row-kernel shapes")
    prob = problem("torus256")
    g = gmg()
    from paper_2307_04886_amd.binding import from_problem
    tuned, _ = from_problem(prob, g.default_options(min_coarse_points=1000, autotune=1))
    fixed, _ = from_problem(prob, g.default_options(min_coarse_points=1000, autotune=0))
    for l in range(tuned.num_levels):
        t = tuned.tuning(l)
        assert t["lanes_A"] in (0, 4, 8, 16, 32, 64) and t["lanes_PT"] in (0, 1, 4, 8, 16, 32, 64)
        assert t["chunk"] in (0, 4, 8, 16) and (t["uniform_width"] == 0 or (l == 0 and t["uniform_width"] >= 1))
        _say(f"[gpu]   level {l}: {t}")
    assert tuned.tuning(0)["chunk"] > 0 and tuned.tuning(1)["block_sweep"] == 1
    b = torch.from_numpy(prob.rhs).cuda()
    assert torch.equal(tuned.solve(b)[0], fixed.solve(b)[0])
    for precision in ("f64", "f32"):
        assert torch.equal(tuned.solve_pcg(b, precision=precision)[0], fixed.solve_pcg(b, precision=precision)[0])
