"""GPU: new matrix values on a kept hierarchy (gmg_update_matrix), the
pattern product (gmg_pattern_outer) and the differentiable solve
(torch.autograd.Function) built on them.

- update: a hierarchy built for A_1 and updated to A_2 must equal, bit for bit,
  a hierarchy built for A_2 (the geometric parts do not depend on A; the
  Galerkin operators and the coarsest factorisation are recomputed by the
  same kernels), and must match the oracle built for A_2;
- gradients: against the dense formula (oracle.adjoint_gradients) on the
  2,562-vertex icosphere, and against central finite differences (h = 1e-6)
  on 32 stored entries of A and 8 entries of b of the 499,849-vertex torus.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.conftest import problem
from tests.test_gpu_parity import BITWISE, compare_hierarchies, compare_solves

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _g():
    import paper_2307_04886_amd as g
    g.library()
    return g


def upload(prob, data=None):
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return dict(points=dev(prob.points), edges=dev(prob.edges), rowptr=dev(prob.indptr),
                col=dev(prob.indices), val=dev(prob.data if data is None else data))


def build(t, **opt):
    g = _g()
    from paper_2307_04886_amd.binding import build_hierarchy
    return build_hierarchy(t["points"], t["edges"], t["rowptr"], t["col"], t["val"], g.default_options(**opt))


def second_system(name):
    """The same surface with a different smoothing weight: same pattern, new values."""
    if name == "torus96":
        return synth.config_torus(96, 80, alpha=1e-2)
    if name == "ico5":
        return synth.config_icosphere(5, alpha=3e-3)
    return synth.small_pointcloud(4000)


@pytest.mark.parametrize("name,minc", [("torus96", 200), ("ico5", 1000), ("pc4k", 200)])
def test_update_matrix_equals_fresh_build(name, minc):
    _say(f"[gpu] update_matrix {name}")
    p1 = problem(name)
    p2 = second_system(name)
    if name == "pc4k":
        p2.data = p2.data * 1.7 + 0.0                    # same pattern, scaled values
        p2.rhs = p2.rhs.copy()
    assert np.array_equal(p1.indices, p2.indices)
    t1 = upload(p1)
    h = build(t1, min_coarse_points=minc)
    h.update_matrix(torch.from_numpy(p2.data).cuda())
    fresh = build(upload(p2), min_coarse_points=minc)
    for l in range(fresh.num_levels):
        for what in BITWISE + ["a_val"]:
            a, b = fresh.export(l, what), h.export(l, what)
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (l, what)
    assert np.array_equal(fresh.export(fresh.num_levels - 1, "chol"), h.export(h.num_levels - 1, "chol"))
    orc = oracle.Hierarchy(p2.points, p2.edges, p2.indptr, p2.indices, p2.data,
                           oracle.default_options(min_coarse_points=minc))
    compare_hierarchies(orc, h, name + " updated")
    compare_solves(orc, h, p2)
    b = torch.from_numpy(p2.rhs).cuda()
    for precision in ("f64", "f32"):
        xa = h.solve_pcg(b, precision=precision)[0]
        xb = fresh.solve_pcg(b, precision=precision)[0]
        assert torch.equal(xa, xb), precision


def test_update_matrix_refreshes_float_copies():
    _say("[gpu] update_matrix after a float CG solve")
    p1, p2 = problem("torus96"), second_system("torus96")
    h = build(upload(p1), min_coarse_points=200)
    b = torch.from_numpy(p2.rhs).cuda()
    h.solve_pcg(b, precision="f32")                       # float copies of A_1 exist now
    h.update_matrix(torch.from_numpy(p2.data).cuda())
    fresh = build(upload(p2), min_coarse_points=200)
    assert torch.equal(h.solve_pcg(b, precision="f32")[0], fresh.solve_pcg(b, precision="f32")[0])
    assert torch.equal(h.solve(b)[0], fresh.solve(b)[0])


def test_update_matrix_errors():
    _say("[gpu] update_matrix errors")
    g = _g()
    prob = problem("ico4")
    h = build(upload(prob), min_coarse_points=100)
    bad = prob.data.copy()
    bad[3] = np.nan
    with pytest.raises(g.GMGError) as e:
        h.update_matrix(torch.from_numpy(bad).cuda())
    assert e.value.status == -1
    neg = prob.data.copy()
    d = prob.indptr[7] + np.nonzero(prob.indices[prob.indptr[7]:prob.indptr[8]] == 7)[0][0]
    neg[d] = -1.0
    with pytest.raises(g.GMGError) as e:
        h.update_matrix(torch.from_numpy(neg).cuda())
    assert e.value.status == -4
    h.update_matrix(torch.from_numpy(prob.data).cuda())  # a valid update restores the handle
    fresh = build(upload(prob), min_coarse_points=100)
    b = torch.from_numpy(prob.rhs).cuda()
    assert torch.equal(h.solve(b)[0], fresh.solve(b)[0])


def test_pattern_outer():
    _say("[gpu] pattern product")
    _g()
    from paper_2307_04886_amd.binding import pattern_outer
    prob = problem("pc4k")
    rng = np.random.default_rng(5)
    u, v = rng.standard_normal(prob.n), rng.standard_normal(prob.n)
    t = upload(prob)
    out = pattern_outer(t["rowptr"], t["col"], torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda(), -2.5)
    rows = np.repeat(np.arange(prob.n), np.diff(prob.indptr))
    ref = (-2.5 * u[rows]) * v[prob.indices]
    assert np.array_equal(out.cpu().numpy(), ref)


@pytest.mark.parametrize("method", ["vcycle", "pcg_f64", "pcg_f32"])
def test_autograd_dense_reference(method):
    """2,562-vertex icosphere: gradients of ||x - x*||^2 against the dense formula."""
    _say(f"[gpu] autograd dense reference ({method})")
    _g()
    from paper_2307_04886_amd import autograd
    prob = problem("ico4")
    assert prob.n == 2562
    target = synth.uniform(0, "target", prob.n, -1.0, 1.0)
    t = upload(prob)
    h = build(t, min_coarse_points=100)
    A = t["val"].clone().requires_grad_(True)
    b = torch.from_numpy(prob.rhs).cuda().requires_grad_(True)
    x = autograd.solve(h, A, b, tol=1e-13, max_iters=400, method=method)
    loss = ((x - torch.from_numpy(target).cuda()) ** 2).sum()
    loss.backward()
    xs = np.linalg.solve(prob.matrix().toarray(), prob.rhs)
    gb, gA = oracle.adjoint_gradients(prob.indptr, prob.indices, prob.data, xs, 2.0 * (xs - target))
    assert np.allclose(x.detach().cpu().numpy(), xs, rtol=0, atol=1e-10 * np.abs(xs).max())
    assert np.abs(b.grad.cpu().numpy() - gb).max() <= 1e-8 * np.abs(gb).max()
    assert np.abs(A.grad.cpu().numpy() - gA).max() <= 1e-8 * np.abs(gA).max()


def test_autograd_finite_differences_torus707():
    """499,849-vertex torus: central differences (h = 1e-6) of the loss on 32 stored
    entries of A and 8 entries of b.  Every solve runs the same fixed number of
    V-cycles from zero, so the two sides of a difference differ smoothly in h."""
    _say("[gpu] autograd finite differences, torus 707 x 707")
    _g()
    from paper_2307_04886_amd import autograd
    prob, target, a_idx, b_idx = synth.config_adjoint()
    t = upload(prob)
    h = build(t)
    tgt = torch.from_numpy(target).cuda()
    A = t["val"].clone().requires_grad_(True)
    b = torch.from_numpy(prob.rhs).cuda().requires_grad_(True)
    x = autograd.solve(h, A, b, tol=1e-12, max_iters=400, method="pcg_f64")
    ((x - tgt) ** 2).sum().backward()
    gA, gb = A.grad.cpu().numpy(), b.grad.cpu().numpy()
    cycles = 80

    def run(vals, rhs):
        h.update_matrix(vals)
        xx = torch.zeros_like(rhs)
        h.solve(rhs, xx, tol=0.0, max_iters=cycles)
        return xx

    step = 1e-6
    va = t["val"]
    bb = torch.from_numpy(prob.rhs).cuda()
    worst = 0.0
    for e in a_idx:
        vp, vm = va.clone(), va.clone()
        vp[e] += step
        vm[e] -= step
        xp, xm = run(vp, bb), run(vm, bb)
        fd = ((xp - xm) * (xp + xm - 2 * tgt)).sum().item() / (2 * step)
        worst = max(worst, abs(fd - gA[e]) / np.abs(gA[a_idx]).max())
    h.update_matrix(va)
    for i in b_idx:
        bp, bm = bb.clone(), bb.clone()
        bp[i] += step
        bm[i] -= step
        xp, xm = run(va, bp), run(va, bm)
        fd = ((xp - xm) * (xp + xm - 2 * tgt)).sum().item() / (2 * step)
        worst = max(worst, abs(fd - gb[i]) / np.abs(gb[b_idx]).max())
    _say(f"[gpu] torus707 finite differences: worst relative deviation {worst:.2e}")
    assert worst <= 1e-5
