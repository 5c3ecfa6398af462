"""GPU parity of the CG preconditioner (symmetric V-cycle, double and float)
and of preconditioned CG against the CPU oracle, through the C ABI.

Tolerances:
- the cycle (double and float): the GPU performs the oracle's operations in
  its order on every level, the coarsest solve included (the product with the
  inverse whose columns are the oracle's substitutions), so z = B r is
  compared bit for bit, entry by entry;
- CG: the dot products are summed in a different order (tree vs. sequential),
  which perturbs the iterates at the rounding level of the previous residual:
  each iteration adds a difference of about u |r_{k-1}| (u the unit roundoff
  of the cycle; in the float cycle one input that lands on the other side of
  a rounding boundary changes an output by one float ulp), which shows up in
  r_k, smaller by the convergence factor, and CG carries the differences of
  earlier iterations forward instead of damping them.  So the residual
  histories must agree to 1e-6 |r_k| + 64 (k+1) u |r_{k-1}| (k from 0), the
  iteration counts must be equal (one more or less only when the last
  residual is within that bound of the tolerance),
  the solutions within 1e-6 relative, and every returned solution must meet
  the tolerance by its true residual.
"""
import sys

import numpy as np
import pytest

import oracle
from tests.conftest import problem
from tests.test_gpu_parity import assert_same_bits

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PREC = {"f64": 0, "f32": 1}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def both(prob, **opt):
    import paper_2307_04886_amd as g
    from paper_2307_04886_amd.binding import from_problem
    g.library()
    orc = oracle.Hierarchy.from_problem(prob, oracle.default_options(**opt))
    gpu, _ = from_problem(prob, g.default_options(**opt))
    return orc, gpu


SMALL = [("ico3", 100), ("ico4", 100), ("ico5", 1000), ("torus48", 100), ("torus96", 200), ("flat", 100),
         ("pc4k", 200), ("pc20k", 500), ("hubs_big", 1000), ("torus256", 1000), ("pc100k", 1000)]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,minc", SMALL)
def test_preconditioner_parity(name, minc, precision):
    _say(f"[gpu] preconditioner {precision} {name}")
    prob = problem(name)
    orc, gpu = both(prob, min_coarse_points=minc)
    r = np.random.default_rng(11).uniform(-1, 1, prob.n)
    zo = orc.precondition(r, PREC[precision])
    zg = gpu.precondition(torch.from_numpy(r).cuda(), precision=precision).cpu().numpy()
    assert_same_bits(zo, zg, f"{name} {precision} preconditioner")
    if precision == "f32":
        assert np.array_equal(zg, zg.astype(np.float32).astype(np.float64))


def test_preconditioner_single_level():
    _say("[gpu] preconditioner on a single level (direct solve)")
    prob = problem("ico3")
    orc, gpu = both(prob, min_coarse_points=prob.n)
    assert gpu.num_levels == 1
    r = np.random.default_rng(12).uniform(-1, 1, prob.n)
    for precision in ("f64", "f32"):
        zo = orc.precondition(r, PREC[precision])
        zg = gpu.precondition(torch.from_numpy(r).cuda(), precision=precision).cpu().numpy()
        assert_same_bits(zo, zg, f"single level {precision}")


def compare_pcg(orc, gpu, prob, precision, tol=1e-8, max_iters=100, check_x=True):
    x_o, it_o, hist_o, st_o, fin_o = orc.solve_pcg(prob.rhs, tol=tol, max_iters=max_iters,
                                                    precision=PREC[precision])
    b = torch.from_numpy(prob.rhs).cuda()
    x_g, info, st_g, hist_g = gpu.solve_pcg(b, tol=tol, max_iters=max_iters, precision=precision, history=True)
    x_g = x_g.cpu().numpy()
    u = 2.0 ** -53 if precision == "f64" else 2.0 ** -24
    prev = np.concatenate([[1.0], hist_o[:-1]])
    bound = 1e-6 * hist_o + 64 * u * np.arange(1, len(hist_o) + 1) * prev
    near = abs(hist_o[-1] - tol) <= bound[-1] or (it_o > 1 and abs(hist_o[-2] - tol) <= bound[-2])
    assert info.iterations == it_o or (near and abs(info.iterations - it_o) == 1), (info.iterations, it_o)
    k = min(it_o, info.iterations)
    assert np.all(np.abs(hist_g[:k] - hist_o[:k]) <= bound[:k]), (hist_g[:k], hist_o[:k])
    assert st_g == st_o
    A = prob.matrix()
    res = np.linalg.norm(prob.rhs - A @ x_g) / np.linalg.norm(prob.rhs)
    assert abs(res - info.rel_residual) <= 1e-6 * res
    if st_g == 0:
        assert res <= tol * (1 + 1e-9)
    err = np.linalg.norm(x_g - x_o) / np.linalg.norm(x_o)
    if check_x:
        assert err <= 1e-6, err
    return info, err, res


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("name,minc", SMALL)
def test_pcg_parity_small(name, minc, precision):
    _say(f"[gpu] PCG {precision} {name}")
    prob = problem(name)
    orc, gpu = both(prob, min_coarse_points=minc)
    compare_pcg(orc, gpu, prob, precision)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_pcg_parity_torus_full(precision):
    _say(f"[gpu] PCG {precision} torus 1024x1024")
    prob = problem("torus1024")
    orc, gpu = both(prob)
    info, err, res = compare_pcg(orc, gpu, prob, precision)
    _say(f"[gpu] torus1024 PCG {precision}: {info.iterations} iterations, true rel. residual {res:.3e}, "
         f"|x_gpu - x_oracle| / |x_oracle| = {err:.2e}")


@pytest.mark.timeout(900)
def test_mixed_form_bumpy_sphere_full():
    """2M-point point cloud, mixed form: float V-cycles preconditioning double CG to 1e-10;
    the error against the double-precision oracle solution is stated."""
    _say("[gpu] mixed form, bumpy sphere 2M points, CG to 1e-10")
    prob = problem("bumpy2m")
    orc, gpu = both(prob)
    x_o, it_o, hist_o, st_o, fin_o = orc.solve_pcg(prob.rhs, tol=1e-10, max_iters=200, precision=0)
    assert st_o == 0
    b = torch.from_numpy(prob.rhs).cuda()
    x_g, info, st = gpu.solve_pcg(b, tol=1e-10, max_iters=200, precision="f32")
    assert st == 0
    x_g = x_g.cpu().numpy()
    A = prob.matrix()
    res = np.linalg.norm(prob.rhs - A @ x_g) / np.linalg.norm(prob.rhs)
    assert res <= 1e-10 * (1 + 1e-9)
    err = np.linalg.norm(x_g - x_o) / np.linalg.norm(x_o)
    assert err <= 1e-8, err
    _say(f"[gpu] bumpy2m mixed: {info.iterations} CG iterations (oracle double: {it_o}), true rel. residual "
         f"{res:.3e}, |x_mixed - x_oracle_f64| / |x_oracle_f64| = {err:.2e}")


def test_pcg_edge_cases_and_errors():
    _say("[gpu] PCG edge cases")
    import paper_2307_04886_amd as g
    prob = problem("ico4")
    orc, gpu = both(prob, min_coarse_points=100)
    n = prob.n
    for precision in ("f64", "f32"):
        x, info, st = gpu.solve_pcg(torch.zeros(n, dtype=torch.float64).cuda(), precision=precision)
        assert st == 0 and info.iterations == 0 and not x.abs().sum().item()
        x, info, st = gpu.solve_pcg(torch.from_numpy(prob.rhs).cuda(), tol=1e-15, max_iters=1,
                                    precision=precision)
        assert st == 1 and info.iterations == 1
        xs = torch.from_numpy(np.linalg.solve(prob.matrix().toarray(), prob.rhs)).cuda()
        x, info, st = gpu.solve_pcg(torch.from_numpy(prob.rhs).cuda(), x=xs.clone(), precision=precision)
        assert st == 0 and info.iterations == 0
    bad = torch.from_numpy(prob.rhs).cuda()
    bad[5] = float("nan")
    with pytest.raises(g.GMGError) as e:
        gpu.solve_pcg(bad)
    assert e.value.status == -1
    with pytest.raises(g.GMGError) as e:
        gpu.precondition(bad)
    assert e.value.status == -1
    # the plain solve still works on a handle that ran CG, and vice versa
    x1, i1, s1 = gpu.solve(torch.from_numpy(prob.rhs).cuda())
    x2, i2, s2 = gpu.solve_pcg(torch.from_numpy(prob.rhs).cuda(), precision="f32")
    x3, i3, s3 = gpu.solve(torch.from_numpy(prob.rhs).cuda())
    assert s1 == s2 == s3 == 0 and torch.equal(x1, x3)


def test_pcg_deterministic():
    _say("[gpu] PCG determinism")
    prob = problem("torus96")
    orc, gpu = both(prob, min_coarse_points=200)
    b = torch.from_numpy(prob.rhs).cuda()
    for precision in ("f64", "f32"):
        xa = gpu.solve_pcg(b, precision=precision)[0]
        xb = gpu.solve_pcg(b, precision=precision)[0]
        assert torch.equal(xa, xb)
