"""Pins of the oracle's CG preconditioner and preconditioned CG (double and
float V-cycles inside double-precision CG).

- The symmetric V-cycle is restated as dense linear algebra: Gauss-Seidel in
  matrix-splitting form, colours ascending before the coarse correction and
  descending after it, exact solve on the coarsest level.
- B must be a symmetric positive definite operator (that is what CG needs and
  what the descending post-smoothing buys).
- The float cycle must stay within float rounding of the double cycle.
- CG must obey the textbook bound ||e_k||_A <= 2 q^k ||e_0||_A with
  q = (sqrt(k) - 1) / (sqrt(k) + 1), k = cond(B A), computed densely; its
  A-norm error must decrease monotonically; with one level (B = A^-1) it must
  finish in one iteration.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from tests.conftest import problem
from tests.test_oracle_solve import dense_hierarchy


def sweep_split(A, colors, descending):
    """D plus the entries of the unknowns visited before row i in one sweep."""
    earlier = colors[None, :] > colors[:, None] if descending else colors[None, :] < colors[:, None]
    return np.diag(np.diag(A)) + np.where(earlier, A, 0.0)


def dense_sym_vcycle(levels, l, b, nu_pre=2, nu_post=2):
    L = levels[l]
    A = L["A"]
    if l == len(levels) - 1:
        return np.linalg.solve(A, b)
    x = np.zeros_like(b)
    Mf = sweep_split(A, L["colors"], False)
    Mb = sweep_split(A, L["colors"], True)
    for _ in range(nu_pre):
        x = x + np.linalg.solve(Mf, b - A @ x)
    P = L["P"]
    x = x + P @ dense_sym_vcycle(levels, l + 1, P.T @ (b - A @ x), nu_pre, nu_post)
    for _ in range(nu_post):
        x = x + np.linalg.solve(Mb, b - A @ x)
    return x


CASES = [("torus48", 300), ("torus48", 100), ("ico4", 100), ("flat", 200), ("pc4k", 200)]


@pytest.mark.parametrize("name,minc", CASES)
def test_symmetric_vcycle_matches_dense_restatement(name, minc):
    p = problem(name)
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=minc))
    assert h.num_levels >= 2
    levels = dense_hierarchy(h)
    r = np.random.default_rng(3).uniform(-1, 1, p.n)
    z = h.precondition(r, 0)
    ref = dense_sym_vcycle(levels, 0, r)
    assert np.linalg.norm(z - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("name,minc", CASES)
def test_preconditioner_is_symmetric_positive_definite(name, minc):
    p = problem(name)
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=minc))
    rng = np.random.default_rng(4)
    for _ in range(3):
        r1, r2 = rng.uniform(-1, 1, p.n), rng.uniform(-1, 1, p.n)
        z1, z2 = h.precondition(r1), h.precondition(r2)
        scale = np.linalg.norm(r1) * np.linalg.norm(z2)
        assert abs(r2 @ z1 - r1 @ z2) <= 1e-12 * scale
        assert r1 @ z1 > 0 and r2 @ z2 > 0


def test_forward_post_smoothing_would_not_be_symmetric():
    """Sanity of the pin above: the plain V-cycle (colours ascending in both
    smoothing phases), applied from zero, is measurably non-symmetric."""
    p = problem("torus48")
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=100))
    rng = np.random.default_rng(5)
    r1, r2 = rng.uniform(-1, 1, p.n), rng.uniform(-1, 1, p.n)
    z1 = h.solve(r1, max_iters=1, tol=0.0)[0]
    z2 = h.solve(r2, max_iters=1, tol=0.0)[0]
    assert abs(r2 @ z1 - r1 @ z2) > 1e-6 * np.linalg.norm(r1) * np.linalg.norm(z2)


@pytest.mark.parametrize("name,minc", CASES + [("pc20k", 500), ("ico5", 1000)])
def test_float_cycle_within_float_rounding_of_double_cycle(name, minc):
    p = problem(name)
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=minc))
    r = np.random.default_rng(6).uniform(-1, 1, p.n)
    z64 = h.precondition(r, 0)
    z32 = h.precondition(r, 1)
    assert np.array_equal(z32, z32.astype(np.float32).astype(np.float64))   # float results
    rel = np.linalg.norm(z32 - z64) / np.linalg.norm(z64)
    assert 1e-9 < rel <= 2e-6, rel


def test_float_cycle_on_one_level_rounds_the_direct_solve():
    """One level: B r = A^-1 r, with r rounded to float and the solution rounded to float."""
    p = problem("ico3")
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=p.n))
    assert h.num_levels == 1
    r = np.random.default_rng(7).uniform(-1, 1, p.n)
    z = h.precondition(r, 1)
    exact = np.linalg.solve(p.matrix().toarray(), r.astype(np.float32).astype(np.float64))
    ulp = np.spacing(np.abs(exact).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(z - exact) <= ulp)
    assert np.array_equal(h.precondition(r, 0), h.solve(r, max_iters=1, tol=0.0)[0])


def dense_preconditioner(h, n):
    return np.stack([h.precondition(e) for e in np.eye(n)], axis=1)


@pytest.mark.parametrize("name,minc", [("torus48", 100), ("ico4", 100), ("pc4k", 200)])
def test_pcg_obeys_the_condition_number_bound(name, minc):
    p = problem(name)
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=minc))
    A = p.matrix().toarray()
    B = dense_preconditioner(h, p.n)
    B = 0.5 * (B + B.T)
    Bh = np.linalg.cholesky(B)
    ev = np.linalg.eigvalsh(Bh.T @ A @ Bh)             # spectrum of B A
    kappa = ev[-1] / ev[0]
    q = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
    xs = np.linalg.solve(A, p.rhs)
    anorm = lambda e: np.sqrt(e @ A @ e)
    e0 = anorm(xs)
    prev = e0
    for k in range(1, 12):
        x, it, hist, st, fin = h.solve_pcg(p.rhs, tol=0.0, max_iters=k)
        ek = anorm(x - xs)
        if ek <= 1e-13 * e0:
            break
        assert ek <= 2 * q ** k * e0 * (1 + 1e-8), (k, ek / e0, 2 * q ** k)
        assert ek < prev
        prev = ek


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", ["ico4", "torus96", "flat", "pc4k", "pc20k"])
def test_pcg_solution_matches_direct_solve(name, precision):
    p = problem(name)
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=200))
    x, it, hist, st, fin = h.solve_pcg(p.rhs, tol=1e-10, max_iters=100, precision=precision)
    assert st == 0
    A = p.matrix()
    xs = spla.spsolve(A.tocsc(), p.rhs)
    res = np.linalg.norm(p.rhs - A @ x) / np.linalg.norm(p.rhs)
    assert res <= 1e-10 and abs(res - fin) <= 1e-6 * res
    cond = np.linalg.cond(A.toarray()) if p.n <= 5000 else 1e4
    assert np.linalg.norm(x - xs) <= 10 * cond * 1e-10 * np.linalg.norm(xs)
    x_plain, it_plain, _, _ = h.solve(p.rhs, tol=1e-10, max_iters=200)
    assert it <= it_plain + 1


def test_pcg_one_level_is_one_iteration():
    p = problem("ico3")
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=p.n))
    x, it, hist, st, fin = h.solve_pcg(p.rhs, tol=1e-12)
    assert st == 0 and it == 1 and fin <= 1e-14


def test_pcg_status_and_edge_cases():
    p = problem("ico4")
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=100))
    x, it, hist, st, fin = h.solve_pcg(np.zeros(p.n))
    assert st == 0 and it == 0 and not x.any()
    x, it, hist, st, fin = h.solve_pcg(p.rhs, tol=1e-14, max_iters=1)
    assert st == 1 and it == 1 and fin > 1e-14
    xs = np.linalg.solve(p.matrix().toarray(), p.rhs)
    x, it, hist, st, fin = h.solve_pcg(p.rhs, x0=xs, tol=1e-8)
    assert st == 0 and it == 0
    with pytest.raises(oracle.OracleError):
        h.solve_pcg(p.rhs, precision=2)
    bad = p.rhs.copy()
    bad[0] = np.nan
    with pytest.raises(oracle.OracleError):
        h.solve_pcg(bad)


@pytest.mark.parametrize("precision", [0, 1])
def test_pcg_matches_flexible_cg_restatement(precision):
    """With unequal smoothing counts B is not symmetric, and only the flexible
    form keeps CG's local A-orthogonality.  Restated here in Notay's form: the
    new direction is z A-orthogonalised against the previous one, and the step
    is (p.r) / (p.A p).  It must give the oracle's iterates."""
    p = problem("torus48")
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=100, nu_pre=1, nu_post=3))
    A = p.matrix()
    b = p.rhs
    x = np.zeros(p.n)
    r = b.copy()
    d = None
    for k in range(1, 9):
        z = h.precondition(r, precision)
        if d is None:
            d = z
        else:
            Ad_prev = A @ d
            d = z - (z @ Ad_prev) / (d @ Ad_prev) * d
        Ad = A @ d
        x = x + (d @ r) / (d @ Ad) * d
        r = r - (d @ r) / (d @ Ad) * Ad
        xo, it, hist, st, fin = h.solve_pcg(b, tol=0.0, max_iters=k, precision=precision)
        assert np.linalg.norm(xo - x) <= 1e-9 * np.linalg.norm(x), k
