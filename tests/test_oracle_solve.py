"""Pins of the CPU oracle's solve phase (Alg. 1, Alg. 2) against independent checks.

The V-cycle is restated here as dense linear algebra over the exported
hierarchy (matrix-splitting form of Gauss-Seidel, explicit inverse on the
coarsest level), and the converged solution is compared with a sparse direct
solve.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from tests import brute
from tests.conftest import problem


def dense_hierarchy(h):
    levels = []
    for l in range(h.num_levels):
        lv = h.level(l)
        n = lv["n"]
        d = dict(A=brute.dense(lv["arp"], lv["acol"], lv["aval"], (n, n)), colors=sweep_key(lv))
        if l + 1 < h.num_levels:
            d["P"] = brute.ell_to_dense(lv["pcol"], lv["pval"], lv["pcnt"], h.sizes(l + 1)["n"])
        levels.append(d)
    return levels


def sweep_key(lv):
    """Sweep class of each row: its colour, preceded by its block colour on
    levels swept in block order."""
    c = lv["colors"]
    if len(lv["block_colors"]) == 0:
        return c
    return lv["block_colors"].astype(np.int64) * (int(c.max()) + 1) + c


def gs_split(A, colors, mode):
    """Lower part of the Gauss-Seidel splitting: D + (entries of earlier-visited unknowns)."""
    n = A.shape[0]
    if mode == 1:
        return np.tril(A)
    earlier = colors[None, :] < colors[:, None]
    return np.diag(np.diag(A)) + np.where(earlier, A, 0.0)


def dense_vcycle(levels, l, x, b, nu=2, mode=0):
    L = levels[l]
    A = L["A"]
    if l == len(levels) - 1:
        return np.linalg.solve(A, b)
    M = gs_split(A, L["colors"], mode)
    for _ in range(nu):
        x = x + np.linalg.solve(M, b - A @ x)
    P = L["P"]
    u = dense_vcycle(levels, l + 1, np.zeros(P.shape[1]), P.T @ (b - A @ x), nu, mode)
    x = x + P @ u
    for _ in range(nu):
        x = x + np.linalg.solve(M, b - A @ x)
    return x


CASES = [("torus48", 300, 4096), ("torus48", 100, 4096), ("ico4", 100, 4096), ("flat", 200, 4096),
         ("pc4k", 200, 4096), ("torus48", 100, 50), ("pc4k", 100, 100)]


@pytest.mark.parametrize("name,minc,bmin", CASES)
@pytest.mark.parametrize("mode", [0, 1])
def test_one_vcycle_matches_dense_restatement(name, minc, bmin, mode):
    """One V-cycle equals the matrix-splitting form of Gauss-Seidel in the sweep
    order (colours, or block colours then colours), with bmin lowered so that
    the small meshes have levels swept in block order."""
    p = problem(name)
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=minc, block_min_rows=bmin))
    if bmin < 4096 and mode == 0:
        assert any(h.sizes(l)["blocks"] for l in range(h.num_levels))
    assert h.num_levels >= 2
    levels = dense_hierarchy(h)
    rng = np.random.default_rng(1)
    x0 = rng.uniform(-1, 1, p.n)
    x1, it, hist, st = h.solve(p.rhs, x0=x0, max_iters=1, gs_mode=mode, tol=0.0)
    assert st == 1 and it == 1
    ref = dense_vcycle(levels, 0, x0, p.rhs, 2, mode)
    assert np.linalg.norm(x1 - ref) <= 1e-10 * np.linalg.norm(ref)
    res = np.linalg.norm(p.rhs - p.matrix() @ x1) / np.linalg.norm(p.rhs)
    assert abs(hist[0] - res) <= 1e-10 * res


@pytest.mark.parametrize("name", ["ico4", "torus96", "flat", "pc4k", "pc20k"])
def test_converged_solution_matches_direct_solve(name):
    p = problem(name)
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=200))
    x, it, hist, st = h.solve(p.rhs, tol=1e-8, max_iters=200)
    assert st == 0
    A = p.matrix().tocsc()
    xs = spla.spsolve(A, p.rhs)
    res = np.linalg.norm(p.rhs - p.matrix() @ x) / np.linalg.norm(p.rhs)
    assert res <= 1e-8 and abs(res - hist[-1]) <= 1e-10 * res
    assert hist[-2] > 1e-8 if it > 1 else True
    # error bound from the residual: |x - x*| <= |A^-1| |r|
    lam_min = spla.eigsh(A, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
    bound = np.linalg.norm(p.rhs - p.matrix() @ x) / lam_min
    assert np.linalg.norm(x - xs) <= 1.01 * bound + 1e-14 * np.linalg.norm(xs)


@pytest.mark.parametrize("mode", [0, 1])
def test_energy_error_decreases_every_cycle(mode):
    """Each V-cycle is an A-norm contraction for SPD A (GS smoothing + Galerkin correction)."""
    p = problem("torus96")
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=200))
    A = p.matrix()
    xs = spla.spsolve(A.tocsc(), p.rhs)
    errs = []
    for k in range(1, 9):
        x, it, hist, st = h.solve(p.rhs, max_iters=k, tol=0.0, gs_mode=mode)
        e = x - xs
        errs.append(np.sqrt(e @ (A @ e)))
    assert all(b < a for a, b in zip(errs, errs[1:]))


def test_asymptotic_rate_is_the_two_grid_spectral_radius():
    """The residual contraction per cycle approaches the spectral radius of the dense
    two-grid error operator S^2 (I - P A_c^-1 P^T A) S^2.  (First-fit colouring
    without recolouring passes: its slower contraction leaves enough cycles above
    the rounding floor for the asymptotic rate to show.)"""
    import synth
    p = synth.config_torus(64, 32)
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=300, color_passes=0))
    assert h.num_levels == 2
    lv = dense_hierarchy(h)
    A, P, colors = lv[0]["A"], lv[0]["P"], lv[0]["colors"]
    n = A.shape[0]
    S = np.eye(n) - np.linalg.solve(gs_split(A, colors, 0), A)
    S2 = S @ S
    C = np.eye(n) - P @ np.linalg.solve(lv[1]["A"], P.T @ A)
    rho = np.abs(np.linalg.eigvals(S2 @ C @ S2)).max()
    x, it, hist, st = h.solve(p.rhs, tol=1e-15, max_iters=50)
    ratios = (hist[1:] / hist[:-1])[hist[1:] > 1e-13]
    rate = np.exp(np.log(ratios[-3:]).mean())
    assert abs(rate - rho) <= 0.05 * rho, (rate, rho)


def test_single_level_is_a_direct_solve():
    p = problem("flat")           # 1440 points
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=2000))
    assert h.num_levels == 1
    x, it, hist, st = h.solve(p.rhs)
    assert st == 0 and it == 1 and hist[0] <= 1e-13


def test_status_codes():
    p = problem("torus48")
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=300))
    x, it, hist, st = h.solve(p.rhs, max_iters=1)
    assert st == 1 and it == 1
    x, it, hist, st = h.solve(np.zeros(p.n))
    assert st == 0 and it == 0 and not x.any()
    b = p.rhs.copy()
    b[3] = np.inf
    with pytest.raises(oracle.OracleError):
        h.solve(b)


def test_indefinite_matrix_is_reported():
    """A symmetric matrix with positive diagonal but a negative eigenvalue fails the factorisation."""
    p = problem("flat")
    M = p.matrix()
    off = M - sp.diags(M.diagonal())
    L = off - sp.diags(np.asarray(off.sum(axis=1)).ravel())
    A = (L - 0.05 * sp.diags(L.diagonal().min() * np.ones(p.n))).tocsr()
    A.sort_indices()
    assert A.diagonal().min() > 0
    with pytest.raises(oracle.OracleError) as e:
        oracle.Hierarchy(p.points, p.edges, A.indptr, A.indices, A.data,
                         oracle.default_options(min_coarse_points=2000))
    assert e.value.status == -4


@pytest.mark.parametrize("name,minc", [("torus48", 300), ("ico4", 100), ("pc4k", 200)])
def test_coarse_inverse_is_the_inverse(name, minc):
    """The coarsest direct solve (Alg. 2) is a product with A^-1, whose columns
    come from substitutions with the Cholesky factor.  Checked against LAPACK's
    inverse and triangular solves (other operation orders), A A^-1 = I, and
    symmetry, each within the rounding bound of a backward-stable solve."""
    import scipy.linalg as sla
    p = problem(name)
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=minc))
    L = h.num_levels - 1
    lv = h.level(L)
    n = lv["n"]
    A = brute.dense(lv["arp"], lv["acol"], lv["aval"], (n, n))
    inv = h.coarse_inverse().T                # column k = A^-1 e_k
    u = 2.0 ** -53
    kappa = np.linalg.cond(A)
    bound = 8 * n * kappa * u
    ref = np.linalg.inv(A)
    assert np.linalg.norm(inv - ref) <= bound * np.linalg.norm(ref)
    assert np.linalg.norm(A @ inv - np.eye(n)) <= 8 * n * kappa * u * np.sqrt(n)
    assert np.linalg.norm(inv - inv.T) <= bound * np.linalg.norm(ref)
    # every column is the substitution solve with the exported factor
    Lf = h.chol()
    y = sla.solve_triangular(Lf, np.eye(n), lower=True)
    x = sla.solve_triangular(Lf.T, y, lower=False)
    assert np.linalg.norm(inv - x) <= bound * np.linalg.norm(x)


def test_one_level_solve_is_the_inverse_product():
    """On one level the V-cycle is the coarsest solve: x_i = sum_k (A^-1 e_k)_i b_k.
    Compared with the product formed by NumPy in another summation order (within
    n u |A^-1||b|), and with the exact solution of the rounded inverse."""
    p = problem("ico3")
    h = oracle.Hierarchy.from_problem(p, oracle.default_options(min_coarse_points=p.n))
    assert h.num_levels == 1
    inv = h.coarse_inverse().T
    x, it, hist, st = h.solve(p.rhs, max_iters=1, tol=0.0)
    ref = inv @ p.rhs
    scale = np.abs(inv) @ np.abs(p.rhs)
    assert np.all(np.abs(x - ref) <= p.n * 2.0 ** -53 * scale)
