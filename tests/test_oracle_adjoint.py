"""Pins of the gradient formula of a loss through the solve (the oracle's
adjoint_gradients), by central finite differences of the oracle's own
multigrid solve run to convergence: dL/db_i and dL/dA_ij (one stored entry at
a time, the matrix then no longer symmetric) for L = ||x - x*||^2."""
import numpy as np
import pytest

import oracle
import synth
from tests.conftest import problem


def loss_and_x(prob, data, b, target):
    h = oracle.Hierarchy(prob.points, prob.edges, prob.indptr, prob.indices, data,
                         oracle.default_options(min_coarse_points=100))
    x, it, hist, st = h.solve(b, tol=1e-14, max_iters=400)
    assert st == 0 or hist[-1] < 1e-13
    return float(((x - target) ** 2).sum()), x


@pytest.mark.parametrize("name", ["ico3", "torus48"])
def test_adjoint_gradients_match_finite_differences(name):
    prob = problem(name)
    target = synth.uniform(0, "target", prob.n, -1.0, 1.0)
    L0, x = loss_and_x(prob, prob.data, prob.rhs, target)
    gb, gA = oracle.adjoint_gradients(prob.indptr, prob.indices, prob.data, x, 2.0 * (x - target))
    rng = np.random.default_rng(21)
    h = 1e-5
    for e in rng.choice(prob.nnz, 12, replace=False):
        dp, dm = prob.data.copy(), prob.data.copy()
        dp[e] += h
        dm[e] -= h
        fd = (loss_and_x(prob, dp, prob.rhs, target)[0] - loss_and_x(prob, dm, prob.rhs, target)[0]) / (2 * h)
        assert abs(fd - gA[e]) <= 1e-5 * max(1.0, abs(gA).max()), (e, fd, gA[e])
    for i in rng.choice(prob.n, 6, replace=False):
        bp, bm = prob.rhs.copy(), prob.rhs.copy()
        bp[i] += h
        bm[i] -= h
        fd = (loss_and_x(prob, prob.data, bp, target)[0] - loss_and_x(prob, prob.data, bm, target)[0]) / (2 * h)
        assert abs(fd - gb[i]) <= 1e-5 * max(1.0, abs(gb).max()), (i, fd, gb[i])


def test_adjoint_gradients_dense_identities():
    """For L = c.x: dL/db = A^-T c and sum_ij dL/dA_ij A_ij = -lambda.(A x) = -c.x (on the pattern)."""
    prob = problem("ico3")
    A = prob.matrix().toarray()
    x = np.linalg.solve(A, prob.rhs)
    c = synth.uniform(1, "target", prob.n, -1.0, 1.0)
    gb, gA = oracle.adjoint_gradients(prob.indptr, prob.indices, prob.data, x, c)
    assert np.allclose(gb, np.linalg.solve(A.T, c), rtol=1e-10, atol=1e-12)
    assert abs((gA * prob.data).sum() + c @ x) <= 1e-10 * abs(c @ x)
