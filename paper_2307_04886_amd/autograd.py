"""Differentiable solve: a torch.autograd.Function whose backward pass solves
the adjoint system with the same multigrid hierarchy.

For A x = b with A symmetric (the systems of the method are), a loss L(x)
has
    dL/db = lambda,   dL/dA_ij = -lambda_i x_j  (on A's stored entries),
where A lambda = dL/dx.  The forward and the adjoint solve both run through
the C ABI (gmg_solve or gmg_solve_pcg); the pattern product is
gmg_pattern_outer.  The hierarchy must hold the same values of A as the
A_val tensor passed in: build it from them, or refresh it with
Hierarchy.update_matrix (refresh=True does that before the solve).
"""
import torch

from .binding import pattern_outer


def _run(hier, rhs, tol, max_iters, method):
    x = torch.zeros_like(rhs)
    if method == "vcycle":
        _, info, st = hier.solve(rhs, x, tol=tol, max_iters=max_iters)
    else:
        _, info, st = hier.solve_pcg(rhs, x, tol=tol, max_iters=max_iters, precision=method[-3:])
    if st != 0:
        raise RuntimeError(f"solve did not reach tol {tol} in {max_iters} iterations "
                           f"(rel. residual {info.rel_residual:.3e})")
    return x


class GMGSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A_val, b, hier, tol, max_iters, method):
        x = _run(hier, b.detach().contiguous(), tol, max_iters, method)
        ctx.hier = hier
        ctx.opts = (tol, max_iters, method)
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, grad_x):
        (x,) = ctx.saved_tensors
        tol, max_iters, method = ctx.opts
        lam = _run(ctx.hier, grad_x.contiguous(), tol, max_iters, method)
        grad_A = None
        if ctx.needs_input_grad[0]:
            grad_A = pattern_outer(ctx.hier.rowptr, ctx.hier.col, lam, x, scale=-1.0)
        grad_b = lam if ctx.needs_input_grad[1] else None
        return grad_A, grad_b, None, None, None, None


def solve(hier, A_val, b, tol=1e-10, max_iters=200, method="pcg_f64", refresh=False):
    """x = A^-1 b, differentiable in A_val (values of A on the hierarchy's pattern) and b.

    method: "vcycle" (Alg. 1), "pcg_f64" or "pcg_f32" (CG preconditioned by the
    symmetric V-cycle in double or float).  refresh=True first loads A_val into
    the hierarchy (gmg_update_matrix)."""
    if refresh:
        hier.update_matrix(A_val.detach().contiguous())
    return GMGSolve.apply(A_val, b, hier, tol, max_iters, method)
