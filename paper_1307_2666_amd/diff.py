"""Differentiable solve through the factorization.

``solve(points, a, f, ...)`` returns ``u = A(a)^{-1} f`` for the operator of
eqn 1.1 with ``b = c = 1`` and weights ``h^d`` (the linear system of
Section 3.1), as a ``torch.autograd.Function``: the forward factors ``A(a)``
on the device (``hif_factor``) and solves (``hif_solve``, or ``hif_gmres``
to the exact operator with ``refine``); the backward solves the adjoint
system ``A^T lambda = dL/du`` with the same factorization (``hif_solve_T``,
or ``hif_gmres_T``) and returns ``dL/df = lambda`` and
``dL/da = -sum_r lambda_r * u_r`` (``hif_diag_grad``).

Without ``refine`` the gradients are those of the factored map ``F^{-1}``,
accurate to about the factorization's ``eps``; with ``refine`` they are
those of the exact map to the GMRES tolerance.  The factorization is held
by the autograd graph until it is released.
"""
from __future__ import annotations

import torch

from ._binding import HIF_FP64, diag_grad, factor

__all__ = ["solve"]


class _HifSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, f, points, eps, leaf, h, precision, refine, tol, maxit):
        fac = factor(points, eps, leaf, a=a.detach(), h=h, precision=precision)
        fd = f.detach()
        if refine:
            u, its, rr = fac.gmres(fd, tol=tol, maxit=maxit)
            _converged(its, rr, tol, maxit, "forward")
        else:
            u = fac.solve(fd)
        ctx.fac = fac
        ctx.refine = (refine, tol, maxit)
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, gu):
        (u,) = ctx.saved_tensors
        refine, tol, maxit = ctx.refine
        g = gu.to(torch.float64).contiguous()
        if refine:
            lam, its, rr = ctx.fac.gmres(g, tol=tol, maxit=maxit, transpose=True)
            _converged(its, rr, tol, maxit, "adjoint")
        else:
            lam = ctx.fac.solve_T(g)
        grad_a = diag_grad(lam, u) if ctx.needs_input_grad[0] else None
        grad_f = lam if ctx.needs_input_grad[1] else None
        return grad_a, grad_f, None, None, None, None, None, None, None, None


def _converged(its, rr, tol, maxit, what):
    bad = [r for r, i in zip(rr, its) if i >= maxit and r > tol]
    if bad:
        raise RuntimeError(f"GMRES ({what}) stopped at {maxit} iterations with relative residual {max(bad):.3e}")


def solve(points, a, f, eps, leaf, *, h, precision=HIF_FP64, refine=False, tol=1e-12, maxit=50):
    """``u = A(a)^{-1} f`` with gradients in ``a`` and ``f``.

    ``points``: ``(n, d)``; ``a``: ``(n,)``; ``f``: ``(n,)`` or ``(nrhs, n)``; ``h``:
    grid step (weights ``h^d`` and the closed-form self term).  ``a`` and ``f``
    are moved to the GPU in float64 (differentiably); ``u`` lives there.
    """
    n = points.shape[0]
    if tuple(a.shape) != (n,):
        raise ValueError(f"a must have shape ({n},)")
    if f.dim() not in (1, 2) or f.shape[-1] != n:
        raise ValueError(f"f must have shape ({n},) or (nrhs, {n})")
    if refine and not (0.0 < tol < 1.0):
        raise ValueError("tol must satisfy 0 < tol < 1")
    a_d = a.to(device="cuda", dtype=torch.float64)
    f_d = f.to(device="cuda", dtype=torch.float64)
    return _HifSolve.apply(a_d, f_d, points, float(eps), int(leaf), float(h), int(precision), bool(refine),
                           float(tol), int(maxit))
