"""Dense adjoint of the discretized system (oracle; test infrastructure only).

The paper solves ``A u = f`` for the linear system of Section 3.1,
``A = diag(a) + diag(b) K diag(c)``; it does not differentiate the solve.
For a loss ``L(u)`` the adjoint of that system gives, with
``lambda = A^{-T} dL/du``:

* ``dL/df = lambda`` (``u`` is linear in ``f``);
* ``dL/da_i = -lambda_i u_i``, because ``dA/da_i = e_i e_i^T`` and
  ``du = -A^{-1} (dA) u``.

Here ``L = |u - u_target|^2 / 2`` summed over the right-hand sides, so
``dL/du = u - u_target``; the gradient in ``a`` is summed over right-hand
sides that share ``A``.  Everything is dense FP64 and LAPACK (small ``N``).
"""
from __future__ import annotations

import numpy as np

from .kernels import Operator


def dense_solve_loss(op: Operator, f: np.ndarray, u_target: np.ndarray):
    """``(u, L)`` with ``u = A^{-1} f`` by dense LU and ``L = |u - u_target|^2 / 2``."""
    A = op.dense()
    F = np.atleast_2d(np.asarray(f, dtype=np.float64))
    U = np.linalg.solve(A, F.T).T
    R = U - np.atleast_2d(u_target)
    u = U[0] if np.ndim(f) == 1 else U
    return u, 0.5 * float(np.sum(R * R))


def dense_solve_loss_grad(op: Operator, f: np.ndarray, u_target: np.ndarray):
    """``(u, L, dL/da, dL/df)`` of the dense solve, by the adjoint equation ``A^T lambda = u - u_target``."""
    A = op.dense()
    F = np.atleast_2d(np.asarray(f, dtype=np.float64))
    U = np.linalg.solve(A, F.T).T
    R = U - np.atleast_2d(u_target)
    lam = np.linalg.solve(A.T, R.T).T
    grad_a = -np.sum(lam * U, axis=0)
    vec = np.ndim(f) == 1
    return (U[0] if vec else U), 0.5 * float(np.sum(R * R)), grad_a, (lam[0] if vec else lam)
