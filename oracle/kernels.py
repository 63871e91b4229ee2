"""Discretized integral operator (oracle; test infrastructure only).

Eqn (1.1): ``a(x) u(x) + b(x) int K(|x-y|) c(y) u(y) dy = f(x)``.  Under the
piecewise-constant collocation of Section 3.1 the linear system (eqn
linear-system) reads ``a_i u_i + b_i sum_j K_ij c_j u_j = f_i`` with ``K_ij``
the integral of the kernel over the source element (eqn kernel-integral).
Section 5 approximates every off-diagonal ``K_ij`` by the one-point rule
``K(|x_i - x_j|) h^d`` and integrates the singular diagonal term exactly; here
the diagonal term is the closed-form cell integral.

The kernel is the Laplace fundamental solution, eqn (laplace-kernel):
``G(r) = -log(r)/(2 pi)`` in 2D and ``1/(4 pi r)`` in 3D.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def green(r: np.ndarray, d: int) -> np.ndarray:
    """Laplace fundamental solution G(r), eqn (laplace-kernel)."""
    if d == 2:
        return -np.log(r) / (2.0 * np.pi)
    if d == 3:
        return 1.0 / (4.0 * np.pi * r)
    raise ValueError("d must be 2 or 3")


def self_integral(h: float, d: int) -> float:
    """Integral of G(|y|) over the element ``[-h/2, h/2]^d`` (the diagonal K_ii of eqn kernel-integral).

    2D: ``int -log r / (2 pi) = -(h^2 / (2 pi)) (log(h / sqrt 2) - 3/2 + pi/4)``.
    3D: ``int 1 / (4 pi r)    = h^2 (3 log(2 + sqrt 3) - pi/2) / (4 pi)``.
    Both are checked against adaptive quadrature of the definition in the tests.
    """
    if d == 2:
        return -(h * h / (2.0 * np.pi)) * (np.log(h / np.sqrt(2.0)) - 1.5 + np.pi / 4.0)
    if d == 3:
        return h * h * (3.0 * np.log(2.0 + np.sqrt(3.0)) - np.pi / 2.0) / (4.0 * np.pi)
    raise ValueError("d must be 2 or 3")


@dataclass
class Operator:
    """``A = diag(a) + diag(b) K diag(c)`` on collocation points (Section 3.1).

    ``weights[j]`` is the one-point quadrature weight of source element ``j``
    (``h^d`` on a uniform grid) and ``selfk[i]`` the diagonal ``K_ii``.
    """

    points: np.ndarray
    a: np.ndarray
    b: np.ndarray
    c: np.ndarray
    weights: np.ndarray
    selfk: np.ndarray

    @property
    def N(self) -> int:
        return self.points.shape[0]

    @property
    def d(self) -> int:
        return self.points.shape[1]

    @property
    def symmetric(self) -> bool:
        """True when ``b_i K_ij c_j == b_j K_ji c_i`` for all i != j, i.e. A is symmetric."""
        cw = self.c * self.weights
        return bool(np.all(self.b * cw[0] == cw * self.b[0]))

    @classmethod
    def uniform(cls, points: np.ndarray, h: float, a=None, b=None, c=None,
                weights=None, selfk=None) -> "Operator":
        """Operator on a uniform grid of step ``h``; ``a`` defaults to 0, ``b, c`` to 1."""
        N, d = points.shape
        one = np.ones(N)
        a = np.zeros(N) if a is None else np.asarray(a, dtype=np.float64)
        b = one if b is None else np.asarray(b, dtype=np.float64)
        c = one if c is None else np.asarray(c, dtype=np.float64)
        w = np.full(N, h ** d) if weights is None else np.asarray(weights, dtype=np.float64)
        s = np.full(N, self_integral(h, d)) if selfk is None else np.asarray(selfk, dtype=np.float64)
        return cls(np.asarray(points, dtype=np.float64), a, b, c, w, s)

    def kernel_block(self, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
        """``b_i K_ij c_j`` for ``i in rows, j in cols`` (no ``a`` term).

        Off-diagonal: one-point rule ``G(|x_i - x_j|) w_j``; coincident indices
        take the cell integral ``K_ii``.
        """
        rows = np.asarray(rows)
        cols = np.asarray(cols)
        diff = self.points[rows][:, None, :] - self.points[cols][None, :, :]
        r = np.sqrt(np.sum(diff * diff, axis=2))
        same = rows[:, None] == cols[None, :]
        with np.errstate(divide="ignore"):
            g = green(np.where(same, 1.0, r), self.d)
        K = g * self.weights[cols][None, :]
        ii, jj = np.nonzero(same)
        K[ii, jj] = self.selfk[rows[ii]]
        return self.b[rows][:, None] * K * self.c[cols][None, :]

    def block(self, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
        """``A[rows][:, cols]`` including the ``a`` term on coincident indices."""
        rows = np.asarray(rows)
        cols = np.asarray(cols)
        B = self.kernel_block(rows, cols)
        ii, jj = np.nonzero(rows[:, None] == cols[None, :])
        B[ii, jj] += self.a[rows[ii]]
        return B

    def dense(self) -> np.ndarray:
        """The full ``N x N`` matrix A (only for small N)."""
        idx = np.arange(self.N)
        return self.block(idx, idx)

    def matvec(self, x: np.ndarray, chunk: int = 1024, rows: np.ndarray | None = None) -> np.ndarray:
        """Exact ``A x`` evaluated on the fly, ``O(N^2)``; ``x`` is ``(N,)`` or ``(nrhs, N)``.

        With ``rows`` only those entries of ``A x`` are returned.
        """
        x = np.asarray(x, dtype=np.float64)
        X = x[None, :] if x.ndim == 1 else x
        rows = np.arange(self.N) if rows is None else np.asarray(rows)
        out = np.empty((X.shape[0], rows.size))
        cols = np.arange(self.N)
        for s in range(0, rows.size, chunk):
            rr = rows[s:s + chunk]
            out[:, s:s + chunk] = (self.block(rr, cols) @ X.T).T
        return out[0] if x.ndim == 1 else out

    def rmatvec(self, x: np.ndarray, chunk: int = 1024) -> np.ndarray:
        """Exact ``A^T x`` on the fly."""
        x = np.asarray(x, dtype=np.float64)
        X = x[None, :] if x.ndim == 1 else x
        out = np.zeros((X.shape[0], self.N))
        cols = np.arange(self.N)
        for s in range(0, self.N, chunk):
            rr = cols[s:s + chunk]
            out += (self.block(rr, cols).T @ X[:, s:s + chunk].T).T
        return out[0] if x.ndim == 1 else out
