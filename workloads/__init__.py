"""Seeded synthetic inputs for the HIF-IE workloads.

This module only builds input arrays: grid points, coefficient fields and
right-hand sides, from fixed seeds.  It holds none of the factorization's
arithmetic, so that the CPU oracle (``oracle/``) and the HIP library
(``paper_1307_2666_amd``) can both be fed identical arrays without sharing
any code of the method.

Grids follow the piecewise-constant collocation set-up of the paper
(Section 3.1 for 2D, Section 3.2 for 3D): the unit square / cube is cut into
an ``n^d`` uniform grid of step ``h = 1/n`` and each unknown sits at a cell
centre.  Point ``i + n*j (+ n^2*k)`` is at ``((i+1/2)h, (j+1/2)h[, (k+1/2)h])``,
i.e. the x index runs fastest.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "grid_points",
    "Workload",
    "WORKLOADS",
    "workload",
    "rhs",
    "gaussian_bump_field",
    "DiffProblem",
    "diff_problem",
    "batch_problems",
]


def grid_points(n: int, d: int) -> np.ndarray:
    """Cell centres of the uniform ``n^d`` grid on ``[0,1]^d`` as an ``(n^d, d)`` float64 array."""
    if d not in (2, 3):
        raise ValueError("d must be 2 or 3")
    h = 1.0 / n
    c = (np.arange(n, dtype=np.float64) + 0.5) * h
    if d == 2:
        yy, xx = np.meshgrid(c, c, indexing="ij")
        return np.ascontiguousarray(np.stack([xx.ravel(), yy.ravel()], axis=1))
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    return np.ascontiguousarray(np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1))


@dataclass(frozen=True)
class Workload:
    """One synthetic problem: grid side ``n``, dimension ``d``, ID precision, leaf size, RHS."""

    name: str
    n: int
    d: int
    eps: float
    leaf: int
    nrhs: int
    seed: int

    @property
    def N(self) -> int:
        return self.n ** self.d

    @property
    def h(self) -> float:
        return 1.0 / self.n

    def points(self) -> np.ndarray:
        return grid_points(self.n, self.d)

    def rhs(self) -> np.ndarray:
        return rhs(self.N, self.nrhs, self.seed)


# Second-kind Laplace volume IEs with a = b = c = 1 (the paper's Examples 2
# and 6), leaf boxes of 64 points.
WORKLOADS = {
    "sq64": Workload("sq64", 64, 2, 1e-6, 64, 1, 0),
    "sq512": Workload("sq512", 512, 2, 1e-6, 64, 8, 1),
    "cube32": Workload("cube32", 32, 3, 1e-6, 64, 1, 2),
    "cube64": Workload("cube64", 64, 3, 1e-6, 64, 1, 3),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def rhs(N: int, nrhs: int, seed: int) -> np.ndarray:
    """``nrhs`` standard-normal right-hand sides as a ``(nrhs, N)`` array (each RHS contiguous)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.standard_normal((nrhs, N)))


def gaussian_bump_field(points: np.ndarray, n_bumps: int, sigma: float, wmax: float,
                        seed: int, normalize: bool = False) -> np.ndarray:
    """Smooth random field ``sum_k w_k exp(-|x-c_k|^2/(2 sigma^2))`` at ``points``.

    ``w_k ~ U(0, wmax)`` and ``c_k ~ U[0,1]^d`` come from ``default_rng(seed)``.
    With ``normalize`` the field is min-max scaled to ``[0, 1]`` over the points.
    """
    rng = np.random.default_rng(seed)
    d = points.shape[1]
    w = rng.uniform(0.0, wmax, n_bumps)
    ctr = rng.uniform(0.0, 1.0, (n_bumps, d))
    g = np.zeros(points.shape[0])
    for k in range(n_bumps):
        r2 = np.sum((points - ctr[k]) ** 2, axis=1)
        g += w[k] * np.exp(-r2 / (2.0 * sigma * sigma))
    if normalize:
        lo, hi = g.min(), g.max()
        g = (g - lo) / (hi - lo) if hi > lo else np.zeros_like(g)
    return g


@dataclass(frozen=True)
class DiffProblem:
    """Inputs of a differentiated solve ``L = |u - u_target|^2 / 2`` with ``A(a) u = f``."""

    n: int
    h: float
    points: np.ndarray
    a: np.ndarray
    f: np.ndarray
    u_target: np.ndarray


def diff_problem(n: int = 256, seed_a: int = 5, seed_target: int = 6, seed_f: int = 7) -> DiffProblem:
    """2D grid ``n x n`` with ``a = 1 + sum_{k<64} w_k exp(-|x-c_k|^2 / (2 * 0.05^2))``,
    ``w_k ~ U(0, 0.5)``, ``c_k ~ U[0,1]^2`` (seed ``seed_a``); ``f`` and ``u_target``
    standard normal from their own seeds; ``b = c = 1``."""
    P = grid_points(n, 2)
    a = 1.0 + gaussian_bump_field(P, 64, 0.05, 0.5, seed_a)
    N = P.shape[0]
    return DiffProblem(n, 1.0 / n, P, a, rhs(N, 1, seed_f)[0], rhs(N, 1, seed_target)[0])


def batch_problems(count: int = 48, seed: int = 4):
    """Independent 2D problems of uneven sizes: sides drawn from
    ``{64, 96, 128, 192, 256}`` (``default_rng(seed)``); leaves of 6 x 6 points
    for sides 96 and 192 and 8 x 8 otherwise (uniform tree depth);
    ``a = 1 + g`` with ``g`` a field of 16 Gaussian bumps (width 0.1, weights
    ``U(0, 1)``, seed ``1000 + i``) min-max scaled to ``[0, 1]``; 4 standard
    normal right-hand sides (seed ``2000 + i``); ``b = c = 1``, eps 1e-6.
    Returns a list of dicts with ``n``, ``h``, ``leaf``, ``eps``, ``points``,
    ``a``, ``f``."""
    rng = np.random.default_rng(seed)
    sides = rng.choice([64, 96, 128, 192, 256], count)
    out = []
    for i, n in enumerate(int(s) for s in sides):
        P = grid_points(n, 2)
        a = 1.0 + gaussian_bump_field(P, 16, 0.1, 1.0, 1000 + i, normalize=True)
        out.append(dict(n=n, h=1.0 / n, leaf=36 if n in (96, 192) else 64, eps=1e-6, points=P, a=a,
                        f=rhs(P.shape[0], 4, 2000 + i)))
    return out
