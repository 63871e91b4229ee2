"""Error estimators and GMRES (oracle; test infrastructure only).

Section 5: ``e_a ~ |A - F| / |A|`` and ``e_s ~ |I - A F^{-1}|`` are estimated by
power iteration from a standard uniform random start vector, stopped at a
relative change of 1e-2 in the norm estimate.  GMRES (used with ``F^{-1}`` as
preconditioner, Section 5 and Lemma 5.1) is written out with modified
Gram-Schmidt Arnoldi and Givens rotations; right preconditioning so the
monitored residual is the true residual of ``A u = f``.
"""
from __future__ import annotations

import numpy as np


def power_norm(op, op_T, n: int, seed: int = 0, rtol: float = 1e-2, maxit: int = 200) -> float:
    """Estimate the 2-norm of a linear map by power iteration on ``op_T(op(.))``."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(size=n)
    v /= np.linalg.norm(v)
    est = 0.0
    for _ in range(maxit):
        w = op_T(op(v))
        nw = np.linalg.norm(w)
        new = np.sqrt(nw)
        if nw == 0.0:
            return 0.0
        v = w / nw
        if est > 0.0 and abs(new - est) <= rtol * new:
            return new
        est = new
    return est


def e_apply(A_mv, A_rmv, F, n: int, seed: int = 0) -> float:
    """``e_a``: power-iteration estimate of ``|A - F| / |A|``."""
    num = power_norm(lambda x: A_mv(x) - F.apply(x), lambda y: A_rmv(y) - F.apply_T(y), n, seed)
    den = power_norm(A_mv, A_rmv, n, seed)
    return num / den


def e_solve(A_mv, A_rmv, F, n: int, seed: int = 0) -> float:
    """``e_s``: power-iteration estimate of ``|I - A F^{-1}|``."""
    return power_norm(lambda x: x - A_mv(F.solve(x)), lambda y: y - F.solve_T(A_rmv(y)), n, seed)


def gmres(A_mv, f: np.ndarray, M=None, tol: float = 1e-12, maxit: int = 50, x0=None):
    """Right-preconditioned GMRES without restart for ``A u = f``.

    Solves ``A M z = f`` and returns ``(u = M z, iterations, relative residual history)``.
    """
    f = np.asarray(f, dtype=np.float64)
    M = (lambda v: v) if M is None else M
    n = f.size
    u0 = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    r0 = f - A_mv(u0) if x0 is not None else f.copy()
    beta = np.linalg.norm(r0)
    nf = np.linalg.norm(f)
    hist = [beta / nf]
    if beta == 0.0 or beta / nf <= tol:
        return u0, 0, hist
    V = np.zeros((maxit + 1, n))
    H = np.zeros((maxit + 1, maxit))
    cs = np.zeros(maxit)
    sn = np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    V[0] = r0 / beta
    k = 0
    for j in range(maxit):
        w = A_mv(M(V[j]))
        for i in range(j + 1):
            H[i, j] = w @ V[i]
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] > 0.0:
            V[j + 1] = w / H[j + 1, j]
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        den = np.hypot(H[j, j], H[j + 1, j])
        cs[j] = H[j, j] / den
        sn[j] = H[j + 1, j] / den
        H[j, j] = den
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        k = j + 1
        hist.append(abs(g[j + 1]) / nf)
        if hist[-1] <= tol:
            break
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
    z = V[:k].T @ y
    return u0 + M(z), k, hist
