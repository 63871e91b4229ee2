"""Pins of the oracle's estimators and GMRES (Section 5, Lemma 5.1)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.estimators import e_apply, e_solve, gmres, power_norm
from oracle.factor import factorize
from oracle.kernels import Operator
from workloads import grid_points


def test_power_norm_matches_svd():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((80, 80)) @ np.diag(np.linspace(1, 10, 80))
    est = power_norm(lambda x: M @ x, lambda y: M.T @ y, 80)
    assert abs(est - np.linalg.norm(M, 2)) <= 2e-2 * np.linalg.norm(M, 2)


def test_error_estimates_match_dense_norms():
    # e_a and e_s estimated by power iteration (Section 5) against dense 2-norms.
    n = 32
    pts = grid_points(n, 2)
    N = n * n
    op = Operator.uniform(pts, 1.0 / n, a=np.ones(N))
    A = op.dense()
    F = factorize(op, 1e-4, leaf=16, second_kind=False)
    I = np.eye(N)
    Fd = F.apply(I).T
    Fi = F.solve(I).T
    ea_true = np.linalg.norm(A - Fd, 2) / np.linalg.norm(A, 2)
    es_true = np.linalg.norm(I - A @ Fi, 2)
    ea = e_apply(lambda x: A @ x, lambda y: A.T @ y, F, N)
    es = e_solve(lambda x: A @ x, lambda y: A.T @ y, F, N)
    assert 0.5 * ea_true <= ea <= 1.02 * ea_true
    assert 0.5 * es_true <= es <= 1.02 * es_true


def test_gmres_matches_scipy_and_direct():
    rng = np.random.default_rng(1)
    n = 60
    A = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    f = rng.standard_normal(n)
    u, it, hist = gmres(lambda x: A @ x, f, tol=1e-12, maxit=60)
    assert np.linalg.norm(A @ u - f) <= 1e-11 * np.linalg.norm(f)
    assert np.allclose(u, np.linalg.solve(A, f), rtol=1e-9, atol=1e-11)
    us, info = spla.gmres(A, f, rtol=1e-12, restart=60, maxiter=1)
    assert info == 0 and np.allclose(u, us, rtol=1e-8, atol=1e-10)
    # the monitored residual is non-increasing (GMRES minimizes it)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(hist, hist[1:]))


@pytest.mark.parametrize("eps", [1e-3, 1e-6])
def test_gmres_iterations_obey_lemma_5_1(eps):
    # Lemma 5.1: preconditioning with F^{-1} gives I + E, |E| = e_s, so GMRES
    # reaches eps0 within log(eps0)/log(e_s) iterations (plus one for the
    # estimate's slack).
    n = 32
    pts = grid_points(n, 2)
    N = n * n
    op = Operator.uniform(pts, 1.0 / n, a=np.zeros(N))   # first kind: a = 0
    A = op.dense()
    F = factorize(op, eps, leaf=16, second_kind=False)
    es = np.linalg.norm(np.eye(N) - A @ F.solve(np.eye(N)).T, 2)
    f = np.random.default_rng(2).uniform(size=N)
    eps0 = 1e-12
    u, it, hist = gmres(lambda x: A @ x, f, M=F.solve, tol=eps0, maxit=50)
    assert np.linalg.norm(A @ u - f) <= 10 * eps0 * np.linalg.norm(f)
    if es < 1:
        assert it <= int(np.ceil(np.log(eps0) / np.log(es))) + 1
