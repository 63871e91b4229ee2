"""Pins of the oracle's dense adjoint (no GPU): gradients of
``L = |A(a)^{-1} f - u_target|^2 / 2`` against central differences of the
dense solve itself, on a non-symmetric operator so that a transposed
operand in the adjoint would show."""
import numpy as np

from oracle.adjoint import dense_solve_loss, dense_solve_loss_grad
from oracle.kernels import Operator
from workloads import diff_problem, grid_points


def _nonsym_op(n=12, seed=3):
    rng = np.random.default_rng(seed)
    P = grid_points(n, 2)
    N = P.shape[0]
    return Operator.uniform(P, 1.0 / n, a=1.0 + rng.uniform(0, 0.5, N), b=rng.uniform(0.5, 2.0, N),
                            c=rng.uniform(0.5, 2.0, N)), rng


def _with_a(op, a):
    return Operator(op.points, a, op.b, op.c, op.weights, op.selfk)


def test_grad_a_matches_central_differences_every_entry():
    op, rng = _nonsym_op()
    N = op.N
    f = rng.standard_normal((2, N))
    t = rng.standard_normal((2, N))
    _, L, ga, _ = dense_solve_loss_grad(op, f, t)
    assert L > 0
    d = 1e-6
    fd = np.empty(N)
    for i in range(N):
        ap, am = op.a.copy(), op.a.copy()
        ap[i] += d
        am[i] -= d
        fd[i] = (dense_solve_loss(_with_a(op, ap), f, t)[1] - dense_solve_loss(_with_a(op, am), f, t)[1]) / (2 * d)
    assert np.max(np.abs(fd - ga)) <= 1e-6 * np.max(np.abs(ga))


def test_grad_f_matches_central_differences():
    op, rng = _nonsym_op(n=10, seed=4)
    N = op.N
    f = rng.standard_normal(N)
    t = rng.standard_normal(N)
    _, _, _, gf = dense_solve_loss_grad(op, f, t)
    for _ in range(8):
        w = rng.standard_normal(N)
        d = 1e-4
        fd = (dense_solve_loss(op, f + d * w, t)[1] - dense_solve_loss(op, f - d * w, t)[1]) / (2 * d)
        # L is quadratic in f: the central difference is exact up to rounding
        assert abs(fd - gf @ w) <= 1e-8 * np.linalg.norm(gf) * np.linalg.norm(w)


def test_diagonal_operator_closed_form():
    # K = 0 (b = 0): u = f / a, dL/da = -(u - t) u / a, dL/df = (u - t) / a
    op, rng = _nonsym_op(n=8, seed=5)
    op = Operator(op.points, op.a, np.zeros(op.N), op.c, op.weights, op.selfk)
    f = rng.standard_normal(op.N)
    t = rng.standard_normal(op.N)
    u, L, ga, gf = dense_solve_loss_grad(op, f, t)
    np.testing.assert_allclose(u, f / op.a, rtol=1e-15)
    np.testing.assert_allclose(gf, (u - t) / op.a, rtol=1e-14)
    np.testing.assert_allclose(ga, -(u - t) * u / op.a, rtol=1e-14)
    assert abs(L - 0.5 * np.sum((u - t) ** 2)) <= 1e-14 * L


def test_diff_problem_inputs():
    p = diff_problem(32)
    assert p.points.shape == (1024, 2) and p.a.shape == (1024,)
    assert np.all(p.a >= 1.0) and np.all(p.a <= 1.0 + 0.5 * 64)
    assert p.a.max() > 1.1
    assert not np.allclose(p.f, p.u_target)
    q = diff_problem(32)
    assert np.array_equal(p.a, q.a) and np.array_equal(p.f, q.f)


def test_batch_problems_inputs():
    from workloads import batch_problems
    b = batch_problems()
    assert len(b) == 48
    assert {p["n"] for p in b} <= {64, 96, 128, 192, 256}
    for p in b:
        assert p["leaf"] == (36 if p["n"] in (96, 192) else 64)
        assert p["points"].shape == (p["n"] ** 2, 2) and p["f"].shape == (4, p["n"] ** 2)
        assert p["a"].min() == 1.0 and p["a"].max() == 2.0
    c = batch_problems()
    assert all(np.array_equal(x["a"], y["a"]) and np.array_equal(x["f"], y["f"]) for x, y in zip(b, c))
