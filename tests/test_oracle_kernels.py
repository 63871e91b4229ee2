"""Pins of the oracle's operator (CPU): kernel, self terms, dense assembly, matvec.

Each check compares against something the mathematics fixes independently of
the oracle's own formulas: adaptive quadrature of the defining integral,
Gauss's flux law for the fundamental solution, and convergence of the
discretized potential of a uniform square to its exact value.
"""
import numpy as np
import pytest
from scipy import integrate

from oracle.kernels import Operator, green, self_integral
from workloads import grid_points


@pytest.mark.parametrize("h", [1 / 64, 1 / 512, 1 / 96])
def test_self_integral_2d_matches_quadrature(h):
    # K_ii of eqn (kernel-integral): integral of -log r/(2 pi) over the h x h cell.
    q = 4 * integrate.dblquad(lambda y, x: -np.log(np.hypot(x, y)) / (2 * np.pi),
                              0, h / 2, 0, h / 2, epsabs=0, epsrel=1e-13)[0]
    assert abs(q - self_integral(h, 2)) <= 1e-13 * abs(q)


@pytest.mark.parametrize("h", [1 / 32, 1 / 64])
def test_self_integral_3d_matches_quadrature(h):
    q = 8 * integrate.tplquad(lambda z, y, x: 1.0 / (4 * np.pi * np.sqrt(x * x + y * y + z * z)),
                              0, h / 2, 0, h / 2, 0, h / 2, epsabs=0, epsrel=1e-11)[0]
    assert abs(q - self_integral(h, 3)) <= 1e-10 * abs(q)


@pytest.mark.parametrize("d", [2, 3])
def test_green_flux_is_minus_one(d):
    # Fundamental solution of -Laplace (eqn laplace-kernel): the outward flux of grad G
    # through any sphere about the source is -1, and G is harmonic away from it.
    for r in (0.3, 1.0, 2.5):
        dr = 1e-5
        dG = (green(np.array(r + dr), d) - green(np.array(r - dr), d)) / (2 * dr)
        area = 2 * np.pi * r if d == 2 else 4 * np.pi * r * r
        assert abs(dG * area + 1.0) < 1e-8
    # Harmonic: radial Laplacian G'' + (d-1)/r G' vanishes.
    r, dr = 0.7, 1e-4
    g = lambda t: green(np.array(t), d)
    lap = (g(r + dr) - 2 * g(r) + g(r - dr)) / dr ** 2 + (d - 1) / r * (g(r + dr) - g(r - dr)) / (2 * dr)
    assert abs(lap) < 1e-5


def test_green_2d_zero_at_unit_distance():
    assert green(np.array(1.0), 2) == 0.0


def test_discrete_potential_converges_to_square_potential():
    # sum_j K_cj over the unit square from its centre approximates the exact
    # potential int_{[-1/2,1/2]^2} G = self_integral(1, 2); the one-point rule
    # error shrinks as h^2 (up to log factors).
    exact = self_integral(1.0, 2)
    errs = []
    for n in (33, 65, 129):
        pts = grid_points(n, 2)
        op = Operator.uniform(pts, 1.0 / n)
        ctr = (n * n) // 2
        assert np.allclose(pts[ctr], [0.5, 0.5])
        s = op.kernel_block(np.array([ctr]), np.arange(n * n)).sum()
        errs.append(abs(s - exact) / abs(exact))
    assert errs[-1] < 2e-4
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_dense_assembly_properties():
    n = 16
    pts = grid_points(n, 2)
    N = n * n
    h = 1.0 / n
    op = Operator.uniform(pts, h, a=np.ones(N))
    A = op.dense()
    assert op.symmetric
    assert np.array_equal(A, A.T)
    assert np.allclose(np.diag(A), 1.0 + self_integral(h, 2), rtol=0, atol=0)
    # An off-diagonal entry from its definition: G(|x_i - x_j|) h^2.
    i, j = 3, 200
    r = np.linalg.norm(pts[i] - pts[j])
    assert A[i, j] == pytest.approx(-np.log(r) / (2 * np.pi) * h * h, rel=1e-15)
    # Non-symmetric coefficients make A non-symmetric.
    rng = np.random.default_rng(0)
    op2 = Operator.uniform(pts, h, a=np.ones(N), b=1 + rng.uniform(size=N), c=np.ones(N))
    assert not op2.symmetric
    A2 = op2.dense()
    assert A2[i, j] == pytest.approx(op2.b[i] * A[i, j], rel=1e-14)


def test_matvec_matches_dense():
    n = 20
    pts = grid_points(n, 2)
    N = n * n
    rng = np.random.default_rng(1)
    op = Operator.uniform(pts, 1.0 / n, a=rng.uniform(size=N), b=rng.uniform(size=N) + 0.5,
                          c=rng.uniform(size=N) + 0.5)
    A = op.dense()
    X = rng.standard_normal((3, N))
    assert np.allclose(op.matvec(X, chunk=37), X @ A.T, rtol=1e-13, atol=1e-14)
    assert np.allclose(op.rmatvec(X, chunk=37), X @ A, rtol=1e-13, atol=1e-14)
    rows = np.array([0, 5, 399])
    assert np.allclose(op.matvec(X[0], rows=rows), (A @ X[0])[rows], rtol=1e-13)
