"""GPU parity of the differentiated solve and its two entry points
(hif_gmres_T, hif_diag_grad), all through the C ABI.

* hif_gmres_T against a dense FP64 solve with A^T on a non-symmetric operator.
* hif_diag_grad against its definition.
* diff.solve (forward + backward) against the oracle's dense adjoint at 64^2,
  refined (GMRES to 1e-12) and direct, FP64 and mixed.
* At 256^2 (the differentiated-solve workload): central differences of the
  refined map along 16 random directions of a and 4 of f, and agreement of
  the FP64 and mixed refined gradients.
"""
import numpy as np
import pytest
import torch

import paper_1307_2666_amd as hif
from oracle.adjoint import dense_solve_loss_grad
from oracle.kernels import Operator
from workloads import diff_problem, grid_points

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(x, **kw):
    return torch.tensor(np.ascontiguousarray(x), device=DEV, **kw)


def _np(t):
    return t.detach().cpu().numpy()


def _rel(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def test_gmres_T_matches_dense_transposed_solve():
    n = 48
    P = grid_points(n, 2)
    N = P.shape[0]
    rng = np.random.default_rng(8)
    b = 1.0 + 0.5 * rng.uniform(size=N)
    c = 1.0 + 0.5 * rng.uniform(size=N)
    a = 1.0 + 0.2 * rng.uniform(size=N)
    op = Operator.uniform(P, 1.0 / n, a=a, b=b, c=c)
    F = hif.factor(_t(P), 1e-4, 64, a=_t(a), b=_t(b), c=_t(c), h=1.0 / n)
    f = rng.standard_normal((2, N))
    u, its, rr = F.gmres(_t(f), tol=1e-11, maxit=40, transpose=True)
    A = op.dense()
    uT = np.linalg.solve(A.T, f.T).T
    u0 = np.linalg.solve(A, f.T).T
    assert max(rr) <= 2e-11, rr
    assert max(its) <= 12, its
    for v in range(2):
        assert _rel(_np(u)[v], uT[v]) <= 1e-10
        assert _rel(u0[v], uT[v]) > 1e-6  # the transpose matters for this operator
    # the non-transposed refinement on the same handle still solves A u = f
    w, _, rr0 = F.gmres(_t(f), tol=1e-11, maxit=40)
    assert max(rr0) <= 2e-11 and _rel(_np(w), u0) <= 1e-10


@pytest.mark.parametrize("nrhs,n", [(1, 1), (3, 1000), (2, 70001)])
def test_diag_grad_matches_definition(nrhs, n):
    rng = np.random.default_rng(nrhs * 7 + n)
    lam = rng.standard_normal((nrhs, n))
    u = rng.standard_normal((nrhs, n))
    g = _np(hif.diag_grad(_t(lam), _t(u)))
    ref = -np.sum(lam * u, axis=0)
    bound = 4 * 2.0 ** -53 * np.sum(np.abs(lam * u), axis=0)
    assert np.all(np.abs(g - ref) <= bound)


def _loss(u, t):
    return 0.5 * torch.sum((u - t) ** 2)


@pytest.mark.parametrize("mode", ["fp64_refined", "fp64_direct", "mixed_refined"])
def test_diff_solve_matches_dense_adjoint(mode):
    p = diff_problem(64)
    op = Operator.uniform(p.points, p.h, a=p.a)
    u_o, L_o, ga_o, gf_o = dense_solve_loss_grad(op, p.f, p.u_target)
    prec = hif.HIF_FP32_MIXED if mode.startswith("mixed") else hif.HIF_FP64
    refine = mode.endswith("refined")
    eps = 1e-9 if mode == "fp64_direct" else 1e-6
    a = torch.tensor(p.a, requires_grad=True)  # host leaves: moved to the device differentiably
    f = torch.tensor(p.f, requires_grad=True)
    u = hif.diff.solve(torch.tensor(p.points), a, f, eps, 64, h=p.h, precision=prec, refine=refine, tol=1e-12)
    L = _loss(u, _t(p.u_target))
    L.backward()
    tol = 1e-9 if refine else 100 * eps
    assert _rel(_np(u), u_o) <= tol
    assert abs(L.item() - L_o) <= tol * L_o
    assert _rel(_np(a.grad), ga_o) <= tol, _rel(_np(a.grad), ga_o)
    assert _rel(_np(f.grad), gf_o) <= tol, _rel(_np(f.grad), gf_o)


def _setup256():
    p = diff_problem(256)
    return p, _t(p.points), _t(p.u_target)


@pytest.mark.parametrize("precision", [0, 1])
def test_diff_solve_256_central_differences(precision):
    # dL/da and dL/df of the refined map (GMRES to 1e-12 in both directions)
    # against central differences along 16 random directions of a and 4 of
    # f, to 1e-6 relative.  Central differences at steps d and d/2 are
    # combined by Richardson extrapolation, (4 D(d/2) - D(d)) / 3, which
    # removes the d^2 term of the truncation error; the solve tolerance
    # contributes about 1e-12 |L| / d.
    prec = hif.HIF_FP32_MIXED if precision else hif.HIF_FP64
    p, P, t = _setup256()
    N = P.shape[0]
    a = _t(p.a, requires_grad=True)
    f = _t(p.f, requires_grad=True)
    kw = dict(h=p.h, precision=prec, refine=True, tol=1e-12)
    u = hif.diff.solve(P, a, f, 1e-6, 64, **kw)
    _loss(u, t).backward()
    ga, gf = a.grad.detach(), f.grad.detach()

    def L(av, fv):
        with torch.no_grad():
            return _loss(hif.diff.solve(P, av, fv, 1e-6, 64, **kw), t).item()

    def richardson(g, d):
        c1 = (g(d) - g(-d)) / (2 * d)
        c2 = (g(d / 2) - g(-d / 2)) / d
        return (4 * c2 - c1) / 3

    rng = np.random.default_rng(11)
    a0, f0 = a.detach(), f.detach()
    worst = 0.0
    for k in range(16):
        v = rng.standard_normal(N)
        v = _t(v / np.max(np.abs(v)))
        fd = richardson(lambda s: L(a0 + s * v, f0), 1e-2)
        ex = torch.dot(ga, v).item()
        worst = max(worst, abs(fd - ex) / abs(ex))
        assert abs(fd - ex) <= 1e-6 * abs(ex), (k, fd, ex)
    for k in range(4):
        w = _t(rng.standard_normal(N))
        # L is quadratic in f: the central difference is exact up to the solves
        fd = (L(a0, f0 + 1e-2 * w) - L(a0, f0 - 1e-2 * w)) / 2e-2
        ex = torch.dot(gf, w).item()
        worst = max(worst, abs(fd - ex) / abs(ex))
        assert abs(fd - ex) <= 1e-6 * abs(ex), (k, fd, ex)
    print(f"256^2 precision {precision}: worst relative difference to central differences {worst:.2e}")


def test_diff_solve_256_modes_agree():
    # Refined gradients are those of the exact map, whichever factorization
    # preconditions them; the direct FP64 gradient is that of F^{-1}.
    p, P, t = _setup256()
    grads = {}
    for name, prec, refine in [("fp64", hif.HIF_FP64, True), ("mixed", hif.HIF_FP32_MIXED, True),
                               ("direct", hif.HIF_FP64, False)]:
        a = _t(p.a, requires_grad=True)
        f = _t(p.f, requires_grad=True)
        u = hif.diff.solve(P, a, f, 1e-6, 64, h=p.h, precision=prec, refine=refine, tol=1e-12)
        _loss(u, t).backward()
        grads[name] = (_np(a.grad), _np(f.grad))
    for i in range(2):
        assert _rel(grads["mixed"][i], grads["fp64"][i]) <= 1e-9
        assert _rel(grads["direct"][i], grads["fp64"][i]) <= 1e-4
