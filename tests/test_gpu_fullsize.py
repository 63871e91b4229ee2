"""GPU parity at the full sizes of the workloads, through the C ABI, checked
against the CPU oracle's own arithmetic (never against another HIP result):

* Sampled rows of the exact operator.  At N = 262144 no dense A exists, so
  the oracle evaluates chosen rows of ``A x`` one by one
  (``Operator.matvec(rows=...)``, plain NumPy); the factorization's apply
  error ``|(F x - A x)_rows| / |(A x)_rows|`` and the solve residual
  ``|(f - A F^{-1} f)_rows| / |f_rows|`` are taken on those rows.
* The paper's own accuracy measures (Section 5, Tables 4 and 13):
  ``e_a ~ |A - F| / |A|`` and ``e_s ~ |I - A F^{-1}|`` by the oracle's power
  iteration (``oracle.estimators``), driven through hif_apply, hif_apply_T,
  hif_solve, hif_solve_T and the exact pair-by-pair operator.
* The 2-norm ``|A - F|_2 / |A|_2`` with a dense F at 64 x 64.
* Configurations not covered elsewhere: 512 x 512 at eps = 1e-9, 64^3 in
  FP64, 32^3 in FP32-mixed mode refined by GMRES.
* Degenerate cases: a leaf holding every point (no levels: F is the dense LU
  of A) and a tree whose leaves sit at different depths (HIF_EUNSUPPORTED).

Every accuracy gate is 10 eps (eps the ID precision); next to it a
regression bound, about 20 times the error measured on MI355X, catches a
loss of accuracy that would still pass the gate.
"""
import numpy as np
import pytest
import torch
from scipy.sparse.linalg import svds

import paper_1307_2666_amd as hif
from oracle.estimators import e_apply, e_solve
from oracle.kernels import Operator
from workloads import grid_points, rhs, workload

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(x):
    return torch.tensor(np.ascontiguousarray(x), device=DEV)


def _np(t):
    return t.detach().cpu().numpy()


def _rows(N, count, seed):
    return np.sort(np.random.default_rng(seed).choice(N, count, replace=False))


def _row_errors(op, F, f, x, rows):
    """Apply error and solve residual of F on the given rows, the exact values from the oracle."""
    u = _np(F.solve(_t(f)))
    y = _np(F.apply(_t(x)))
    Au = op.matvec(u, rows=rows, chunk=32)
    Ax = op.matvec(x, rows=rows, chunk=32)
    fr = f[..., rows]
    res = np.linalg.norm(fr - Au) / np.linalg.norm(fr)
    app = np.linalg.norm(y[..., rows] - Ax) / np.linalg.norm(Ax)
    return float(app), float(res)


def _factor_uniform(wl, eps=None, **kw):
    P = _t(wl.points())
    a = torch.ones(wl.N, dtype=torch.float64, device=DEV)
    return hif.factor(P, wl.eps if eps is None else eps, wl.leaf, a=a, h=wl.h, **kw), P, a


# ---------------------------------------------------------------------------
# measured 4.5e-10 / 5.0e-10 (eps 1e-6) and 2.7e-13 / 3.2e-13 (eps 1e-9)
_SQ512_REGRESSION = {1e-6: 1e-8, 1e-9: 1e-11}


@pytest.mark.parametrize("eps", [1e-6, 1e-9])
def test_sq512_sampled_oracle_rows(eps):
    # 512 x 512, 8 right-hand sides; 256 rows of A u and A x from the oracle.
    wl = workload("sq512")
    op = Operator.uniform(wl.points(), wl.h, a=np.ones(wl.N))
    F, P, a = _factor_uniform(wl, eps)
    f = wl.rhs()
    x = np.random.default_rng(31).standard_normal((2, wl.N))
    rows = _rows(wl.N, 256, 32)
    app, res = _row_errors(op, F, f, x, rows)
    print(f"sq512 eps={eps:g}: apply error {app:.2e}, solve residual {res:.2e} on {rows.size} oracle rows")
    assert app <= 10 * eps and res <= 10 * eps, (app, res)
    assert app <= _SQ512_REGRESSION[eps] and res <= _SQ512_REGRESSION[eps], (app, res)  # regression bound
    # the same residual over all N rows through the pair-by-pair operator
    U = F.solve(_t(f))
    R = _t(f) - hif.matvec(P, U, a=a, h=wl.h)
    full = (torch.linalg.norm(R, dim=1) / torch.linalg.norm(_t(f), dim=1)).max().item()
    assert full <= 10 * eps, full
    F.free()


def test_power_iteration_errors_sq512():
    # e_a and e_s of Section 5 for the 512 x 512 factorization at eps 1e-6
    # (the paper's hifie2x row of Table 4 gives 5.9e-7 and 6.7e-7 with its
    # adaptive leaves).
    wl = workload("sq512")
    F, P, a = _factor_uniform(wl)
    A = lambda v: _np(F.apply_A(_t(v))[0])
    AT = lambda v: _np(F.apply_A(_t(v), transpose=True)[0])

    class _F:
        apply = staticmethod(lambda v: _np(F.apply(_t(v))))
        apply_T = staticmethod(lambda v: _np(F.apply_T(_t(v))))
        solve = staticmethod(lambda v: _np(F.solve(_t(v))))
        solve_T = staticmethod(lambda v: _np(F.solve_T(_t(v))))

    ea = e_apply(A, AT, _F, wl.N, seed=1)
    es = e_solve(A, AT, _F, wl.N, seed=2)
    print(f"sq512 eps=1e-6: e_a {ea:.2e}, e_s {es:.2e}")
    assert ea <= 10 * wl.eps and es <= 10 * wl.eps, (ea, es)
    assert ea <= 1.5e-6 and es <= 1.5e-6, (ea, es)  # regression bound (measured 6.6e-8, 7.2e-8)
    F.free()


def test_power_iteration_errors_cube32():
    # e_a and e_s for 32^3 at eps 1e-6 (Table 13, hifie3x: 2.9e-7 and 3.4e-7)
    wl = workload("cube32")
    F, P, a = _factor_uniform(wl)
    A = lambda v: _np(F.apply_A(_t(v))[0])
    AT = lambda v: _np(F.apply_A(_t(v), transpose=True)[0])

    class _F:
        apply = staticmethod(lambda v: _np(F.apply(_t(v))))
        apply_T = staticmethod(lambda v: _np(F.apply_T(_t(v))))
        solve = staticmethod(lambda v: _np(F.solve(_t(v))))
        solve_T = staticmethod(lambda v: _np(F.solve_T(_t(v))))

    ea = e_apply(A, AT, _F, wl.N, seed=3)
    es = e_solve(A, AT, _F, wl.N, seed=4)
    print(f"cube32 eps=1e-6: e_a {ea:.2e}, e_s {es:.2e}")
    assert ea <= 10 * wl.eps and es <= 10 * wl.eps, (ea, es)
    assert ea <= 5e-7 and es <= 5e-7, (ea, es)  # regression bound (measured 2.3e-8, 2.6e-8)
    F.free()


def test_sq64_dense_two_norm():
    # |A - F|_2 / |A|_2 <= 10 eps with F materialized column by column on the
    # 64 x 64 workload (N = 4096); A from the oracle.
    wl = workload("sq64")
    op = Operator.uniform(wl.points(), wl.h, a=np.ones(wl.N))
    F, P, a = _factor_uniform(wl)
    I = torch.eye(wl.N, dtype=torch.float64, device=DEV)
    Fd = _np(F.apply(I)).T
    A = op.dense()
    D = A - Fd
    nD = svds(D, k=1, tol=1e-10, return_singular_vectors=False, random_state=0)[0]
    nA = svds(A, k=1, tol=1e-10, return_singular_vectors=False, random_state=0)[0]
    print(f"sq64: |A - F|_2 / |A|_2 = {nD / nA:.2e}")
    assert nD <= 10 * wl.eps * nA, nD / nA
    assert nD <= 3e-7 * nA, nD / nA  # regression bound (measured 1.6e-8)
    F.free()


def test_cube64_full_size_fp64():
    # 64^3 (N = 262144), eps 1e-6, FP64 with the second-kind modification;
    # 256 oracle rows of A u and A x.
    wl = workload("cube64")
    op = Operator.uniform(wl.points(), wl.h, a=np.ones(wl.N))
    F, P, a = _factor_uniform(wl)
    st = F.stats()
    f = wl.rhs()
    x = np.random.default_rng(33).standard_normal(wl.N)
    rows = _rows(wl.N, 256, 34)
    app, res = _row_errors(op, F, f[0], x, rows)
    print(f"cube64: |s_L| {st['top_size']}, m_f {st['factor_bytes'] / 1e9:.1f} GB, apply error {app:.2e}, "
          f"solve residual {res:.2e}")
    assert st["levels"] == 4 and st["n_sublevels"] == 12
    assert app <= 10 * wl.eps and res <= 10 * wl.eps, (app, res)
    assert app <= 2e-8 and res <= 2e-8, (app, res)  # regression bound (measured 1.0e-9, 9.3e-10)
    F.free()


def test_cube32_mixed_refined():
    # 32^3 in FP32-mixed mode (FP32 kernel entries and matrix-core GEMMs,
    # plain compression), as a preconditioner: GMRES against the exact FP64
    # operator reaches a true residual of 1e-10, checked on oracle rows; the
    # unrefined mixed solve is accurate to about single precision.
    wl = workload("cube32")
    op = Operator.uniform(wl.points(), wl.h, a=np.ones(wl.N))
    F, P, a = _factor_uniform(wl, precision=hif.HIF_FP32_MIXED)
    f = wl.rhs()
    rows = _rows(wl.N, 256, 35)
    u0 = _np(F.solve(_t(f[0])))
    r0 = np.linalg.norm(f[0][rows] - op.matvec(u0, rows=rows, chunk=32)) / np.linalg.norm(f[0][rows])
    u, its, rr = F.gmres(_t(f), tol=1e-10, maxit=30)
    u = _np(u)[0]
    r1 = np.linalg.norm(f[0][rows] - op.matvec(u, rows=rows, chunk=32)) / np.linalg.norm(f[0][rows])
    print(f"cube32 mixed: unrefined residual {r0:.2e}, GMRES {its[0]} iterations, residual {rr[0]:.2e} "
          f"(oracle rows {r1:.2e})")
    assert 1e-9 < r0 <= 1e-4, r0
    assert rr[0] <= 1.5e-10 and r1 <= 1.5e-10, (rr, r1)
    assert its[0] <= 8
    F.free()


# ---------------------------------------------------------------------------
def test_leaf_holds_every_point():
    # leaf >= N: no levels, F is the dense LU of A (top block = all points)
    n = 24
    pts = grid_points(n, 2)
    N = pts.shape[0]
    rng = np.random.default_rng(36)
    a = 1.0 + rng.uniform(size=N)
    op = Operator.uniform(pts, 1.0 / n, a=a)
    F = hif.factor(_t(pts), 1e-6, N, a=_t(a), h=1.0 / n)
    st = F.stats()
    assert st["levels"] == 0 and st["n_sublevels"] == 0 and st["top_size"] == N
    A = op.dense()
    f = rng.standard_normal((3, N))
    u = _np(F.solve(_t(f)))
    ref = np.linalg.solve(A, f.T).T
    assert np.linalg.norm(u - ref) <= 1e-13 * np.linalg.norm(ref)
    y = _np(F.apply(_t(f)))
    assert np.linalg.norm(y - f @ A.T) <= 1e-14 * np.linalg.norm(f @ A.T)
    F.free()


def test_non_uniform_depth_is_unsupported():
    # 256 points packed into the lower-left quarter and 12 spread over the
    # rest: leaves of 16 points sit at depth 3 in the packed quarter and at
    # depth 1 elsewhere, which the uniform-depth levels do not handle.
    dense = grid_points(16, 2) * 0.5
    sparse = np.array([[0.5 + 0.5 * (i + 0.5) / 4, 0.5 * (j + 0.5) / 3 + 0.5 * (j % 2)] for i in range(4)
                       for j in range(3)])
    pts = np.vstack([dense, sparse])
    with pytest.raises(hif.HifError) as e:
        hif.factor(_t(pts), 1e-6, 16, h=1.0 / 32)
    assert e.value.status == hif.HIF_EUNSUPPORTED
