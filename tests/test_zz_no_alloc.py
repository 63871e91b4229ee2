"""hif_solve_noalloc: the solve for callers that cannot allocate, against
hif_solve on the same handles (same kernels, same order: identical bits),
two calls in a row with the second on a smaller problem, plus the size limit
rejected on the host.  All through the C ABI."""
import numpy as np
import pytest
import torch

import paper_1307_2666_amd as hif
from workloads import grid_points, workload

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _factor(n, d, eps, seed):
    pts = grid_points(n, d)
    N = pts.shape[0]
    a = 1.0 + np.random.default_rng(seed).uniform(size=N)
    return hif.factor(torch.tensor(pts, device=DEV), eps, 64, a=torch.tensor(a, device=DEV), h=1.0 / n), N


def test_solve_noalloc_matches_solve_twice():
    cases = [(workload("sq512").n, 2, 1e-6, 8, 1), (48, 2, 1e-6, 3, 2)]  # second call: smaller input
    for n, d, eps, nrhs, seed in cases:
        F, N = _factor(n, d, eps, seed)
        f = torch.tensor(np.random.default_rng(seed + 10).standard_normal((nrhs, N)), device=DEV)
        ref = F.solve(f)
        out = torch.full_like(f, float("nan"))
        got = F.solve_noalloc(f, out)
        torch.cuda.synchronize()
        assert got.data_ptr() == out.data_ptr()
        assert torch.equal(got, ref), (n, nrhs, (got - ref).abs().max().item())
        F.free()


def test_solve_noalloc_in_place_and_3d():
    # in place (u == f) on a 3D problem whose top block takes the
    # many-workgroup solve
    F, N = _factor(32, 3, 1e-6, 3)
    assert F.stats()["top_size"] > 8192  # 2 |s_L| above the LDS capacity
    f = torch.tensor(np.random.default_rng(4).standard_normal((2, N)), device=DEV)
    ref = F.solve(f)
    u = f.clone()
    F.solve_noalloc(u, u)
    torch.cuda.synchronize()
    assert torch.equal(u, ref)
    F.free()


def test_solve_noalloc_rejects_sizes_beyond_the_scratch():
    # min(nrhs, 8) * n above the scratch: 768 x 768 with 8 right-hand sides
    F, N = _factor(768, 2, 1e-3, 5)
    assert 8 * N > hif.HIF_SOLVE_NOALLOC_MAX
    f = torch.zeros((8, N), dtype=torch.float64, device=DEV)
    out = torch.empty_like(f)
    with pytest.raises(hif.HifError) as e:
        F.solve_noalloc(f, out)
    assert e.value.status == hif.HIF_EINVAL and "scratch" in str(e.value)
    # fewer right-hand sides fit, and still match hif_solve
    g = torch.tensor(np.random.default_rng(6).standard_normal((2, N)), device=DEV)
    out2 = torch.empty_like(g)
    F.solve_noalloc(g, out2)
    assert torch.equal(out2, F.solve(g))
    F.free()
