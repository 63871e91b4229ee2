"""Per-step parity: HIP steps of the factorization fed the inputs the CPU
oracle produces for real sub-levels of a factorization (the oracle's
``trace`` hook hands out each group's intermediate quantities), compared with
what the oracle computed from the same inputs.  All through the C ABI.

* a1 partition: the oracle's active sets after elimination (upper levels),
  cells and edges / faces, against the oracle's assignment, bit for bit.
* a4 ID: every class of the oracle's compressed blocks Y_c (kernel + proxy
  rows + SCI entries, second-kind classes and tolerances) through
  hif_id_batched: rank within one of the oracle's, the same skeleton where
  the pivots are unique, the reconstruction bound of Section 2.2 and |T|
  bounded like the oracle's.
* a2 near field and a3 assembly: the library's copy of a sub-level as
  assembled (opts.trace_sublevel) against the oracle's, on the first three
  sub-levels of a factorization, where both start from the same state (the
  same active DOFs and SCI pattern): the groups and their near fields
  identical, the entries of Y_c and A_cc to 12 units of roundoff (the
  SCI entries, products of the previous eliminations, to 1e-12 of the
  block's SCI scale).
* a6 elimination: the oracle's transformed blocks [B_rr B_rs; B_sr B_ss]
  (Lemma 2.4) through hif_lu_batched (partial LU over the redundant part,
  Lemma 2.1): the Schur complement B_ss - B_sr B_rr^{-1} B_rs against the
  oracle's B_ss + dS to 1e-12, and P B_rr = L U.
"""
import numpy as np
import pytest
import torch

import paper_1307_2666_amd as hif
from oracle.factor import factorize
from oracle.kernels import Operator
from oracle.tree import CELL, EDGE, FACE, assign
from workloads import grid_points

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _trace(n, d, eps, leaf, a=1.0):
    pts = grid_points(n, d)
    op = Operator.uniform(pts, 1.0 / n, a=np.full(pts.shape[0], a))
    groups = []
    factorize(op, eps, leaf, trace=groups.append)
    return op, groups


@pytest.fixture(scope="module")
def trace2d():
    return _trace(32, 2, 1e-6, 16)


@pytest.fixture(scope="module")
def trace3d():
    return _trace(12, 3, 1e-6, 27)


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_step_partition_on_oracle_active_sets(which, trace2d, trace3d):
    op, groups = trace2d if which == "2d" else trace3d
    n = round(op.N ** (1 / op.d))
    seen = set()
    for g in groups:
        key = (g["level"], g["kind"])
        if key in seen:
            continue
        seen.add(key)
        active = np.zeros(op.N, dtype=bool)
        active[g["active"]] = True
        L = max(x["level"] for x in groups) + 1  # tree depth
        S = 2 ** (L - g["level"])
        want = assign(op.points, active, g["kind"], S)
        kid = {CELL: 0, FACE: 1, EDGE: 2}[g["kind"]]
        got = hif.partition(torch.tensor(op.points, device=DEV), torch.tensor(active.astype(np.uint8)), kid, S)
        got = got.cpu().numpy()
        assert np.all(got[~active] == -1)
        assert np.array_equal(got[active], want), key
    assert len(seen) >= 4


def _id_cases(groups, limit=400):
    cases = []
    for g in groups:
        for cols, tol in zip(g["classes"], g["tols"]):
            cases.append((np.ascontiguousarray(g["Y"][:, cols]), tol))
        if len(cases) >= limit:
            break
    return cases


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_step_id_on_oracle_blocks(which, trace2d, trace3d):
    from oracle.idqr import interp_decomp

    _, groups = trace2d if which == "2d" else trace3d
    cases = _id_cases(groups)
    out = hif.id_batched([torch.tensor(Y) for Y, _ in cases], [t for _, t in cases])
    same = 0
    for (Y, tol), (sk, rd, T) in zip(cases, out):
        sk, rd, T = sk.numpy(), rd.numpy(), T.numpy()
        osk, ord_, oT = interp_decomp(Y, tol)
        assert abs(sk.size - osk.size) <= 1, (Y.shape, sk.size, osk.size)
        assert np.array_equal(np.sort(np.concatenate([sk, rd])), np.arange(Y.shape[1]))
        r00 = np.max(np.linalg.norm(Y, axis=0))
        if rd.size:
            err = np.linalg.norm(Y[:, rd] - Y[:, sk] @ T)
            assert err <= np.sqrt(rd.size) * tol * r00 * 1.01 + 1e-14 * r00
        # the interpolation matrix stays as well scaled as the oracle's
        tmax = np.abs(T).max() if T.size else 0.0
        otmax = np.abs(oT).max() if oT.size else 0.0
        assert tmax <= max(2.0, 4.0 * otmax), (tmax, otmax)
        if sk.size == osk.size and np.array_equal(np.sort(sk), np.sort(osk)):
            same += 1
    # ties in the pivot order are rare: nearly every class has the oracle's skeleton
    assert same >= 0.9 * len(cases), (same, len(cases))


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_step_elimination_schur_on_oracle_blocks(which, trace2d, trace3d):
    _, groups = trace2d if which == "2d" else trace3d
    blocks = [g for g in groups if "dS" in g and g["sk"].size > 0][:300]
    mats, rs = [], []
    for g in blocks:
        M = np.block([[g["Brr"], g["Brs"]], [g["Bsr"], g["Bss"]]])
        mats.append(torch.tensor(M))
        rs.append(g["rd"].size)
    out, piv, zero = hif.lu_batched(mats, rs)
    assert not zero
    for g, M, p in zip(blocks, out, piv):
        M = M.numpy()
        r = g["rd"].size
        want = g["Bss"] + g["dS"]
        scale = max(np.abs(g["Bss"]).max(), np.abs(g["dS"]).max())
        assert np.abs(M[r:, r:] - want).max() <= 1e-12 * scale
        # P B_rr = L U with the interchanges applied in order
        P = np.arange(r)
        for j, pj in enumerate(p.numpy()):
            P[[j, pj]] = P[[pj, j]]
        Lm = np.tril(M[:r, :r], -1) + np.eye(r)
        Um = np.triu(M[:r, :r])
        assert np.abs(g["Brr"][P] - Lm @ Um).max() <= 1e-12 * np.abs(g["Brr"]).max()
    assert len(blocks) >= (20 if which == "2d" else 5)


def test_lu_batched_mixed_sizes_and_tuning_tables():
    # Every launch shape of the tuning table gives the same factorization
    # (the panel threads only change the schedule), and the table round-trips.
    rng = np.random.default_rng(61)
    mats, rs = [], []
    for n in (40, 300, 700, 1000):
        A = rng.standard_normal((n, n)) + n * np.eye(n)
        mats.append(torch.tensor(A))
        rs.append(n // 2 + 3)
    base = hif.tuning_get()
    try:
        results = []
        for th in ((256, 512), (512, 1024), (1024, 1024)):
            hif.tuning_set(dict(base, lu_panel_threads=list(th)))
            assert hif.tuning_get()["lu_panel_threads"] == list(th)
            results.append(hif.lu_batched(mats, rs))
        for out, piv, zero in results:
            assert not zero
            for M0, M1 in zip(results[0][0], out):
                assert torch.equal(M0, M1)
        # Schur complement of the largest block against numpy
        A = mats[3].numpy()
        r = rs[3]
        S = A[r:, r:] - A[r:, :r] @ np.linalg.solve(A[:r, :r], A[:r, r:])
        assert np.abs(results[0][0][3].numpy()[r:, r:] - S).max() <= 1e-11 * np.abs(S).max()
        with pytest.raises(hif.HifError):
            hif.tuning_set(dict(base, lu_panel_threads=[128, 512]))
        assert hif.tuning_get()["lu_panel_threads"] == [1024, 1024]
    finally:
        hif.tuning_set(None)
    assert hif.tuning_get() == base


def test_id_reg_shapes_agree():
    # The register-resident ID with every allowed waves-per-problem gives the
    # same skeletons and interpolation matrices.
    rng = np.random.default_rng(62)
    cases = []
    for n in (50, 64, 100, 128, 170, 192):
        for _ in range(8):
            Y = np.triu(rng.standard_normal((n, n))) * (1.1 ** -np.arange(n))[rng.permutation(n)]
            cases.append(Y)
    base = hif.tuning_get()
    try:
        outs = []
        for w in ((4, 4, 8), (8, 8, 16), (16, 16, 16)):
            hif.tuning_set(dict(base, id_reg_waves=list(w)))
            outs.append(hif.id_batched([torch.tensor(Y) for Y in cases], [1e-8] * len(cases)))
        for out in outs[1:]:
            for (sk0, rd0, T0), (sk1, rd1, T1) in zip(outs[0], out):
                assert torch.equal(sk0, sk1) and torch.equal(rd0, rd1)
                assert torch.allclose(T0, T1, rtol=1e-10, atol=1e-12)
    finally:
        hif.tuning_set(None)


@pytest.mark.parametrize("si", [0, 1, 2])
def test_step_nearfield_and_assembly_on_first_sublevels(si, trace2d):
    # sub-level 0 (level-0 cells): no SCIs yet, every DOF active; sub-level 1
    # (level-0 edges): the SCIs of the cell eliminations, on the skeletons
    # both implementations chose; sub-level 2 (level-1 cells): the same state,
    # since on this grid the level-0 edges keep every DOF, now with blocks
    # A_cc that carry SCI entries
    op, groups = trace2d
    n = round(op.N ** 0.5)
    level, kind = si // 2, (CELL if si % 2 == 0 else EDGE)
    og = [g for g in groups if g["level"] == level and g["kind"] == kind]
    F = hif.factor(torch.tensor(op.points, device=DEV), 1e-6, 16, a=torch.tensor(op.a, device=DEV), h=1.0 / n,
                   trace_sublevel=si)
    tr = F.trace()
    gs, ns = tr["group_start"], tr["near_start"]
    G = gs.size - 1
    gpu = {}
    for g in range(G):
        dofs = tr["group_dofs"][gs[g]:gs[g + 1]]
        gpu[tuple(np.sort(dofs))] = g
    if si >= 1:
        # the same skeletons at level 0 give the same active set here
        act_gpu = np.sort(tr["group_dofs"])
        assert np.array_equal(act_gpu, np.sort(og[0]["active"]))
    assert len(gpu) == len(og)
    # Kernel part: each side evaluates an entry as the log of a rounded
    # distance times up to four rounded factors (Green's constant, quadrature
    # weight, b_i, c_j); the oracle takes log r, the library log r^2 / 2.
    # Either is within 6u of the exact entry relative to |Y| + h^2 / (2 pi)
    # (the floor where log r is near zero), so the two differ by at most 12u
    # of that.  SCI part (sub-level 1): the Schur updates of the level-0 cell
    # eliminations, linear in each side's own interpolation matrices T =
    # R11^{-1} R12, whose relative difference is bounded by cond(R11) u, and
    # cond(R11) <= about 1/eps by the rank rule; with a factor 100 for the
    # growth in the products the SCI entries agree to 100 u / eps of the
    # block's largest SCI entry.
    u = 2.0 ** -53
    eps = 1e-6
    h2pi = (1.0 / n) ** 2 / (2 * np.pi)
    nacc = 0
    worst_sci = 0.0
    for o in og:
        g = gpu[tuple(np.sort(o["c"]))]
        dofs = tr["group_dofs"][gs[g]:gs[g + 1]]
        near = tr["near_dofs"][ns[g]:ns[g + 1]]
        assert np.array_equal(near, o["near"]), (si, g)
        pos = {int(d): i for i, d in enumerate(o["c"])}
        cols = np.array([pos[int(d)] for d in dofs])
        m, nc = o["Y"].shape
        Y = tr["Y"][tr["y_off"][g]:tr["y_off"][g] + m * nc].reshape(m, nc)
        Yo = o["Y"][:, cols]
        Ko = Yo.copy()
        Ko[:near.size] = op.kernel_block(near, dofs)  # proxy rows hold no SCI entries
        So = Yo - Ko
        if si == 0:
            assert not So.any()
        tol = 12 * u * (np.abs(Ko) + h2pi) + 100 * u / eps * np.abs(So).max()
        assert np.all(np.abs(Y - Yo) <= tol), (si, g, np.abs(Y - Yo).max())
        if So.any():
            worst_sci = max(worst_sci, np.abs(Y - Yo).max() / np.abs(So).max())
        if "Acc" in o:
            A = tr["Acc"][tr["acc_off"][g]:tr["acc_off"][g] + nc * nc].reshape(nc, nc)
            Ao = o["Acc"][np.ix_(cols, cols)]
            Bo = op.block(dofs, dofs)
            Sc = Ao - Bo
            tol = 12 * u * (np.abs(Bo) + h2pi) + 100 * u / eps * np.abs(Sc).max()
            assert np.all(np.abs(A - Ao) <= tol), (si, g, np.abs(A - Ao).max())
            nacc += 1
    print(f"sub-level {si}: {len(og)} groups, largest difference / largest SCI entry {worst_sci:.2e}")
    # the level-0 edges of this grid eliminate nothing: no A_cc to compare there
    assert nacc > 0 or si == 1
    F.free()


def test_sweep_and_rowqr_shapes_agree():
    # The sweep's threads per record (sub-levels of >= 1024 records) change
    # which wave handles which row, and the transposed products sum their
    # rows in as many slices as the shape has waves (up to 4): the solves
    # agree to rounding (each shape is deterministic on its own).
    # The row compression's update shapes sum the same products in other
    # orders: rank decisions at the threshold may differ in a few classes
    # (ranks are not unique), so the factorizations agree to a tenth of eps,
    # as GPU and oracle factors do, with top blocks within 1%.
    n = 256
    pts = torch.tensor(grid_points(n, 2), device=DEV)
    a = torch.ones(n * n, dtype=torch.float64, device=DEV)
    f = torch.randn(8, n * n, dtype=torch.float64, device=DEV, generator=torch.Generator(DEV).manual_seed(5))
    base = hif.tuning_get()
    try:
        F = hif.factor(pts, 1e-6, 64, a=a, h=1.0 / n)
        assert F.stats()["sub_groups"][0] >= 1024
        sols = []
        for th in (64, 128, 256):
            hif.tuning_set(dict(base, sweep_many_threads=th))
            sols.append(F.solve(f))
        for u in sols[1:]:
            assert (u - sols[0]).abs().max().item() <= 1e-13 * sols[0].abs().max().item()
        F.free()
        outs = []
        for w, kind in ((4, 0), (8, 1), (8, 2)):
            hif.tuning_set(dict(base, rowqr_update_waves=w, rowqr_update_kind=kind))
            G = hif.factor(pts, 1e-6, 64, a=a, h=1.0 / n)
            outs.append((G.stats()["top_size"], G.apply(f[0])))
            G.free()
        for top, y in outs[1:]:
            assert abs(top - outs[0][0]) <= 0.01 * outs[0][0] + 2
            assert torch.linalg.norm(y - outs[0][1]) <= 1e-7 * torch.linalg.norm(outs[0][1])
        with pytest.raises(hif.HifError):
            hif.tuning_set(dict(base, sweep_many_threads=96))
    finally:
        hif.tuning_set(None)
