"""Pins of the oracle's tree, partitions and proxy surfaces (CPU)."""
import numpy as np
import pytest

from oracle.idqr import interp_decomp
from oracle.kernels import green
from oracle.tree import (CELL, EDGE, FACE, assign, centres, proxy_directions,
                         sublevel_kinds, tree_depth)
from workloads import grid_points


@pytest.mark.parametrize("n,d,leaf,L", [(64, 2, 64, 3), (512, 2, 64, 6), (32, 3, 64, 3),
                                        (64, 3, 64, 4), (96, 2, 64, 4), (192, 2, 64, 5),
                                        (8, 2, 64, 0), (16, 2, 4, 3)])
def test_tree_depth_uniform_grids(n, d, leaf, L):
    # n = 2^L m with leaf boxes of m^d <= leaf points (Section 3.1).
    assert tree_depth(grid_points(n, d), leaf) == L


def test_tree_depth_rejects_nonuniform():
    pts = np.vstack([grid_points(16, 2) * 0.5, np.array([[0.9, 0.9]])])
    with pytest.raises(ValueError):
        tree_depth(pts, 16)


@pytest.mark.parametrize("S", [1, 2, 4, 8])
def test_centre_counts_closed_form(S):
    # Index ranges of Sections 4.1 and 4.2: cells S^d, 2D edges 2S(S-1),
    # 3D faces 3S^2(S-1), 3D edges 3S(S-1)^2.
    assert centres(CELL, 2, S).shape == (S * S, 2)
    assert centres(EDGE, 2, S).shape == (2 * S * (S - 1), 2)
    assert centres(CELL, 3, S).shape == (S ** 3, 3)
    assert centres(FACE, 3, S).shape == (3 * S * S * (S - 1), 3)
    assert centres(EDGE, 3, S).shape == (3 * S * (S - 1) ** 2, 3)


def test_centre_enumeration_order_2d():
    # First family (j1 w, (j2 - 1/2) w), j1 slowest; then ((j1 - 1/2) w, j2 w).
    Z = centres(EDGE, 2, 2)
    assert np.allclose(Z, [[0.5, 0.25], [0.5, 0.75], [0.25, 0.5], [0.75, 0.5]])


def test_sublevel_kinds():
    assert sublevel_kinds(2) == (CELL, EDGE)
    assert sublevel_kinds(3) == (CELL, FACE, EDGE)
    assert sublevel_kinds(3, "rskel") == (CELL,)


def _brute_assign(points, Z):
    out = []
    for p in points:
        best, bi = None, -1
        for i, z in enumerate(Z):
            d2 = 0.0
            for k in range(len(p)):
                d2 += (p[k] - z[k]) * (p[k] - z[k])
            if best is None or d2 < best:
                best, bi = d2, i
        out.append(bi)
    return np.array(out)


@pytest.mark.parametrize("n,d,kind,S", [(16, 2, EDGE, 2), (16, 2, EDGE, 4), (8, 3, FACE, 2),
                                        (8, 3, EDGE, 2), (12, 2, EDGE, 2)])
def test_voronoi_assignment_brute_force(n, d, kind, S):
    pts = grid_points(n, d)
    rng = np.random.default_rng(3)
    active = rng.uniform(size=pts.shape[0]) < 0.6
    got = assign(pts, active, kind, S)
    want = _brute_assign(pts[active], centres(kind, d, S))
    assert np.array_equal(got, want)


def test_edge_ties_on_cell_diagonals():
    # An interior 8x8 cell has 16 points on its two diagonals, each equidistant
    # from two edge centres; the tie goes to the lower enumeration index.
    n, S = 32, 4
    pts = grid_points(n, 2)
    Z = centres(EDGE, 2, S)
    incell = np.all((pts > 0.25) & (pts < 0.5), axis=1)
    ties = 0
    for p in pts[incell]:
        d2 = np.sum((Z - p) ** 2, axis=1)
        ties += int(np.sum(d2 == d2.min()) > 1)
    assert incell.sum() == 64 and ties == 16
    # In the corner cell only the right and top edges are interior: its main
    # diagonal points are equidistant from the vertical centre (0.25, 0.125)
    # [index 0] and the horizontal centre (0.125, 0.25) [index 12]; index 0 wins.
    got = assign(pts, np.ones(n * n, bool), EDGE, S)
    diag = np.isclose(pts[:, 0], pts[:, 1]) & (pts[:, 0] < 0.25) & (pts[:, 0] > 0.125)
    assert diag.sum() == 4 and np.all(got[diag] == 0)
    assert np.allclose(Z[0], [0.25, 0.125]) and np.allclose(Z[12], [0.125, 0.25])


@pytest.mark.parametrize("d,P", [(2, 64), (3, 512)])
def test_proxy_directions_unit(d, P):
    U = proxy_directions(d, P)
    assert U.shape == (P, d)
    assert np.allclose(np.linalg.norm(U, axis=1), 1.0, atol=1e-15)
    assert np.allclose(U.mean(axis=0), 0.0, atol=2e-3)


@pytest.mark.parametrize("d,m,P,tol", [(2, 8, 64, 1e-10), (2, 8, 64, 1e-12), (3, 6, 512, 1e-12)])
def test_proxy_reproduces_far_field(d, m, P, tol):
    # Lemma 3.2 (Green's theorem): interactions of a box with every source
    # outside the proxy sphere of radius 1.5 (box width 1) lie in the row space
    # of the proxy interactions, so an ID of the proxy rows alone interpolates
    # the whole far field to the ID's tolerance.
    h = 1.0 / m
    ax = (np.arange(-3 * m, 4 * m) + 0.5) * h - 0.5
    grid = np.stack(np.meshgrid(*([ax] * d), indexing="ij"), -1).reshape(-1, d)
    inbox = np.all(np.abs(grid) < 0.5, axis=1)
    r = np.linalg.norm(grid, axis=1)
    box = grid[inbox]
    near = grid[~inbox & (r < 1.5)]
    far = grid[r >= 1.5]
    prox = 1.5 * proxy_directions(d, P)

    def K(X, Y):
        return green(np.linalg.norm(X[:, None, :] - Y[None, :, :], axis=2), d)

    W = K(far, box)
    sk, rd, T = interp_decomp(K(prox, box), tol)
    assert rd.size > 0
    assert np.linalg.norm(W[:, rd] - W[:, sk] @ T) <= 10 * tol * np.linalg.norm(W)
    # Lemma 3.1 with eqn (proxy-id): adding the near-field rows keeps this true.
    sk, rd, T = interp_decomp(np.vstack([K(near, box), K(prox, box)]), tol)
    if rd.size:
        assert np.linalg.norm(W[:, rd] - W[:, sk] @ T) <= 10 * tol * np.linalg.norm(W)
