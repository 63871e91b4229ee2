"""Tree, level partitions and proxy surfaces (oracle; test infrastructure only).

* Tree: the adaptive quadtree / octree of Section 3.1 (Algorithm 3.1's remark
  on adaptive trees), splitting a box while it holds more than ``leaf``
  points.  Only trees whose leaves all sit at one depth ``L`` are handled
  (true for the uniform grids used throughout Section 5).
* Partitions: at level ``l`` the cells have width ``w = 2^l / 2^L`` (the
  ``2^l m h`` of Section 3.1).  Algorithm 4.1 (2D) follows each cell level
  by an edge level; Algorithm 4.2 (3D) by a face level and an edge level.
  The face and edge centres are the interior ones enumerated in Section 4.1
  (edges) and Section 4.2 (faces, then edges), family by family in the order
  the paper lists them, each family with its first index slowest.  Cells use
  the containing box; faces and edges the nearest centre, exact ties going
  to the lowest centre index.
* Proxy surface (Section 3.3): a circle / sphere of radius ``1.5 w`` about the
  group centre with 64 / 512 points.  The paper draws the 3D points by
  normalizing Gaussian vectors; this oracle takes the deterministic
  spherical Fibonacci set instead (a documented reading).
"""
from __future__ import annotations

import itertools

import numpy as np

# Sub-level kinds: number of integer (interface) coordinates of the centres.
CELL, FACE, EDGE = "cell", "face", "edge"


def box_index(points: np.ndarray, S: int) -> np.ndarray:
    """Per-dimension index ``floor(x * S)`` of the box containing each point, clamped to ``[0, S-1]``."""
    j = np.floor(points * S).astype(np.int64)
    return np.clip(j, 0, S - 1)


def flat_box(jj: np.ndarray, S: int) -> np.ndarray:
    """Flatten per-dimension box indices with the first coordinate slowest."""
    d = jj.shape[1]
    out = np.zeros(jj.shape[0], dtype=np.int64)
    for k in range(d):
        out = out * S + jj[:, k]
    return out


def tree_depth(points: np.ndarray, leaf: int) -> int:
    """Depth ``L`` of the adaptive tree over ``[0,1]^d`` that splits boxes holding more than ``leaf`` points.

    Raises ``ValueError`` when the leaves would not all sit at one depth.
    """
    N, d = points.shape
    L = 0
    while True:
        S = 2 ** L
        counts = np.bincount(flat_box(box_index(points, S), S), minlength=S ** d)
        if counts.max() <= leaf:
            break
        L += 1
        if L > 30:
            raise ValueError("tree too deep (coincident points?)")
    if L > 0:
        S = 2 ** (L - 1)
        counts = np.bincount(flat_box(box_index(points, S), S), minlength=S ** d)
        if counts.min() <= leaf:
            raise ValueError("adaptive tree is not uniform in depth")
    return L


def sublevel_kinds(d: int, variant: str = "hifie") -> tuple:
    """Sub-levels per level: Algorithm 3.1 (cells) or Algorithm 4.1 / 4.2 (cells, [faces,] edges)."""
    if variant == "rskel":
        return (CELL,)
    return (CELL, EDGE) if d == 2 else (CELL, FACE, EDGE)


def _families(kind: str, d: int) -> list:
    """Integer-coordinate sets of each centre family, in the order the paper lists them."""
    if kind == CELL:
        return [()]
    if kind == FACE:
        return [(0,), (1,), (2,)]
    if d == 2:
        return [(0,), (1,)]
    return [(0, 1), (0, 2), (1, 2)]


def centres(kind: str, d: int, S: int) -> np.ndarray:
    """Centres of the level's cells (S^d), interior faces or interior edges, in enumeration order.

    A coordinate that is "integer" takes the interior values ``j w`` for
    ``j = 1..S-1``; the others take ``(j + 1/2) w`` for ``j = 0..S-1``.
    """
    w = 1.0 / S
    out = []
    for fam in _families(kind, d):
        axes = []
        for k in range(d):
            if k in fam:
                axes.append(np.arange(1, S, dtype=np.float64) * w)
            else:
                axes.append((np.arange(S, dtype=np.float64) + 0.5) * w)
        grid = np.meshgrid(*axes, indexing="ij")
        out.append(np.stack([g.ravel() for g in grid], axis=1))
    return np.concatenate(out, axis=0) if out else np.zeros((0, d))


def assign(points: np.ndarray, active: np.ndarray, kind: str, S: int,
           chunk: int = 1 << 22) -> np.ndarray:
    """Centre index of every active point (Voronoi partition of Sections 3.1, 4.1, 4.2).

    Cells: the containing box.  Faces / edges: the nearest centre by squared
    distance ``sum_k (x_k - z_k)^2`` (summed in coordinate order), exact ties
    to the lowest centre index; brute force over all centres.
    """
    d = points.shape[1]
    act = np.nonzero(active)[0]
    if kind == CELL:
        return flat_box(box_index(points[act], S), S)
    Z = centres(kind, d, S)
    out = np.empty(act.size, dtype=np.int64)
    step = max(1, chunk // max(1, Z.shape[0]))
    for s in range(0, act.size, step):
        P = points[act[s:s + step]]
        d2 = np.zeros((P.shape[0], Z.shape[0]))
        for k in range(d):
            t = P[:, k][:, None] - Z[:, k][None, :]
            d2 += t * t
        out[s:s + step] = np.argmin(d2, axis=1)
    return out


def proxy_directions(d: int, n_proxy: int) -> np.ndarray:
    """Unit vectors of the proxy surface (Section 3.3).

    2D: ``(cos t_p, sin t_p)``, ``t_p = 2 pi p / P``.
    3D: spherical Fibonacci set ``z_p = 1 - (2p+1)/P``, ``phi_p = p pi (3 - sqrt 5)``.
    """
    p = np.arange(n_proxy, dtype=np.float64)
    if d == 2:
        t = 2.0 * np.pi * p / n_proxy
        return np.stack([np.cos(t), np.sin(t)], axis=1)
    z = 1.0 - (2.0 * p + 1.0) / n_proxy
    rho = np.sqrt(1.0 - z * z)
    phi = p * np.pi * (3.0 - np.sqrt(5.0))
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def default_proxy_count(d: int) -> int:
    """64 points on the circle, 512 on the sphere (Section 3.3)."""
    return 64 if d == 2 else 512


def all_box_ids(d: int, S: int) -> np.ndarray:
    return np.array(list(itertools.product(range(S), repeat=d)), dtype=np.int64)
