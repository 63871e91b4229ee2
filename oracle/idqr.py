"""Interpolative decomposition by column-pivoted QR (oracle; test infrastructure only).

Lemma 2.2: with ``Y P = Q [R1 R2]`` a column-pivoted QR, the first ``k`` pivots
are the skeleton columns, the rest the redundant ones, and ``T = R1^{-1} R2``
gives ``Y[:, redundant] ~= Y[:, skeleton] T``.  Section 2.2 picks ``k``
adaptively from the relative magnitudes of the pivots; reading used here:
pivot ``i`` is kept iff ``|R_ii| > tol * |R_00|``, stopping at the first pivot
that fails.  The pivoted QR itself is LAPACK's (``dgeqp3`` through
``scipy.linalg.qr(pivoting=True)``), the routine the proof of Lemma 2.2
describes.  The redundant columns are returned in ascending original order,
the skeleton columns in pivot order.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
from scipy.linalg import solve_triangular


def interp_decomp(Y: np.ndarray, tol: float):
    """ID of ``Y`` (m x n) at relative tolerance ``tol``.

    Returns ``(sk, rd, T)``: skeleton column indices (pivot order), redundant
    column indices (ascending) and ``T`` (``len(sk) x len(rd)``).
    """
    Y = np.asarray(Y, dtype=np.float64)
    m, n = Y.shape
    if m == 0 or n == 0:
        return np.zeros(0, np.int64), np.arange(n), np.zeros((0, n))
    R, perm = scipy.linalg.qr(Y, mode="r", pivoting=True)
    diag = np.abs(np.diag(R))
    k = 0
    if diag.size and diag[0] > 0.0:
        thr = tol * diag[0]
        fail = np.nonzero(~(diag > thr))[0]
        k = int(fail[0]) if fail.size else diag.size
    sk = perm[:k].astype(np.int64)
    rd = perm[k:].astype(np.int64)
    if k > 0 and rd.size > 0:
        T = solve_triangular(R[:k, :k], R[:k, k:], lower=False)
    else:
        T = np.zeros((k, rd.size))
    srt = np.argsort(rd, kind="stable")
    return sk, rd[srt], T[:, srt]
