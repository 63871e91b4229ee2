"""Pins of the oracle's interpolative decomposition (Lemma 2.2, Corollary 2.3, Section 2.2)."""
import numpy as np
import pytest

from oracle.idqr import interp_decomp


@pytest.mark.parametrize("m,n,k", [(40, 30, 7), (30, 40, 12), (100, 64, 64), (64, 64, 1)])
def test_exact_low_rank_is_reproduced(m, n, k):
    # Lemma 2.2: a rank-k matrix has an exact ID with k skeleton columns.
    rng = np.random.default_rng(m + n + k)
    Y = rng.standard_normal((m, k)) @ rng.standard_normal((k, n))
    sk, rd, T = interp_decomp(Y, 1e-12)
    assert sk.size == k and rd.size == n - k
    assert np.array_equal(np.sort(np.concatenate([sk, rd])), np.arange(n))
    assert np.all(np.diff(rd) > 0)
    # Corollary 2.3: [Y_rd Y_sk] [I; -T I] = [0 Y_sk].
    assert np.linalg.norm(Y[:, rd] - Y[:, sk] @ T) <= 1e-12 * np.linalg.norm(Y)


def test_recovers_generating_coefficients():
    # Redundant columns built as known combinations of skeleton columns.
    rng = np.random.default_rng(5)
    B = rng.standard_normal((50, 6)) * np.array([10.0, 8, 6, 4, 2, 1])
    C = 0.05 * rng.standard_normal((6, 9))   # redundant columns smaller than every generator
    Y = np.hstack([B, B @ C])
    sk, rd, T = interp_decomp(Y, 1e-13)
    assert np.array_equal(np.sort(sk), np.arange(6))
    # T in terms of the skeleton order equals C permuted accordingly.
    inv = np.argsort(sk)
    assert np.allclose(T[inv], C, atol=1e-11)


def _greedy_pivots(Y, tol):
    """Businger-Golub pivoting from its definition: repeatedly take the column
    with the largest residual after projecting out the columns taken so far
    (Gram-Schmidt, twice for stability); stop when that residual is <= tol
    times the first one."""
    Y = np.array(Y, dtype=float)
    m, n = Y.shape
    Q = np.zeros((m, 0))
    piv, res0 = [], None
    for _ in range(min(m, n)):
        Rres = Y - Q @ (Q.T @ Y)
        Rres = Rres - Q @ (Q.T @ Rres)
        norms = np.linalg.norm(Rres, axis=0)
        norms[piv] = -1.0
        j = int(np.argmax(norms))
        if res0 is None:
            res0 = norms[j]
        if not norms[j] > tol * res0:
            break
        piv.append(j)
        Q = np.hstack([Q, (Rres[:, j] / norms[j])[:, None]])
    return np.array(piv)


def test_pivots_match_greedy_definition():
    # Lemma 2.2's pivoted QR chooses, at each step, the column of largest norm
    # orthogonal to the skeleton chosen so far; with well-separated norms the
    # sequence is unique.
    rng = np.random.default_rng(7)
    m, n = 60, 25
    Y = rng.standard_normal((m, n)) * (2.0 ** -np.arange(n))[rng.permutation(n)]
    want = _greedy_pivots(Y, 1e-6)
    sk, rd, T = interp_decomp(Y, 1e-6)
    assert sk.size == want.size
    assert np.array_equal(sk, want)


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-9])
def test_error_bound_from_trailing_norms(tol):
    # Stopping when the largest trailing column norm is <= tol |R_00| bounds the
    # interpolation error by sqrt(r) tol |R_00| (every column of R_22 is below it).
    rng = np.random.default_rng(11)
    m, n = 80, 50
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = 10.0 ** -np.linspace(0, 12, n)
    Y = (U * s) @ V.T
    sk, rd, T = interp_decomp(Y, tol)
    r00 = np.max(np.linalg.norm(Y, axis=0))
    err = np.linalg.norm(Y[:, rd] - Y[:, sk] @ T)
    assert err <= np.sqrt(rd.size) * tol * r00 * (1 + 1e-8)
    # and it is a rank-revealing cut: one fewer pivot would violate the bound.
    assert 0 < sk.size < n


def test_zero_matrix_has_rank_zero():
    sk, rd, T = interp_decomp(np.zeros((10, 4)), 1e-6)
    assert sk.size == 0 and np.array_equal(rd, np.arange(4)) and T.shape == (0, 4)


def test_wide_matrix_full_row_rank():
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((5, 12))
    sk, rd, T = interp_decomp(Y, 1e-12)
    assert sk.size == 5
    assert np.linalg.norm(Y[:, rd] - Y[:, sk] @ T) <= 1e-12 * np.linalg.norm(Y) * 10
