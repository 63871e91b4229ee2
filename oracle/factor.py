"""RSF and HIF-IE factorization and the factored sweeps (oracle; test infrastructure only).

Follows the paper step by step:

* Algorithm 3.1 (RSF): skeletonize the cells of every level, finest first.
* Algorithm 4.1 / 4.2 (HIF-IE): after the cells of level ``l`` skeletonize the
  edges (2D) or the faces and then the edges (3D) of that level.
* Skeletonization of one index set ``c`` (Lemma 2.4): an ID of the compressed
  block ``Y_c`` gives ``(skeleton, redundant, T)``; the block
  ``A_cc`` is transformed by ``Q_c``, the redundant part is eliminated by
  block LU (Lemma 2.1) and the Schur complement update lands on the skeleton
  block.  Entries are generated on demand as kernel entries plus the
  accumulated Schur-complement interactions (SCIs).
* Accelerated compression (Section 3.3, eqn proxy-id) with the SCI-expanded
  near field of Section 4.3: ``Y_c`` stacks the rows of the near field
  ``c^N`` (DOFs strictly inside the proxy circle / sphere of radius
  ``1.5 w`` about the group centre, plus every DOF coupled to ``c`` by an SCI)
  and the proxy rows.  With a symmetric operator only the column block is
  compressed (Section 5, ``Y'_c``).
* Second-kind modification (Section 4.4): the local tolerance is ``rho eps``
  with ``rho = min(1, |Y^K| / |Y^S|)``, and the columns are split into
  classes with identical SCI sparsity pattern (Lemma 4.2), each compressed
  on its own, ``T = diag(T_g)``.
* Groups of one sub-level commute (Section 2.3, "any order"); every group is
  compressed against the sub-level's starting state, then all updates are
  applied.

The factored operators (eqns rskelf, hifie2, hifie3) are applied as sweeps
over the stored group records; see ``Factorization``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
from scipy.linalg import lu_factor, lu_solve
from scipy.spatial import cKDTree

from .idqr import interp_decomp
from .kernels import Operator, green
from .tree import (CELL, assign, centres, default_proxy_count, proxy_directions,
                   sublevel_kinds, tree_depth)


class SingularBlockError(RuntimeError):
    """A redundant block ``B_rr`` or the top block has a zero pivot (Lemma 2.1 needs it nonsingular)."""


@dataclass
class GroupRecord:
    """Factors of one skeletonized index set (Lemma 2.4)."""

    rd: np.ndarray      # redundant DOFs (global indices)
    sk: np.ndarray      # skeleton DOFs (global indices)
    T: np.ndarray       # k x r interpolation matrix
    Brr: np.ndarray     # r x r transformed redundant block
    lu: tuple           # LU of Brr with partial pivoting
    E: np.ndarray       # k x r, B_sr Brr^{-1}
    G: np.ndarray       # r x k, Brr^{-1} B_rs


@dataclass
class SubLevelStats:
    level: int
    kind: str
    n_groups: int
    sizes: list = field(default_factory=list)       # |c|
    near: list = field(default_factory=list)        # |c^N|
    classes: list = field(default_factory=list)     # number of split classes
    ranks: list = field(default_factory=list)       # |skeleton|
    active_after: int = 0


@dataclass
class Factorization:
    """``F`` and ``F^{-1}`` in factored form (eqns rskelf, hifie2, hifie3)."""

    N: int
    d: int
    L: int
    eps: float
    sublevels: list          # list of lists of GroupRecord, factor order
    top: np.ndarray          # active DOFs at the top, s_L
    top_A: np.ndarray        # A_L(s_L, s_L)
    top_lu: tuple
    stats: list

    # -- sweeps -----------------------------------------------------------
    def _records(self):
        for recs in self.sublevels:
            for r in recs:
                yield r

    @staticmethod
    def _cols(x):
        x = np.asarray(x, dtype=np.float64)
        return (x[:, None].copy() if x.ndim == 1 else x.T.copy()), x.ndim == 1

    @staticmethod
    def _out(u, vec):
        return u[:, 0] if vec else np.ascontiguousarray(u.T)

    def solve(self, f):
        """``u = F^{-1} f = V_0 ... D^{-1} ... U_0^* f``; ``f`` is ``(N,)`` or ``(nrhs, N)``."""
        u, vec = self._cols(f)
        for r in self._records():
            u[r.rd] -= r.T.T @ u[r.sk]
            u[r.sk] -= r.E @ u[r.rd]
        for r in self._records():
            u[r.rd] = lu_solve(r.lu, u[r.rd])
        if self.top.size:
            u[self.top] = lu_solve(self.top_lu, u[self.top])
        for r in reversed(list(self._records())):
            u[r.rd] -= r.G @ u[r.sk]
            u[r.sk] -= r.T @ u[r.rd]
        return self._out(u, vec)

    def solve_T(self, f):
        """``u = F^{-T} f``."""
        u, vec = self._cols(f)
        for r in self._records():
            u[r.rd] -= r.T.T @ u[r.sk]
            u[r.sk] -= r.G.T @ u[r.rd]
        for r in self._records():
            u[r.rd] = lu_solve(r.lu, u[r.rd], trans=1)
        if self.top.size:
            u[self.top] = lu_solve(self.top_lu, u[self.top], trans=1)
        for r in reversed(list(self._records())):
            u[r.rd] -= r.E.T @ u[r.sk]
            u[r.sk] -= r.T @ u[r.rd]
        return self._out(u, vec)

    def apply(self, x):
        """``y = F x = U_0^{-*} ... D ... V_0^{-1} x``."""
        y, vec = self._cols(x)
        for r in self._records():
            y[r.sk] += r.T @ y[r.rd]
            y[r.rd] += r.G @ y[r.sk]
        for r in self._records():
            y[r.rd] = r.Brr @ y[r.rd]
        if self.top.size:
            y[self.top] = self.top_A @ y[self.top]
        for r in reversed(list(self._records())):
            y[r.sk] += r.E @ y[r.rd]
            y[r.rd] += r.T.T @ y[r.sk]
        return self._out(y, vec)

    def apply_T(self, x):
        """``y = F^T x``."""
        y, vec = self._cols(x)
        for r in self._records():
            y[r.sk] += r.T @ y[r.rd]
            y[r.rd] += r.E.T @ y[r.sk]
        for r in self._records():
            y[r.rd] = r.Brr.T @ y[r.rd]
        if self.top.size:
            y[self.top] = self.top_A.T @ y[self.top]
        for r in reversed(list(self._records())):
            y[r.sk] += r.G.T @ y[r.rd]
            y[r.rd] += r.T.T @ y[r.sk]
        return self._out(y, vec)

    # -- bookkeeping ------------------------------------------------------
    def memory_bytes(self) -> int:
        """Bytes of the stored factors: T, E, G, LU(Brr) per group plus the top LU (FP64) and indices."""
        tot = 0
        for r in self._records():
            k, n = r.T.shape
            tot += 8 * (3 * k * n + n * n) + 4 * (2 * n + k)
        m = self.top.size
        return tot + 8 * m * m + 4 * 2 * m


def _lu_checked(M: np.ndarray):
    if M.size == 0:
        return (M.copy(), np.zeros(0, dtype=np.int32))
    lu, piv = lu_factor(M, check_finite=True)
    if np.any(np.diag(lu) == 0.0):
        raise SingularBlockError("zero pivot in block LU")
    return (lu, piv)


def _column_patterns(Ysub: sp.spmatrix):
    """Structural row pattern of every column of a sparse block (stored entries, whatever their value)."""
    C = sp.csc_matrix(Ysub)
    C.sort_indices()
    return [tuple(C.indices[C.indptr[j]:C.indptr[j + 1]]) for j in range(C.shape[1])]


def factorize(op: Operator, eps: float, leaf: int, *, variant: str = "hifie",
              second_kind: bool = True, symmetric: bool | None = None,
              n_proxy: int | None = None, proxy_radius: float = 1.5,
              fp32_blocks: bool = False, trace=None) -> Factorization:
    """Factor ``A`` (RSF for ``variant='rskel'``, HIF-IE otherwise).

    ``second_kind`` switches on the Section 4.4 modification (hifie2x /
    hifie3x); ``symmetric`` forces the column-only compression of Section 5
    (default: whenever A is symmetric).  ``fp32_blocks`` rounds every
    assembled block and Schur update to float32 (an emulation of reduced
    precision assembly; the ID and LU stay FP64).

    ``trace``, if given, is called once per group of every sub-level with a
    dict of that group's intermediate quantities (for per-step parity tests;
    it changes nothing): ``level``, ``kind``, ``active`` (the active DOFs at
    the start of the sub-level), ``c``, ``near`` (c^N), ``Y`` (the compressed
    block), ``classes`` (column index sets), ``tols`` (their ID tolerances),
    ``sk``/``rd`` (group-local), ``T``, and when the group has redundant DOFs
    ``Acc`` (A(c, c) with its SCIs), ``Brr``, ``Brs``, ``Bsr``, ``Bss`` (the
    transformed blocks of Lemma 2.4) and ``dS`` (the Schur update of the
    skeleton block).
    """
    N, d = op.N, op.d
    pts = op.points
    L = tree_depth(pts, leaf)
    sym = op.symmetric if symmetric is None else bool(symmetric)
    P = default_proxy_count(d) if n_proxy is None else int(n_proxy)
    U = proxy_directions(d, P)
    rnd = (lambda M: M.astype(np.float32).astype(np.float64)) if fp32_blocks else (lambda M: M)

    active = np.ones(N, dtype=bool)
    S = sp.csr_matrix((N, N))
    sublevels = []
    stats = []

    for lvl in range(L):
        nbox = 2 ** (L - lvl)
        w = 1.0 / nbox
        R = proxy_radius * w
        for kind in sublevel_kinds(d, variant):
            Z = centres(kind, d, nbox)
            act = np.nonzero(active)[0]
            key = assign(pts, active, kind, nbox)
            grp_of = np.full(N, -1, dtype=np.int64)
            grp_of[act] = key
            order = np.lexsort((act, key))
            skey = key[order]
            sact = act[order]
            gids, starts = np.unique(skey, return_index=True)
            ends = np.append(starts[1:], skey.size)

            # Snapshot of the sub-level's starting state.
            S_csr = S.tocsr()
            S_csr.sort_indices()
            S_csc = S_csr.tocsc()
            kd = cKDTree(pts[act]) if act.size else None
            near_geo = kd.query_ball_point(Z[gids], r=R * (1.0 + 1e-9)) if act.size else [[] for _ in gids]

            st = SubLevelStats(lvl, kind, int(gids.size))
            records = []
            new_rows, new_cols, new_vals = [], [], []
            eliminated = np.zeros(Z.shape[0], dtype=bool)
            for gi, g in enumerate(gids):
                c = sact[starts[gi]:ends[gi]]
                z = Z[g]
                # Near field c^N (Section 3.3 and Section 4.3).
                cand = act[np.asarray(near_geo[gi], dtype=np.int64)]
                dz = pts[cand] - z
                d2 = np.zeros(cand.size)
                for k in range(d):
                    d2 += dz[:, k] * dz[:, k]
                geo = cand[(d2 < R * R) & (grp_of[cand] != g)]
                sci = np.union1d(S_csr[c].indices, S_csc[:, c].indices)
                sci = sci[grp_of[sci] != g] if sci.size else sci
                cN = np.union1d(geo, sci).astype(np.int64)

                # Compressed block Y_c (eqn proxy-id; Y'_c of Section 5 when symmetric).
                xp = z + R * U
                diff = xp[:, None, :] - pts[c][None, :, :]
                rp = np.sqrt(np.sum(diff * diff, axis=2))
                prox_col = green(rp, d) * (op.weights[c] * op.c[c])[None, :]
                YK = [op.kernel_block(cN, c), prox_col]
                YSs = [S_csr[cN][:, c]]
                if not sym:
                    YK.append(op.kernel_block(c, cN).T)
                    prox_row = green(rp, d) * (op.b[c] * op.weights[c])[None, :]
                    YK.append(prox_row)
                    YSs.append(S_csr[c][:, cN].T)
                YKm = rnd(np.vstack(YK))
                ms = sum(M.shape[0] for M in YSs)
                YSsp = sp.vstack(YSs + [sp.csr_matrix((YKm.shape[0] - ms, c.size))]).tocsr()
                YSm = rnd(YSsp.toarray())
                Y = YKm + YSm

                # Column classes (Section 4.4, Lemma 4.2) and local tolerances.
                if second_kind and YSsp.nnz > 0:
                    pats = _column_patterns(YSsp)
                    cls_of, lookup = [], {}
                    for j, pt in enumerate(pats):
                        if pt not in lookup:
                            lookup[pt] = len(lookup)
                        cls_of.append(lookup[pt])
                    cls_of = np.asarray(cls_of)
                    classes = [np.nonzero(cls_of == q)[0] for q in range(len(lookup))]
                else:
                    classes = [np.arange(c.size)]
                sk_loc, rd_loc, Tblocks, tols = [], [], [], []
                for cols in classes:
                    rho = 1.0
                    if second_kind:
                        nS = np.linalg.norm(YSm[:, cols])
                        if nS > 0.0:
                            rho = min(1.0, np.linalg.norm(YKm[:, cols]) / nS)
                    tols.append(rho * eps)
                    s_g, r_g, T_g = interp_decomp(Y[:, cols], rho * eps)
                    sk_loc.append(cols[s_g])
                    rd_loc.append(cols[r_g])
                    Tblocks.append(T_g)
                sk_l = np.concatenate(sk_loc).astype(np.int64)
                rd_l = np.concatenate(rd_loc).astype(np.int64)
                T = np.zeros((sk_l.size, rd_l.size))
                ro = co = 0
                for T_g in Tblocks:
                    T[ro:ro + T_g.shape[0], co:co + T_g.shape[1]] = T_g
                    ro += T_g.shape[0]
                    co += T_g.shape[1]

                st.sizes.append(int(c.size))
                st.near.append(int(cN.size))
                st.classes.append(len(classes))
                st.ranks.append(int(sk_l.size))
                info = None
                if trace is not None:
                    info = dict(level=lvl, kind=kind, active=act, c=c, near=cN, Y=Y, classes=classes, tols=tols,
                                sk=sk_l, rd=rd_l, T=T)
                if rd_l.size == 0:
                    if trace is not None:
                        trace(info)
                    continue

                # Skeletonization of c (Lemma 2.4) with block elimination (Lemma 2.1).
                Scc = S_csr[c][:, c].toarray()
                Acc = rnd(op.block(c, c) + Scc)
                Arr = Acc[np.ix_(rd_l, rd_l)]
                Ars = Acc[np.ix_(rd_l, sk_l)]
                Asr = Acc[np.ix_(sk_l, rd_l)]
                Ass = Acc[np.ix_(sk_l, sk_l)]
                Brs = Ars - T.T @ Ass
                Bsr = Asr - Ass @ T
                Brr = Arr - T.T @ Asr - Ars @ T + T.T @ Ass @ T
                lu = _lu_checked(Brr)
                G = lu_solve(lu, Brs) if sk_l.size else np.zeros((rd_l.size, 0))
                E = lu_solve(lu, Bsr.T, trans=1).T if sk_l.size else np.zeros((0, rd_l.size))
                dS = rnd(-E @ Brs)
                if trace is not None:
                    # the transform of Lemma 2.4 leaves the skeleton block as it was
                    info.update(Acc=Acc, Brr=Brr, Brs=Brs, Bsr=Bsr, Bss=Ass, dS=dS)
                    trace(info)
                sk = c[sk_l]
                rd = c[rd_l]
                records.append(GroupRecord(rd, sk, T, Brr, lu, E, G))
                eliminated[g] = True
                if sk.size:
                    blk = Scc[np.ix_(sk_l, sk_l)] + dS
                    ii, jj = np.meshgrid(sk, sk, indexing="ij")
                    new_rows.append(ii.ravel())
                    new_cols.append(jj.ravel())
                    new_vals.append(blk.ravel())

            # Apply the sub-level: eliminate redundant DOFs, update and purge the SCIs.
            for r in records:
                active[r.rd] = False
            coo = S_csr.tocoo()
            gi_, gj_ = grp_of[coo.row], grp_of[coo.col]
            keep = active[coo.row] & active[coo.col] & ((gi_ != gj_) | ~eliminated[gi_])
            rows = np.concatenate([coo.row[keep]] + new_rows).astype(np.int64)
            cols = np.concatenate([coo.col[keep]] + new_cols).astype(np.int64)
            vals = np.concatenate([coo.data[keep]] + new_vals)
            S = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
            st.active_after = int(active.sum())
            sublevels.append(records)
            stats.append(st)

    top = np.nonzero(active)[0]
    top_A = op.block(top, top) + S.tocsr()[top][:, top].toarray() if top.size else np.zeros((0, 0))
    top_A = rnd(top_A)
    top_lu = _lu_checked(top_A) if top.size else (np.zeros((0, 0)), np.zeros(0, dtype=np.int32))
    return Factorization(N, d, L, eps, sublevels, top, top_A, top_lu, stats)
