"""Oracle results at sampled rows of full-size problems (test infrastructure, CPU only).

The MGR level step of Sec. 5.2 is row-local: row i of A_{l+1} = A_CC - G(A_CF D_FF^{-1}
A_FC) needs only row C[i] of A_l and the rows of A_l at the F-points that row touches.  The
functions here run the oracle's own steps (blocks_of, jacobi_interpolation, spgemm, drop,
merge_sub, transpose) on *row-restricted* matrices: the full shape, with only the rows a
requested output depends on.  Every kept row goes through exactly the arithmetic the oracle
applies to the whole matrix, so the sampled rows equal the oracle's rows bit for bit, at
sizes where the whole oracle setup would take minutes.  Recursion over levels composes the
same way: the rows of A_{l+1} that level l+1 needs are themselves computed from A_l.
"""
from __future__ import annotations

import numpy as np

from oracle import mgr as omgr
from oracle.sparse import CSR, diagonal, gather_rows, merge_sub, spgemm


def restrict_rows(A: CSR, rows) -> CSR:
    """A with every row outside `rows` emptied (same shape)."""
    rows = np.unique(np.asarray(rows, dtype=np.int64))
    pos, _ = gather_rows(A, rows)
    lens = np.zeros(A.shape[0], dtype=np.int64)
    lens[rows] = np.diff(A.indptr)[rows]
    indptr = np.zeros(A.shape[0] + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    return CSR(indptr, A.indices[pos], A.data[pos], A.shape)


def stack_rows(X: CSR, Y: CSR) -> CSR:
    """The union of two row-restricted matrices of one shape whose non-empty rows differ."""
    assert X.shape == Y.shape
    lx, ly = np.diff(X.indptr), np.diff(Y.indptr)
    assert not np.any((lx > 0) & (ly > 0)), "row sets overlap"
    lens = lx + ly
    indptr = np.zeros(X.shape[0] + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    cols = np.empty(indptr[-1], dtype=np.int64)
    vals = np.empty(indptr[-1])
    for M in (X, Y):
        r = M.row_ids()
        off = M.indptr[:-1][r]
        dst = indptr[:-1][r] + (np.arange(M.nnz) - off)
        cols[dst] = M.indices
        vals[dst] = M.data
    return CSR(indptr, cols, vals, X.shape)


class LevelRows:
    """Rows of the operators of one MGR level, computed on demand from the rows of the
    level's matrix A_l (given by `rows_of`, a function: original row indices -> A_l
    restricted to them)."""

    def __init__(self, rows_of, labels: np.ndarray, lp: omgr.LevelPlan):
        self.rows_of = rows_of
        self.labels = np.asarray(labels)
        self.lp = lp
        self.F, self.C = omgr.cf_split(self.labels, lp.f_labels)
        n = self.labels.shape[0]
        self.isF = np.zeros(n, dtype=bool)
        self.isF[self.F] = True
        self.fpos = np.full(n, -1, dtype=np.int64)
        self.fpos[self.F] = np.arange(self.F.shape[0])

    def coarse_rows(self, rows_c):
        """(A_{l+1} restricted to rows_c, W_p restricted to the F rows they touch, those F
        rows as F-indices).  rows_c are C-indices, i.e. row indices of A_{l+1}."""
        rows_c = np.unique(np.asarray(rows_c, dtype=np.int64))
        Arc = self.rows_of(self.C[rows_c])
        touched = Arc.indices[self.isF[Arc.indices]]
        ks = np.unique(touched)
        Ar = stack_rows(Arc, self.rows_of(ks)) if ks.shape[0] else Arc
        A_FF, A_FC, A_CF, A_CC = omgr.blocks_of(Ar, self.F, self.C)
        d = diagonal(A_FF)      # NaN on emptied rows; their rows of A_FC are empty too
        M, Wp = omgr.jacobi_interpolation(A_FC, d)
        Acor = spgemm(omgr.coupling_block(A_CF, self.labels, self.F, self.C,
                                          self.lp.coupling), M)
        G = omgr.drop(Acor, self.labels[self.C], self.lp.nmax, self.lp.drop_tol)
        S = merge_sub(A_CC, G)
        return restrict_rows(S, rows_c), restrict_rows(Wp, self.fpos[ks]), self.fpos[ks]


def level_chain(A: CSR, labels: np.ndarray, plan: omgr.Plan):
    """LevelRows for every level of the plan, each fed by the one above it."""
    chain = []
    rows_of = lambda rows: restrict_rows(A, rows)   # noqa: E731
    lab = np.asarray(labels)
    for lp in plan.levels:
        L = LevelRows(rows_of, lab, lp)
        chain.append(L)
        rows_of = (lambda L: (lambda rows: L.coarse_rows(rows)[0]))(L)
        lab = lab[L.C]
    return chain


def rows_of_export(exp, rows):
    """(row lengths, columns, values) of the given rows of a CSR export tuple."""
    rp, ci, v, _ = exp
    rows = np.asarray(rows, dtype=np.int64)
    lens = rp[rows + 1] - rp[rows]
    pos = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows]) if rows.size else \
        np.zeros(0, dtype=np.int64)
    return lens, ci[pos], v[pos]


def assert_rows_equal(exp_tuple, ref: CSR, rows, what=""):
    """Bit-exact equality of the given rows of a CSR export and a row-restricted oracle
    matrix (patterns, values and signs of zeros)."""
    rows = np.unique(np.asarray(rows, dtype=np.int64))
    assert tuple(exp_tuple[3]) == ref.shape, (what, exp_tuple[3], ref.shape)
    lens, ci, v = rows_of_export(exp_tuple, rows)
    rlens, rci, rv = rows_of_export((ref.indptr, ref.indices, ref.data, ref.shape), rows)
    assert np.array_equal(lens, rlens), f"{what}: row lengths differ"
    assert np.array_equal(ci, rci), f"{what}: columns differ"
    same = (v == rv) | (np.isnan(v) & np.isnan(rv))
    if not np.all(same):
        i = int(np.flatnonzero(~same)[0])
        raise AssertionError(f"{what}: {int((~same).sum())} of {v.size} values differ, "
                             f"first {v[i]!r} vs {rv[i]!r}")
    assert np.array_equal(np.signbit(v), np.signbit(rv)), f"{what}: signs of zeros differ"


def sample_rows(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct rows: the first two, the last two and the rest uniformly at random."""
    rng = np.random.default_rng(seed)
    fixed = np.array([0, 1, n - 2, n - 1], dtype=np.int64)
    rest = rng.choice(n, size=min(n, k), replace=False)
    return np.unique(np.concatenate([fixed[(fixed >= 0) & (fixed < n)], rest]))
