"""Minimal CSR container and the pinned-order sparse operations of the oracle.

Test infrastructure (see the package docstring).  Every routine is written for clarity:
NumPy does the bookkeeping, and the only floating-point operations are the ones the
definitions name, applied one at a time (one multiply, then one add; no fused multiply-add,
since NumPy evaluates `a * b` and `+` as separately rounded operations).
"""
from __future__ import annotations

import numpy as np


class CSR:
    """Compressed sparse rows with int64 indices and float64 values.  Column indices are
    sorted and unique within a row; explicit zeros are kept as part of the pattern."""

    __slots__ = ("indptr", "indices", "data", "shape")

    def __init__(self, indptr, indices, data, shape):
        self.indptr = np.asarray(indptr, dtype=np.int64)
        self.indices = np.asarray(indices, dtype=np.int64)
        self.data = np.asarray(data, dtype=np.float64)
        self.shape = (int(shape[0]), int(shape[1]))

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def row_ids(self) -> np.ndarray:
        return np.repeat(np.arange(self.shape[0], dtype=np.int64), np.diff(self.indptr))

    def to_dense(self) -> np.ndarray:
        D = np.zeros(self.shape)
        D[self.row_ids(), self.indices] = self.data
        return D

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=self.shape)

    def matvec(self, x: np.ndarray) -> np.ndarray:
        return self.scipy() @ x

    def row(self, i):
        s, e = self.indptr[i], self.indptr[i + 1]
        return self.indices[s:e], self.data[s:e]

    @staticmethod
    def from_dense(D: np.ndarray, keep_zeros_mask=None) -> "CSR":
        mask = (D != 0) if keep_zeros_mask is None else keep_zeros_mask
        r, c = np.nonzero(mask)
        indptr = np.zeros(D.shape[0] + 1, dtype=np.int64)
        np.cumsum(np.bincount(r, minlength=D.shape[0]), out=indptr[1:])
        return CSR(indptr, c, D[r, c], D.shape)

    @staticmethod
    def from_coo(rows, cols, vals, shape) -> "CSR":
        """Rows/cols must already be unique pairs; sorted here by (row, col)."""
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        order = np.lexsort((cols, rows))
        indptr = np.zeros(shape[0] + 1, dtype=np.int64)
        np.cumsum(np.bincount(rows, minlength=shape[0]), out=indptr[1:])
        return CSR(indptr, cols[order], np.asarray(vals, dtype=np.float64)[order], shape)


def gather_rows(A: CSR, rows: np.ndarray):
    """Entry positions of the given rows, in row order then column order."""
    rows = np.asarray(rows, dtype=np.int64)
    lens = np.diff(A.indptr)[rows]
    starts = A.indptr[rows]
    tot = int(lens.sum())
    base = np.repeat(starts - (np.cumsum(lens) - lens), lens)
    pos = base + np.arange(tot, dtype=np.int64)
    return pos, np.repeat(np.arange(rows.shape[0], dtype=np.int64), lens)


def submatrix(A: CSR, rows: np.ndarray, colmap: np.ndarray, ncols: int) -> CSR:
    """Rows `rows` (ascending) of A, keeping the entries whose column c has colmap[c] >= 0
    and renumbering that column to colmap[c].  Pattern (explicit zeros) is preserved; an
    increasing colmap keeps the columns sorted."""
    pos, newrow = gather_rows(A, rows)
    newcol = colmap[A.indices[pos]]
    keep = newcol >= 0
    pos, newrow, newcol = pos[keep], newrow[keep], newcol[keep]
    indptr = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(np.bincount(newrow, minlength=len(rows)), out=indptr[1:])
    return CSR(indptr, newcol, A.data[pos], (len(rows), ncols))


def diagonal(A: CSR) -> np.ndarray:
    """a_ii for every row; NaN where the diagonal is structurally missing."""
    n = min(A.shape)
    d = np.full(A.shape[0], np.nan)
    r = A.row_ids()
    m = (A.indices == r) & (r < n)
    d[r[m]] = A.data[m]
    return d


def sequential_segment_sum(values: np.ndarray, seg_start: np.ndarray, seg_len: np.ndarray):
    """out[s] = (((0.0 + v[start]) + v[start+1]) + ...) in index order, one rounding per add."""
    out = np.zeros(seg_start.shape[0])
    if seg_start.shape[0] == 0:
        return out
    for r in range(int(seg_len.max()) if seg_len.size else 0):
        m = seg_len > r
        out[m] = out[m] + values[seg_start[m] + r]
    return out


def row_sum_abs_sequential(A: CSR) -> np.ndarray:
    """sum_j |a_ij| accumulated in ascending column order."""
    return sequential_segment_sum(np.abs(A.data), A.indptr[:-1], np.diff(A.indptr))


def spgemm(A: CSR, B: CSR) -> CSR:
    """C = A B with the pinned summation order.

    c_ij = sum over k of a_ik * b_kj where, for every output entry, the products are taken in
    ascending k and added one at a time to an accumulator that starts at +0.0.  The pattern
    of C is the symbolic one: every (i, j) reached by some product, including entries whose
    value cancels to zero.  This is the plain definition of the matrix product with the
    order of the sum fixed, so that a GPU implementation can reproduce it bit for bit.
    """
    assert A.shape[1] == B.shape[0]
    ai = A.row_ids()
    ak = A.indices
    blen = np.diff(B.indptr)[ak]
    tot = int(blen.sum())
    if tot == 0:
        return CSR(np.zeros(A.shape[0] + 1, dtype=np.int64), np.zeros(0, dtype=np.int64),
                   np.zeros(0), (A.shape[0], B.shape[1]))
    first = np.repeat(B.indptr[ak] - (np.cumsum(blen) - blen), blen)
    bpos = first + np.arange(tot, dtype=np.int64)
    prow = np.repeat(ai, blen)
    pcol = B.indices[bpos]
    pval = np.repeat(A.data, blen) * B.data[bpos]
    # products are generated in (row, ascending k) order; a stable sort on (row, col)
    # therefore leaves the products of each output entry in ascending k.
    key = prow * np.int64(B.shape[1]) + pcol
    order = np.argsort(key, kind="stable")
    key = key[order]
    pval = pval[order]
    is_first = np.empty(key.shape[0], dtype=bool)
    is_first[0] = True
    np.not_equal(key[1:], key[:-1], out=is_first[1:])
    seg_start = np.flatnonzero(is_first)
    seg_len = np.diff(np.append(seg_start, key.shape[0]))
    vals = sequential_segment_sum(pval, seg_start, seg_len)
    ukey = key[seg_start]
    rows = ukey // np.int64(B.shape[1])
    cols = ukey % np.int64(B.shape[1])
    indptr = np.zeros(A.shape[0] + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=A.shape[0]), out=indptr[1:])
    return CSR(indptr, cols, vals, (A.shape[0], B.shape[1]))


def transpose(A: CSR) -> CSR:
    """A^T; entries of each output row in ascending original row index; values copied."""
    r = A.row_ids()
    key = A.indices * np.int64(A.shape[0]) + r
    order = np.argsort(key, kind="stable")
    indptr = np.zeros(A.shape[1] + 1, dtype=np.int64)
    np.cumsum(np.bincount(A.indices, minlength=A.shape[1]), out=indptr[1:])
    return CSR(indptr, r[order], A.data[order], (A.shape[1], A.shape[0]))


def merge_sub(A: CSR, B: CSR, w: np.ndarray | None = None) -> CSR:
    """S = A - diag(w) B on the union pattern.

    s_ij = a_ij - (w_i * b_ij) where both entries exist, a_ij where only A has one and
    -(w_i * b_ij) where only B has one (w_i = 1 when `w` is None, so b_ij is used as is)."""
    assert A.shape == B.shape
    ra, rb = A.row_ids(), B.row_ids()
    bv = B.data if w is None else w[rb] * B.data
    ncol = np.int64(A.shape[1])
    ka = ra * ncol + A.indices
    kb = rb * ncol + B.indices
    keys = np.union1d(ka, kb)
    ia = np.searchsorted(keys, ka)
    ib = np.searchsorted(keys, kb)
    has_a = np.zeros(keys.shape[0], dtype=bool)
    has_b = np.zeros(keys.shape[0], dtype=bool)
    has_a[ia] = True
    has_b[ib] = True
    av = np.zeros(keys.shape[0])
    bb = np.zeros(keys.shape[0])
    av[ia] = A.data
    bb[ib] = bv
    vals = np.where(has_a & has_b, av - bb, np.where(has_a, av, -bb))
    rows = keys // ncol
    indptr = np.zeros(A.shape[0] + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=A.shape[0]), out=indptr[1:])
    return CSR(indptr, keys % ncol, vals, A.shape)
