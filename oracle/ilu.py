"""Incomplete LU factorisation by fine-grained fixed-point sweeps, FP64 on the CPU (test
infrastructure, see the package docstring).

The paper's global smoother on the level that holds only cell unknowns is one step of
pointwise ILU(1) computed by the fine-grained parallel algorithm of Chow and Patel (Sec. 5.3
remarks on the second-level global smoother; Sec. 6, solver description).  What is
computed here:

  * the ILU(k) pattern S: level of fill 0 for every structural entry of A, and for a fill
    entry (i, j) created by eliminating m < min(i, j) the level lev(i,m) + lev(m,j) + 1,
    keeping entries whose level is at most k (the textbook symbolic factorisation, rows in
    order, pivots m of each row in ascending order);
  * the factors L (unit lower) and U (upper) on S as the fixed point of the component
    equations of A = LU restricted to S:
        l_ij = (a_ij - sum_{m < j} l_im u_mj) / u_jj      (i > j)
        u_ij =  a_ij - sum_{m < i} l_im u_mj              (i <= j)
    (a_ij = 0 on fill entries, sums over m with (i, m) and (m, j) in S), iterated in
    synchronous sweeps: every component of the new iterate is computed from the previous
    one, so the result does not depend on an update order.  The starting iterate is
    l_ij = a_ij / a_jj, u_ij = a_ij.  Each sum is accumulated in ascending m, one product
    and one subtraction at a time, starting from a_ij;
  * the triangular solves of the smoother either exactly or, as a fine-grained method
    does, by Jacobi sweeps on each factor: L y = r from y = r by y <- r - (L - I) y, then
    U z = y from z = D_U^{-1} y by z <- D_U^{-1} (y - (U - D_U) z).

Readings (the paper names the method, not these details): no symmetric scaling before the
sweeps (the sweeps are equivariant under it); the number of factor sweeps and of
triangular sweeps are options of the smoother; a structurally missing diagonal is an error.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .sparse import CSR, sequential_segment_sum


class ZeroPivot(ArithmeticError):
    pass


def ilu_pattern(A: CSR, k: int) -> CSR:
    """The ILU(k) pattern of A as a CSR with the values of A on it (+0.0 on fill entries),
    by the symbolic factorisation with levels of fill."""
    n = A.shape[0]
    rows_cols, rows_lev = [], []
    for i in range(n):
        s, e = A.indptr[i], A.indptr[i + 1]
        lev = {int(c): 0 for c in A.indices[s:e]}
        # eliminate pivots m < i in ascending order; fill may add new pivots below i
        done = set()
        while True:
            pend = sorted(m for m in lev if m < i and m not in done)
            if not pend:
                break
            m = pend[0]
            done.add(m)
            lm = lev[m]
            for j, lmj in zip(rows_cols[m], rows_lev[m]):
                if j <= m:
                    continue
                L = lm + lmj + 1
                if L <= k and L < lev.get(j, k + 1):
                    lev[j] = L
        cols = np.array(sorted(lev), dtype=np.int64)
        rows_cols.append(cols)
        rows_lev.append(np.array([lev[c] for c in cols], dtype=np.int64))
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum([c.shape[0] for c in rows_cols], out=indptr[1:])
    indices = np.concatenate(rows_cols) if n else np.zeros(0, dtype=np.int64)
    vals = np.zeros(indices.shape[0])
    # values of A on its own entries
    key_s = np.repeat(np.arange(n, dtype=np.int64), np.diff(indptr)) * n + indices
    key_a = A.row_ids() * n + A.indices
    vals[np.searchsorted(key_s, key_a)] = A.data
    return CSR(indptr, indices, vals, A.shape)


@dataclass
class ILUFactors:
    S: CSR                    # pattern and the current values: l_ij below, u_ij on/above
    a: np.ndarray             # a_ij on S (0 on fill)
    diag: np.ndarray          # position of (i, i) in S
    pair_l: np.ndarray        # for each entry, its (l_im, u_mj) pairs in ascending m
    pair_u: np.ndarray
    pair_start: np.ndarray
    pair_len: np.ndarray


def _pairs(S: CSR):
    """For every entry (i, j) of S the positions of l_im and u_mj, m < min(i, j), both in S,
    in ascending m."""
    n = S.shape[0]
    r = S.row_ids()
    keys = r * n + S.indices
    lo = np.flatnonzero(S.indices < r)                 # entries (i, m), m < i
    out_e, out_l, out_u = [], [], []
    for p in lo:                                       # ascending (i, m)
        i, m = int(r[p]), int(S.indices[p])
        s, e = S.indptr[m], S.indptr[m + 1]
        up = np.arange(s, e)[S.indices[s:e] > m]       # entries (m, j), j > m
        want = i * n + S.indices[up]
        q = np.searchsorted(keys, want)
        q = np.minimum(q, keys.shape[0] - 1)
        hit = keys[q] == want
        out_e.append(q[hit])
        out_l.append(np.full(int(hit.sum()), p, dtype=np.int64))
        out_u.append(up[hit])
    if out_e:
        e = np.concatenate(out_e)
        pl = np.concatenate(out_l)
        pu = np.concatenate(out_u)
    else:
        e = pl = pu = np.zeros(0, dtype=np.int64)
    # pairs were produced by ascending (i, m); a stable sort by entry keeps ascending m
    order = np.argsort(e, kind="stable")
    e, pl, pu = e[order], pl[order], pu[order]
    cnt = np.bincount(e, minlength=S.nnz)
    start = np.concatenate(([0], np.cumsum(cnt)[:-1])).astype(np.int64)
    return pl, pu, start, cnt


def ilu_init(A: CSR, k: int) -> ILUFactors:
    """Pattern, pair lists and the starting iterate l_ij = a_ij / a_jj, u_ij = a_ij."""
    S = ilu_pattern(A, k)
    n = S.shape[0]
    r = S.row_ids()
    dpos = np.full(n, -1, dtype=np.int64)
    isd = S.indices == r
    dpos[r[isd]] = np.flatnonzero(isd)
    if np.any(dpos < 0) or np.any(S.data[dpos] == 0.0):
        raise ZeroPivot("zero or missing diagonal")
    a = S.data.copy()
    v = a.copy()
    low = S.indices < r
    v[low] = a[low] / a[dpos[S.indices[low]]]
    pl, pu, st, ln = _pairs(S)
    return ILUFactors(CSR(S.indptr, S.indices, v, S.shape), a, dpos, pl, pu, st, ln)


def ilu_sweep(F: ILUFactors) -> None:
    """One synchronous fixed-point sweep over every component of L and U."""
    S = F.S
    old = S.data
    prod = old[F.pair_l] * old[F.pair_u]
    # s = a_ij - p_1 - p_2 - ... in ascending m: subtract the running sum of the products
    # one at a time (a_ij + (-p)) so each step is one rounding
    s = F.a.copy()
    for t in range(int(F.pair_len.max()) if F.pair_len.size else 0):
        msk = F.pair_len > t
        s[msk] = s[msk] - prod[F.pair_start[msk] + t]
    r = S.row_ids()
    low = S.indices < r
    new = s.copy()
    new[low] = s[low] / old[F.diag[S.indices[low]]]
    S.data = new


def ilu_factor(A: CSR, k: int, sweeps: int) -> ILUFactors:
    F = ilu_init(A, k)
    for _ in range(sweeps):
        ilu_sweep(F)
    return F


def split_lu(F: ILUFactors):
    """(L - I, U - D_U, d_U) as CSR matrices and the diagonal of U."""
    S = F.S
    r = S.row_ids()
    low, up = S.indices < r, S.indices > r

    def part(m):
        indptr = np.zeros(S.shape[0] + 1, dtype=np.int64)
        np.cumsum(np.bincount(r[m], minlength=S.shape[0]), out=indptr[1:])
        return CSR(indptr, S.indices[m], S.data[m], S.shape)
    return part(low), part(up), S.data[F.diag]


def ilu_solve(F: ILUFactors, rhs: np.ndarray, tri_sweeps: int) -> np.ndarray:
    """z ~ (LU)^{-1} rhs: exact triangular solves when tri_sweeps < 0, else tri_sweeps
    Jacobi sweeps on each factor after the starting iterate."""
    Ls, Us, d = split_lu(F)
    if tri_sweeps < 0:
        import scipy.sparse as sp
        from scipy.sparse.linalg import spsolve_triangular
        n = F.S.shape[0]
        L = (Ls.scipy() + sp.identity(n, format="csr")).tocsr()
        U = (Us.scipy() + sp.diags(d)).tocsr()
        y = spsolve_triangular(L, rhs, lower=True, unit_diagonal=True)
        return spsolve_triangular(U, y, lower=False)
    y = rhs.copy()
    for _ in range(tri_sweeps):
        y = rhs - Ls.matvec(y)
    z = y / d
    for _ in range(tri_sweeps):
        z = (y - Us.matvec(z)) / d
    return z
