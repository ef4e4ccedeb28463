"""Smoothed-aggregation AMG used by the oracle (test infrastructure, see the package
docstring).

The paper uses one V-cycle of an AMG solver for the F-relaxation of the elasticity block
and for the coarsest (pressure) grid (Sec. 5.3 and the solver description of Sec. 6: an
"unknown approach" for the three displacement components, aggressive coarsening, l1
smoothers, direct solve at the coarsest level).  That solver is prior art; this module
defines the AMG of this project precisely, so that the GPU library can be checked against it:

  strength   scalar: j != i is strong when a_ij != 0 and a_ij^2 >= theta^2 |a_ii a_jj|
             nodal (blocks of b unknowns): the same test on squared Frobenius norms,
             f_IJ^2 >= theta^4 f_II f_JJ;  theta_l = 0.08 * 0.5^l; symmetrised by union
  priority   prio(i) = first output of SplitMix64 seeded with i XOR (0x9E3779B97F4A7C15 * (l+1))
  MIS(2)     synchronous rounds: an undecided node whose priority is the largest among the
             undecided nodes within graph distance 2 is selected; nodes within distance 2 of
             a selected node are then removed (Bell, Dalton, Olson 2012)
  aggregates roots = MIS(2); pass 1 joins a root neighbour (highest priority); pass 2 joins
             the aggregate of an aggregated neighbour (highest priority); leftovers become
             singletons; nodes without strong neighbours get no aggregate
  T          T[(node, c), (agg(node), c)] = 1 (components never mixed)
  P          P = T - diag(omega / a_ii) (A T),  omega = (4/3) / rho,
             rho = max_i sum_j |a_ij| / |a_ii|   (Gershgorin bound)
  coarse     R = P^T, A_c = R (A P), both products with the pinned summation order
  stop       n <= coarse_size, or max_levels reached, or n_c > 0.8 n  -> dense LU
  smoother   l1-Jacobi, d_i = sum_j |a_ij| (Baker et al.); one pre-sweep from zero and one
             post-sweep per level
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .sparse import (CSR, diagonal, merge_sub, row_sum_abs_sequential, spgemm,
                     transpose)

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
MIX1 = np.uint64(0xBF58476D1CE4E5B9)
MIX2 = np.uint64(0x94D049BB133111EB)


class ZeroPivot(ArithmeticError):
    pass


@dataclass
class AMGOptions:
    theta0: float = 0.08
    max_levels: int = 10
    coarse_size: int = 256
    block: int = 1          # 1 = scalar, 3 = nodal (unknown approach)


def splitmix64(seed: np.ndarray) -> np.ndarray:
    """First output of a SplitMix64 generator (Steele, Lea, Flood 2014) seeded with `seed`:
    state += 0x9E3779B97F4A7C15, then the variant-13 finaliser."""
    z = np.asarray(seed, dtype=np.uint64) + GOLDEN
    z = (z ^ (z >> np.uint64(30))) * MIX1
    z = (z ^ (z >> np.uint64(27))) * MIX2
    return z ^ (z >> np.uint64(31))


def priorities(n: int, level: int) -> np.ndarray:
    with np.errstate(over="ignore"):
        salt = GOLDEN * np.uint64(level + 1)
        return splitmix64(np.arange(n, dtype=np.uint64) ^ salt)


def theta_at(theta0: float, level: int) -> float:
    return theta0 * 0.5 ** level


def node_blocks(A: CSR, bs: int):
    """Node graph of a scalar CSR whose pattern consists of full bs x bs blocks, with node
    rows bs*I .. bs*I+bs-1.  Returns (node indptr, node cols, squared Frobenius norms), the
    norm of a block summed row by row, left to right, from +0.0."""
    n = A.shape[0]
    assert n % bs == 0
    nn = n // bs
    lens = np.diff(A.indptr)
    rl = lens.reshape(nn, bs)
    if not np.all(rl == rl[:, :1]) or np.any(rl[:, 0] % bs):
        raise ValueError("nodal AMG needs full bs x bs blocks")
    nblk = rl[:, 0] // bs
    nptr = np.zeros(nn + 1, dtype=np.int64)
    np.cumsum(nblk, out=nptr[1:])
    first_rows = np.arange(nn) * bs
    ncols = np.empty(nptr[-1], dtype=np.int64)
    f = np.zeros(nptr[-1])
    for r in range(bs):
        starts = A.indptr[first_rows + r]
        base = np.repeat(starts - bs * nptr[:-1], nblk)
        q = np.arange(nptr[-1], dtype=np.int64)
        pos0 = base + bs * q
        cols = A.indices[pos0]
        if r == 0:
            ncols[:] = cols // bs
        if np.any(cols // bs != ncols) or np.any(cols % bs != 0):
            raise ValueError("nodal AMG needs full bs x bs blocks")
        for c in range(bs):
            if np.any(A.indices[pos0 + c] != cols + c):
                raise ValueError("nodal AMG needs full bs x bs blocks")
            v = A.data[pos0 + c]
            f = f + v * v
    return nptr, ncols, f


def strength_graph(A: CSR, theta: float, bs: int):
    """Symmetrised strength graph (CSR pattern over nodes, no self loops)."""
    if bs == 1:
        r = A.row_ids()
        c = A.indices
        v = A.data
        d = diagonal(A)
        th2 = theta * theta
        off = c != r
        strong = off & (v != 0.0) & (v * v >= th2 * np.abs(d[r] * d[c]))
        nn = A.shape[0]
    else:
        nptr, ncols, f = node_blocks(A, bs)
        nn = nptr.shape[0] - 1
        r = np.repeat(np.arange(nn, dtype=np.int64), np.diff(nptr))
        c = ncols
        fd = np.full(nn, np.nan)
        m = c == r
        fd[r[m]] = f[m]
        th2 = theta * theta
        th4 = th2 * th2
        off = c != r
        strong = off & (f != 0.0) & (f * f >= th4 * (fd[r] * fd[c]))
    er, ec = r[strong], c[strong]
    keys = np.union1d(er * nn + ec, ec * nn + er)
    rows = keys // nn
    gptr = np.zeros(nn + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=nn), out=gptr[1:])
    return gptr, keys % nn


def _row_max(gptr, gcol, vals):
    """out[i] = max(vals[i], max_{j in N(i)} vals[j])."""
    out = vals.copy()
    deg = np.diff(gptr)
    has = deg > 0
    if gcol.shape[0]:
        red = np.maximum.reduceat(vals[gcol], gptr[:-1][has])
        out[has] = np.maximum(out[has], red)
    return out


def _row_any(gptr, gcol, flags):
    return _row_max(gptr, gcol, flags.astype(np.uint8)).astype(bool)


UNDECIDED, SELECTED, REMOVED, ISOLATED = 0, 1, 2, 3


def mis2(gptr, gcol, prio):
    """Distance-2 maximal independent set by synchronous rounds; returns the node states."""
    n = gptr.shape[0] - 1
    state = np.full(n, UNDECIDED, dtype=np.int8)
    state[np.diff(gptr) == 0] = ISOLATED
    while np.any(state == UNDECIDED):
        und = state == UNDECIDED
        pm = np.where(und, prio, np.uint64(0))
        m2 = _row_max(gptr, gcol, _row_max(gptr, gcol, pm))
        new = und & (prio == m2)
        state[new] = SELECTED
        near = _row_any(gptr, gcol, _row_any(gptr, gcol, new))
        state[(state == UNDECIDED) & near] = REMOVED
    return state


def _best_neighbour(gptr, gcol, prio, cand_mask_nbr, want_row):
    """For rows in want_row: the neighbour j with cand_mask_nbr[j] of largest priority, or -1."""
    n = gptr.shape[0] - 1
    r = np.repeat(np.arange(n, dtype=np.int64), np.diff(gptr))
    ok = want_row[r] & cand_mask_nbr[gcol]
    best = np.full(n, -1, dtype=np.int64)
    if np.any(ok):
        rr, jj = r[ok], gcol[ok]
        order = np.lexsort((prio[jj], rr))       # last per row has the largest priority
        rr, jj = rr[order], jj[order]
        last = np.r_[rr[1:] != rr[:-1], True]
        best[rr[last]] = jj[last]
    return best


def aggregate(gptr, gcol, state, prio):
    """Aggregate id per node (-1 = no aggregate) and the number of aggregates."""
    n = gptr.shape[0] - 1
    agg = np.full(n, -1, dtype=np.int64)
    roots = np.flatnonzero(state == SELECTED)
    agg[roots] = np.arange(roots.shape[0])
    eligible = state != ISOLATED
    # pass 1: join a neighbouring root
    want = eligible & (agg < 0)
    best = _best_neighbour(gptr, gcol, prio, state == SELECTED, want)
    sel = best >= 0
    agg[sel] = agg[best[sel]]
    # pass 2: join the aggregate of an aggregated neighbour (aggregates as after pass 1)
    agg1 = agg.copy()
    want = eligible & (agg1 < 0)
    best = _best_neighbour(gptr, gcol, prio, agg1 >= 0, want)
    sel = best >= 0
    agg[sel] = agg1[best[sel]]
    # leftovers: singletons, numbered after the existing aggregates in node order
    left = np.flatnonzero(eligible & (agg < 0))
    nagg = roots.shape[0]
    agg[left] = nagg + np.arange(left.shape[0])
    return agg, nagg + left.shape[0]


def tentative(agg, nagg, bs):
    """T[(node, c), (agg(node), c)] = 1 for aggregated nodes."""
    nn = agg.shape[0]
    rows = (np.arange(nn)[:, None] * bs + np.arange(bs)[None, :]).ravel()
    cols = (agg[:, None] * bs + np.arange(bs)[None, :]).ravel()
    keep = np.repeat(agg >= 0, bs)
    rows, cols = rows[keep], cols[keep]
    indptr = np.zeros(nn * bs + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=nn * bs), out=indptr[1:])
    return CSR(indptr, cols, np.ones(rows.shape[0]), (nn * bs, nagg * bs))


def smoothed_prolongator(A: CSR, T: CSR):
    """P = T - diag(omega / a_ii) (A T), omega = (4/3)/rho, rho = max_i sum_j|a_ij| / |a_ii|."""
    d = diagonal(A)
    if np.any(~np.isfinite(d)) or np.any(d == 0.0):
        raise ZeroPivot("zero or missing diagonal in AMG level matrix")
    rho = np.max(row_sum_abs_sequential(A) / np.abs(d))
    omega = (4.0 / 3.0) / rho
    AT = spgemm(A, T)
    return merge_sub(T, AT, omega / d), omega


@dataclass
class AMGLevel:
    A: CSR
    dinv: np.ndarray | None = None      # 1 / l1 row sums
    P: CSR | None = None
    R: CSR | None = None
    agg: np.ndarray | None = None
    omega: float = 0.0


@dataclass
class AMGHierarchy:
    levels: list = field(default_factory=list)
    lu: tuple | None = None
    opts: AMGOptions = field(default_factory=AMGOptions)


def setup(A: CSR, opts: AMGOptions) -> AMGHierarchy:
    bs = opts.block
    H = AMGHierarchy(opts=opts)
    cur = A
    lvl = 0
    while True:
        n = cur.shape[0]
        L = AMGLevel(A=cur)
        H.levels.append(L)
        if n <= opts.coarse_size or lvl + 1 >= opts.max_levels:
            break
        gptr, gcol = strength_graph(cur, theta_at(opts.theta0, lvl), bs)
        prio = priorities(gptr.shape[0] - 1, lvl)
        state = mis2(gptr, gcol, prio)
        agg, nagg = aggregate(gptr, gcol, state, prio)
        nc = nagg * bs
        if nc == 0 or nc > 0.8 * n:
            break
        T = tentative(agg, nagg, bs)
        P, omega = smoothed_prolongator(cur, T)
        R = transpose(P)
        Ac = spgemm(R, spgemm(cur, P))
        L.P, L.R, L.agg, L.omega = P, R, agg, omega
        cur = Ac
        lvl += 1
    for L in H.levels[:-1]:
        L.dinv = 1.0 / np.add.reduceat(np.abs(L.A.data), L.A.indptr[:-1])
    Ad = H.levels[-1].A.to_dense()
    H.lu = sla.lu_factor(Ad)
    return H


def vcycle(H: AMGHierarchy, b: np.ndarray, lvl: int = 0) -> np.ndarray:
    """One V-cycle for A x = b from x = 0: l1-Jacobi pre-sweep, coarse correction with
    R = P^T, l1-Jacobi post-sweep; dense LU at the coarsest level."""
    if lvl == len(H.levels) - 1:
        return sla.lu_solve(H.lu, b)
    L = H.levels[lvl]
    x = L.dinv * b
    r = b - L.A.matvec(x)
    ec = vcycle(H, L.R.matvec(r), lvl + 1)
    x = x + L.P.matvec(ec)
    x = x + L.dinv * (b - L.A.matvec(x))
    return x
