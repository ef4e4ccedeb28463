"""Multigrid reduction (MGR) setup and V-cycle, FP64 on the CPU (test infrastructure, see
the package docstring).

Follows Sec. 5 of the paper:
  * C/F splitting of the rows into disjoint sets (Sec. 5.1), chosen per level by unknown
    type (Sec. 5.3);
  * approximate interpolation P~ = [W_p; I] and restriction R~ = [W_r, I] (eq. RPoperator1)
    with injection W_r = 0 and Jacobi interpolation W_p = -D_FF^{-1} A_FC, D_FF = diag(A_FF)
    (eq. injective_rp);
  * coarse grid R~ A P~ = A_CC - A_CF D_FF^{-1} A_FC (Sec. 5.2), made sparse by the dropping
    operator G, which keeps the N_max largest entries per row of the correction term plus
    the diagonals of its sub-blocks (eq. drop_operator);
  * the multi-level V-cycle with global relaxation, F-relaxation, restriction, recursion,
    interpolation and correction (Algorithm 2, the recursive form of Algorithm 1).

Readings where the paper is silent (each also listed in the design notes):
  * F and C index lists are ascending, so interleaved orderings stay interleaved;
  * a zero or structurally missing D_FF entry is an error (ZeroPivot);
  * "diagonals of the sub-blocks": entries (i, j) of the correction term whose coarse
    points i and j have the same rank among the coarse points of their own label (the same
    cell); they are kept in addition to the N_max largest;
  * ranking is by |value|, ties to the smaller column; dropped entries are discarded;
  * N_max < 0 means no dropping (Galerkin coarse grid);
  * the residual in the F-relaxation step of Algorithm 2 uses the level's own matrix A_l;
  * the global smoother is block Jacobi over the same-cell blocks (a stand-in for the
    ILU/Gauss-Seidel smoothers of Sec. 5.3): first sweep z = D_B^{-1} v, later sweeps
    z += omega D_B^{-1} (v - A z);
  * the quasi-IMPES option keeps, of A_CF, only the same-entity entries in the coarse
    product ("its diagonal" under the field-ordered view of Sec. 5.3);
  * the ILU global smoother (the paper's pointwise ILU(1)) is the fine-grained ILU(k) of
    ilu.py on the whole level matrix (one GPU has no processor-local blocks) after left
    scaling by the inverses of the same-cell diagonal blocks, D_B^{-1} A (the scaled
    product taken with the pinned order of sparse.spgemm): in SI units the pressure rows'
    own entries are 10^4-10^7 times smaller than their saturation entries, and pointwise
    pivots on the unscaled rows make the factorisation unstable.  First step
    z = (LU)^{-1} D_B^{-1} v, later steps z += omega (LU)^{-1} D_B^{-1} (v - A z).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from . import amg as amg_mod
from . import ilu as ilu_mod
from .sparse import CSR, diagonal, merge_sub, spgemm, submatrix


class ZeroPivot(ArithmeticError):
    pass


@dataclass
class LevelPlan:
    f_labels: tuple                  # labels that are F-points at this level
    interp: str = "jacobi"           # 'jacobi' (eq. injective_rp) | 'zero' | 'ideal' (dense)
    nmax: int = -1                   # N_max of G; < 0: no dropping
    frelax: str = "jacobi"           # 'jacobi' | 'amg' | 'exact' (dense)
    frelax_sweeps: int = 1
    frelax_omega: float = 1.0
    frelax_block: int = 1            # 3: nodal AMG on the F block
    global_smoother: str = "none"    # 'none' | 'block_jacobi' | 'block_gs'
    global_sweeps: int = 1
    global_omega: float = 1.0
    coupling: str = "full"           # 'full' | 'quasi_impes' (A_CF of the coarse product)
    drop_tol: float = -1.0           # >= 0: tolerance form of G instead of nmax
    ilu_level: int = 1               # global_smoother 'ilu': ILU(k) pattern
    ilu_sweeps: int = 3              # fixed-point sweeps of the factorisation
    ilu_tri_sweeps: int = 3          # Jacobi sweeps per triangular solve (< 0: exact)
    restrict: str = "injection"      # 'injection' (W_r = 0) | 'jacobi' (W_r = -A_CF D_FF^-1)
    dff_block: int = 1               # D_FF: pointwise (1) or diagonal blocks of 2 or 3 F rows


@dataclass
class Plan:
    levels: list
    coarse: str = "dense"            # 'dense' | 'amg'
    amg_frelax: amg_mod.AMGOptions = field(default_factory=lambda: amg_mod.AMGOptions(block=3))
    amg_coarse: amg_mod.AMGOptions = field(default_factory=amg_mod.AMGOptions)


@dataclass
class Level:
    A: CSR
    labels: np.ndarray
    F: np.ndarray
    C: np.ndarray
    dFF: np.ndarray
    A_FF: CSR
    A_FC: CSR
    A_CF: CSR
    A_CC: CSR
    Wp: CSR                     # W_p (F rows x C cols)
    Acor: CSR                   # the correction term of the coarse grid before dropping:
                                # A_CF D_FF^{-1} A_FC (injection) or, with Jacobi
                                # restriction, A_CF M + N A_FC - N A_FF M
                                # (M = D_FF^{-1} A_FC, N = A_CF D_FF^{-1})
    G: CSR                      # G(A_cor)
    plan: LevelPlan
    amg: object = None          # F-relaxation AMG hierarchy
    ff_lu: tuple | None = None  # F-relaxation dense LU ('exact')
    blocks: tuple | None = None # global smoother: (rows per block, block inverses)
    colors: np.ndarray | None = None  # block Gauss-Seidel: colour of every cell
    ilu: object = None          # global smoother 'ilu': the incomplete factors
    Wr: CSR | None = None       # W_r = -A_CF D_FF^{-1} (Jacobi restriction)
    dff_inv: np.ndarray | None = None  # block D_FF: inverses of the F-row blocks


@dataclass
class Hierarchy:
    levels: list
    coarse_A: CSR
    coarse_labels: np.ndarray
    coarse_lu: tuple | None = None
    coarse_amg: object = None
    plan: Plan | None = None


def cf_split(labels: np.ndarray, f_labels) -> tuple:
    """F = rows whose label is in f_labels, C = the rest; both ascending."""
    isF = np.isin(labels, np.asarray(f_labels, dtype=labels.dtype))
    return np.flatnonzero(isF), np.flatnonzero(~isF)


def label_rank(labels: np.ndarray) -> np.ndarray:
    """rank[x] = number of points before x that carry the same label as x."""
    rank = np.empty(labels.shape[0], dtype=np.int64)
    for lab in np.unique(labels):
        idx = np.flatnonzero(labels == lab)
        rank[idx] = np.arange(idx.shape[0])
    return rank


def blocks_of(A: CSR, F, C):
    n = A.shape[0]
    fmap = np.full(n, -1, dtype=np.int64)
    cmap = np.full(n, -1, dtype=np.int64)
    fmap[F] = np.arange(F.shape[0])
    cmap[C] = np.arange(C.shape[0])
    nF, nC = F.shape[0], C.shape[0]
    return (submatrix(A, F, fmap, nF), submatrix(A, F, cmap, nC),
            submatrix(A, C, fmap, nF), submatrix(A, C, cmap, nC))


def jacobi_interpolation(A_FC: CSR, dFF: np.ndarray) -> tuple:
    """M = D_FF^{-1} A_FC entrywise (m_kj = a_kj / d_k) and W_p = -M (eq. injective_rp)."""
    r = A_FC.row_ids()
    m = A_FC.data / dFF[r]
    M = CSR(A_FC.indptr, A_FC.indices, m, A_FC.shape)
    Wp = CSR(A_FC.indptr, A_FC.indices, -m, A_FC.shape)
    return M, Wp


def coupling_block(A_CF: CSR, labels: np.ndarray, F, C, coupling: str) -> CSR:
    """The C-F block that enters the coarse product A_CF D_FF^{-1} A_FC.

    'full' keeps A_CF (eq. coarse_grid_pressure).  'quasi_impes' replaces it by its diagonal,
    as the quasi-IMPES reduction described beside that equation does: only the entries
    (i, k) whose C-point C[i] and F-point F[k] are the same entity, i.e. have the same rank
    among the points of their own label (the same cell under cell-wise ordering).  W_p and
    the residual still use the whole block."""
    if coupling == "full":
        return A_CF
    if coupling != "quasi_impes":
        raise ValueError(coupling)
    rank = label_rank(np.asarray(labels))
    r = A_CF.row_ids()
    keep = rank[np.asarray(C)[r]] == rank[np.asarray(F)[A_CF.indices]]
    indptr = np.zeros(A_CF.shape[0] + 1, dtype=np.int64)
    np.cumsum(np.bincount(r[keep], minlength=A_CF.shape[0]), out=indptr[1:])
    return CSR(indptr, A_CF.indices[keep], A_CF.data[keep], A_CF.shape)


def drop(Acor: CSR, labels_c: np.ndarray, nmax: int, tol: float = -1.0) -> CSR:
    """The dropping operator G of eq. drop_operator: per row, keep the entries on the
    diagonals of the sub-blocks (same per-label rank) and the nmax largest |values| among
    the rest (ties to the smaller column).  nmax < 0 keeps everything.

    tol >= 0 selects the tolerance form the paper names beside it (Sec. 5.2) instead: an
    entry off the sub-block diagonals is kept when it is nonzero and its |value| is at least
    tol times the largest |value| of its row; the sub-block diagonals are always kept, so a
    tolerance above 1 keeps exactly what nmax = 0 keeps."""
    if tol >= 0:
        rank = label_rank(labels_c)
        r = Acor.row_ids()
        c = Acor.indices
        prot = rank[c] == rank[r]
        absv = np.abs(Acor.data)
        rowmax = np.zeros(Acor.shape[0])
        np.maximum.at(rowmax, r, absv)
        thr = tol * rowmax
        keep = prot | ((absv > 0.0) & (absv >= thr[r]))
        kr = r[keep]
        indptr = np.zeros(Acor.shape[0] + 1, dtype=np.int64)
        np.cumsum(np.bincount(kr, minlength=Acor.shape[0]), out=indptr[1:])
        return CSR(indptr, c[keep], Acor.data[keep], Acor.shape)
    if nmax < 0:
        return Acor
    rank = label_rank(labels_c)
    r = Acor.row_ids()
    c = Acor.indices
    prot = rank[c] == rank[r]
    idx = np.flatnonzero(~prot)
    keep = prot.copy()
    if idx.shape[0]:
        order = np.lexsort((c[idx], -np.abs(Acor.data[idx]), r[idx]))
        srt = idx[order]
        rs = r[srt]
        first = np.r_[True, rs[1:] != rs[:-1]]
        start_of = np.maximum.accumulate(np.where(first, np.arange(rs.shape[0]), 0))
        pos_in_row = np.arange(rs.shape[0]) - start_of
        keep[srt[pos_in_row < nmax]] = True
    kr = r[keep]
    indptr = np.zeros(Acor.shape[0] + 1, dtype=np.int64)
    np.cumsum(np.bincount(kr, minlength=Acor.shape[0]), out=indptr[1:])
    return CSR(indptr, c[keep], Acor.data[keep], Acor.shape)


def small_inverse(D: np.ndarray) -> np.ndarray:
    """Inverses of a stack of 1x1, 2x2 or 3x3 matrices by their closed form, the adjugate
    over the determinant: cofactors as differences of two products, the determinant by
    cofactor expansion along the first row ((b00 c00 + b01 c01) + b02 c02), each entry of
    the adjugate divided by it; every operation separately rounded, in this order."""
    nb = D.shape[1]
    B = D.reshape(D.shape[0], nb * nb)
    if nb == 1:
        det = B[:, 0]
        adj = np.ones_like(B)
    elif nb == 2:
        det = B[:, 0] * B[:, 3] - B[:, 1] * B[:, 2]
        adj = np.stack([B[:, 3], -B[:, 1], -B[:, 2], B[:, 0]], axis=1)
    elif nb == 3:
        c00 = B[:, 4] * B[:, 8] - B[:, 5] * B[:, 7]
        c01 = B[:, 5] * B[:, 6] - B[:, 3] * B[:, 8]
        c02 = B[:, 3] * B[:, 7] - B[:, 4] * B[:, 6]
        det = (B[:, 0] * c00 + B[:, 1] * c01) + B[:, 2] * c02
        adj = np.stack([c00, B[:, 2] * B[:, 7] - B[:, 1] * B[:, 8],
                        B[:, 1] * B[:, 5] - B[:, 2] * B[:, 4],
                        c01, B[:, 0] * B[:, 8] - B[:, 2] * B[:, 6],
                        B[:, 2] * B[:, 3] - B[:, 0] * B[:, 5],
                        c02, B[:, 1] * B[:, 6] - B[:, 0] * B[:, 7],
                        B[:, 0] * B[:, 4] - B[:, 1] * B[:, 3]], axis=1)
    else:
        raise ValueError("blocks of 1, 2 or 3 unknowns")
    if np.any(~np.isfinite(det)) or np.any(det == 0.0):
        raise ZeroPivot("singular same-cell block")
    return (adj / det[:, None]).reshape(D.shape)


def same_cell_blocks(A: CSR, labels: np.ndarray):
    """Global-smoother blocks: rows grouped by their per-label rank (one block per cell).
    Returns (rows, inverses): rows[e] lists block e's rows ascending, inverses[e] is the
    inverse of the diagonal block A[rows[e], rows[e]] (small_inverse)."""
    rank = label_rank(labels)
    nblk = int(rank.max()) + 1
    sizes = np.bincount(rank, minlength=nblk)
    if np.any(sizes != sizes[0]):
        raise ValueError("same-cell blocks of unequal size")
    nb = int(sizes[0])
    order = np.lexsort((np.arange(rank.shape[0]), rank))
    rows = order.reshape(nblk, nb)
    slot = np.empty(rank.shape[0], dtype=np.int64)
    slot[rows] = np.arange(nb)[None, :]
    r = A.row_ids()
    c = A.indices
    m = rank[r] == rank[c]
    D = np.zeros((nblk, nb, nb))
    D[rank[r[m]], slot[r[m]], slot[c[m]]] = A.data[m]
    return rows, small_inverse(D)


def ff_block_inverses(A_FF: CSR, nb: int) -> np.ndarray:
    """Inverses (small_inverse) of the diagonal blocks of A_FF made of nb consecutive F rows
    (the three displacement components of a node, in node-major order)."""
    nF = A_FF.shape[0]
    if nF % nb:
        raise ValueError("F rows do not come in blocks of %d" % nb)
    D = np.zeros((nF // nb, nb, nb))
    r = A_FF.row_ids()
    c = A_FF.indices
    m = (r // nb) == (c // nb)
    D[r[m] // nb, r[m] % nb, c[m] % nb] = A_FF.data[m]
    return small_inverse(D)


def block_diagonal(rows: np.ndarray, inv: np.ndarray, n: int) -> CSR:
    """The block-diagonal matrix D_B^{-1} with the dense inverses of the same-cell blocks
    (every entry of a block kept, zeros included)."""
    nb = rows.shape[1]
    r = np.repeat(rows, nb, axis=1).ravel()
    c = np.tile(rows, (1, nb)).ravel()
    return CSR.from_coo(r, c, inv.reshape(-1), (n, n))


def cell_graph(A: CSR, labels: np.ndarray):
    """Graph of the same-cell blocks (cell = per-label rank of a row): cells e != f are
    adjacent when A has an entry between a row of e and a row of f, in either direction.
    Returns (indptr, indices), neighbours ascending."""
    rank = label_rank(labels)
    ncell = int(rank.max()) + 1
    r, c = rank[A.row_ids()], rank[A.indices]
    m = r != c
    pairs = np.concatenate([np.stack([r[m], c[m]], 1), np.stack([c[m], r[m]], 1)])
    pairs = np.unique(pairs, axis=0) if pairs.shape[0] else pairs.reshape(0, 2)
    indptr = np.zeros(ncell + 1, dtype=np.int64)
    np.cumsum(np.bincount(pairs[:, 0], minlength=ncell), out=indptr[1:])
    return indptr, pairs[:, 1].astype(np.int64)


def cell_priorities(ncell: int) -> np.ndarray:
    """Colouring priorities: SplitMix64 of the cell index with a fixed salt."""
    with np.errstate(over="ignore"):
        salt = amg_mod.GOLDEN * np.uint64(977)
        return amg_mod.splitmix64(np.arange(ncell, dtype=np.uint64) ^ salt)


def jp_coloring(gptr: np.ndarray, gcol: np.ndarray, prio: np.ndarray) -> np.ndarray:
    """Jones-Plassmann colouring by synchronous rounds: an uncoloured vertex whose
    (priority, index) exceeds that of every uncoloured neighbour takes the smallest colour
    not used by its neighbours coloured in earlier rounds.  Adjacent vertices never share a
    colour; at most 64 colours."""
    n = gptr.shape[0] - 1
    color = np.full(n, -1, dtype=np.int64)
    src = np.repeat(np.arange(n), np.diff(gptr))
    dst = np.asarray(gcol, dtype=np.int64)
    prio = np.asarray(prio, dtype=np.uint64)
    while np.any(color < 0):
        old = color.copy()
        unc = old < 0
        e = unc[src] & unc[dst]
        beats = (prio[dst[e]] > prio[src[e]]) | ((prio[dst[e]] == prio[src[e]]) &
                                                (dst[e] > src[e]))
        loser = np.zeros(n, dtype=bool)
        loser[src[e][beats]] = True
        win = unc & ~loser
        used = np.zeros(n, dtype=np.uint64)
        ce = unc[src] & ~unc[dst]
        if np.any(old[dst[ce]] >= 64):
            raise ValueError("more than 64 colours")
        np.bitwise_or.at(used, src[ce], np.left_shift(np.uint64(1), old[dst[ce]].astype(np.uint64)))
        free = ~used & (used + np.uint64(1))          # lowest clear bit
        k = np.zeros(n, dtype=np.int64)
        nz = free != 0
        k[nz] = np.log2(free[nz].astype(np.float64)).astype(np.int64)
        if np.any(win & ~nz):
            raise ValueError("more than 64 colours")
        color[win] = k[win]
    return color


def setup(A: CSR, labels: np.ndarray, plan: Plan) -> Hierarchy:
    """Level loop of Sec. 5.2: A_{l+1} = A_CC - G(A_CF D_FF^{-1} A_FC) with labels_{l+1} =
    labels_l[C]; then the coarsest-grid solver (dense LU or AMG)."""
    levels = []
    cur, lab = A, np.asarray(labels)
    for lp in plan.levels:
        F, C = cf_split(lab, lp.f_labels)
        if F.shape[0] == 0 or C.shape[0] == 0:
            raise ValueError("empty F or C set")
        A_FF, A_FC, A_CF, A_CC = blocks_of(cur, F, C)
        d = diagonal(A_FF)
        if np.any(~np.isfinite(d)) or np.any(d == 0.0):
            raise ZeroPivot("zero or missing diagonal in A_FF")
        Dinv = None                              # block D_FF^{-1} as a CSR, when blocked
        dff_inv = None
        if lp.dff_block > 1:
            dff_inv = ff_block_inverses(A_FF, lp.dff_block)
            Dinv = block_diagonal(np.arange(F.shape[0]).reshape(-1, lp.dff_block), dff_inv,
                                  F.shape[0])
        if lp.interp == "jacobi" and Dinv is not None:
            M = spgemm(Dinv, A_FC)                 # block D_FF^{-1} A_FC
            Wp = CSR(M.indptr, M.indices, -M.data, M.shape)
        elif lp.interp == "jacobi":
            M, Wp = jacobi_interpolation(A_FC, d)
        elif lp.interp == "zero":
            M = CSR(np.zeros(F.shape[0] + 1, dtype=np.int64), [], [], A_FC.shape)
            Wp = M
        elif lp.interp == "ideal":          # dense W_p = -A_FF^{-1} A_FC, tiny inputs only
            Md = np.linalg.solve(A_FF.to_dense(), A_FC.to_dense())
            M = CSR.from_dense(Md, np.ones_like(Md, dtype=bool))
            Wp = CSR(M.indptr, M.indices, -M.data, M.shape)
        else:
            raise ValueError(lp.interp)
        Acf_c = coupling_block(A_CF, lab, F, C, lp.coupling)
        Acor = spgemm(Acf_c, M)
        Wr = None
        if lp.restrict == "jacobi":
            # R~ = [W_r I], W_r = -N, N = A_CF D_FF^{-1} (Sec. 5.1, Jacobi restriction): the
            # coarse grid R~ A P~ = A_CC - (A_CF M + N A_FC - N A_FF M)
            if lp.coupling != "full" or lp.interp != "jacobi":
                raise ValueError("Jacobi restriction needs full coupling and Jacobi W_p")
            N = (spgemm(A_CF, Dinv) if Dinv is not None else
                 CSR(A_CF.indptr, A_CF.indices, A_CF.data / d[A_CF.indices], A_CF.shape))
            Wr = CSR(N.indptr, N.indices, -N.data, N.shape)
            B1 = merge_sub(Acor, spgemm(N, A_FC), -np.ones(Acor.shape[0]))   # A_CF M + N A_FC
            Acor = merge_sub(B1, spgemm(spgemm(N, A_FF), M))                  # - N A_FF M
        elif lp.restrict != "injection":
            raise ValueError(lp.restrict)
        G = drop(Acor, lab[C], lp.nmax, lp.drop_tol)
        S = merge_sub(A_CC, G)
        L = Level(A=cur, labels=lab, F=F, C=C, dFF=d, A_FF=A_FF, A_FC=A_FC, A_CF=A_CF,
                  A_CC=A_CC, Wp=Wp, Acor=Acor, G=G, plan=lp, Wr=Wr, dff_inv=dff_inv)
        if lp.frelax == "amg":
            opts = amg_mod.AMGOptions(**{**plan.amg_frelax.__dict__, "block": lp.frelax_block})
            L.amg = amg_mod.setup(A_FF, opts)
        elif lp.frelax == "exact":
            L.ff_lu = sla.lu_factor(A_FF.to_dense())
        if lp.global_smoother in ("block_jacobi", "block_gs", "ilu"):
            L.blocks = same_cell_blocks(cur, lab)
        if lp.global_smoother == "block_gs":
            gptr, gcol = cell_graph(cur, lab)
            L.colors = jp_coloring(gptr, gcol, cell_priorities(gptr.shape[0] - 1))
        if lp.global_smoother == "ilu":
            L.ilu = ilu_mod.ilu_factor(spgemm(block_diagonal(*L.blocks, cur.shape[0]), cur),
                                       lp.ilu_level, lp.ilu_sweeps)
        levels.append(L)
        cur, lab = S, lab[C]
    H = Hierarchy(levels=levels, coarse_A=cur, coarse_labels=lab, plan=plan)
    if plan.coarse == "dense":
        H.coarse_lu = sla.lu_factor(cur.to_dense())
    else:
        H.coarse_amg = amg_mod.setup(cur, plan.amg_coarse)
    return H


def _block_jacobi(L: Level, v: np.ndarray) -> np.ndarray:
    rows, inv = L.blocks
    z = np.zeros_like(v)
    z[rows] = np.einsum("eij,ej->ei", inv, v[rows])
    return z


def _block_gs(L: Level, v: np.ndarray, sweeps: int) -> np.ndarray:
    """Multicolour block Gauss-Seidel from z = 0: per sweep, the cells of each colour in
    ascending colour order take z_e += D_e^{-1} (v - A z)_e with the current z."""
    rows, inv = L.blocks
    z = np.zeros_like(v)
    ncol = int(L.colors.max()) + 1
    for _ in range(sweeps):
        for c in range(ncol):
            cells = np.flatnonzero(L.colors == c)
            R = rows[cells]
            r = v[R] - L.A.matvec(z)[R]
            z[R] = z[R] + np.einsum("eij,ej->ei", inv[cells], r)
    return z


def apply(H: Hierarchy, v: np.ndarray, lvl: int = 0) -> np.ndarray:
    """z = M^{-1} v by Algorithm 2 (presmoothing form, eq. MGR-pre)."""
    if lvl == len(H.levels):
        if H.coarse_lu is not None:
            return sla.lu_solve(H.coarse_lu, v)
        return amg_mod.vcycle(H.coarse_amg, v)
    L = H.levels[lvl]
    lp = L.plan
    A = L.A
    # global relaxation
    if lp.global_smoother == "block_jacobi":
        z = _block_jacobi(L, v)
        for _ in range(lp.global_sweeps - 1):
            z = z + lp.global_omega * _block_jacobi(L, v - A.matvec(z))
    elif lp.global_smoother == "block_gs":
        z = _block_gs(L, v, lp.global_sweeps)
    elif lp.global_smoother == "ilu":
        z = ilu_mod.ilu_solve(L.ilu, _block_jacobi(L, v), lp.ilu_tri_sweeps)
        for _ in range(lp.global_sweeps - 1):
            r = _block_jacobi(L, v - A.matvec(z))
            z = z + lp.global_omega * ilu_mod.ilu_solve(L.ilu, r, lp.ilu_tri_sweeps)
    else:
        z = np.zeros_like(v)
    # F-relaxation: z <- z + Q M_FF^{-1} Q^T (v - A z)
    if lp.frelax == "jacobi" and L.dff_inv is not None:
        nb = lp.dff_block
        for _ in range(lp.frelax_sweeps):
            r = v - A.matvec(z)
            rF = r[L.F].reshape(-1, nb)
            z[L.F] = z[L.F] + lp.frelax_omega * np.einsum("eij,ej->ei", L.dff_inv, rF).ravel()
    elif lp.frelax == "jacobi":
        for _ in range(lp.frelax_sweeps):
            r = v - A.matvec(z)
            z[L.F] = z[L.F] + lp.frelax_omega * (r[L.F] / L.dFF)
    elif lp.frelax == "amg":
        r = v - A.matvec(z)
        z[L.F] = z[L.F] + amg_mod.vcycle(L.amg, r[L.F])
    elif lp.frelax == "exact":
        r = v - A.matvec(z)
        z[L.F] = z[L.F] + sla.lu_solve(L.ff_lu, r[L.F])
    else:
        raise ValueError(lp.frelax)
    # restrict the residual (injection, or R~ = [W_r I]), recurse, interpolate, correct
    r = v - A.matvec(z)
    rC = r[L.C] if L.Wr is None else r[L.C] + L.Wr.matvec(r[L.F])
    eC = apply(H, rC, lvl + 1)
    z[L.F] = z[L.F] + L.Wp.matvec(eC)
    z[L.C] = z[L.C] + eC
    return z
