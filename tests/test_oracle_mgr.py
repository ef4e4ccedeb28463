"""Pins of the oracle's MGR setup and V-cycle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a hand-worked example,
the block LDU factorisation and the MGR identities of Sec. 5.1, the closed form of the
Galerkin coarse grid with injection restriction and Jacobi interpolation (Sec. 5.2), a
brute-force sort for the dropping operator, exactness of the two-grid and multi-level
V-cycle with ideal components, and the block-triangular special case W_p = W_r = 0.
"""
import json
import os

import numpy as np
import pytest

from oracle import krylov, mgr
from oracle.sparse import CSR, spgemm, transpose


def csr_from_dense(D):
    return CSR.from_dense(np.asarray(D, dtype=np.float64))


def random_system(rng, labels, density=0.4, diag_ff=False, dominance=3.0):
    """Random sparse nonsymmetric matrix with a dominant diagonal; if diag_ff, the F block of
    label 0 is diagonal."""
    n = len(labels)
    D = rng.standard_normal((n, n)) * (rng.random((n, n)) < density)
    if diag_ff:
        f = np.flatnonzero(np.asarray(labels) == 0)
        D[np.ix_(f, f)] = 0.0
    D[np.arange(n), np.arange(n)] = dominance * (np.abs(D).sum(axis=1) + 1.0)
    return D


# ---------------------------------------------------------------------------------------
def test_golden_hand_worked(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "mgr_two_level_6x6.json")))
    A = csr_from_dense(g["dense_A"])
    labels = np.array(g["labels"], dtype=np.int8)
    F, C = mgr.cf_split(labels, g["f_labels"])
    assert F.tolist() == g["F"] and C.tolist() == g["C"]
    for nmax_s, exp in g["S"].items():
        plan = mgr.Plan(levels=[mgr.LevelPlan(f_labels=tuple(g["f_labels"]), nmax=int(nmax_s))])
        H = mgr.setup(A, labels, plan)
        L = H.levels[0]
        assert np.array_equal(L.Wp.to_dense(), np.array(g["Wp_dense"], dtype=float))
        assert np.array_equal(L.Acor.to_dense(), np.array(g["Acor_dense"], dtype=float))
        S = H.coarse_A
        for i in range(4):
            cols, vals = S.row(i)
            assert cols.tolist() == exp["rows"][i], (nmax_s, i)
            assert vals.tolist() == [float(v) for v in exp["vals"][i]], (nmax_s, i)


def test_cf_split_and_label_rank():
    labels = np.array([0, 0, 0, 1, 2, 1, 2, 0, 1, 2], dtype=np.int8)
    F, C = mgr.cf_split(labels, (0,))
    assert F.tolist() == [0, 1, 2, 7]
    assert C.tolist() == [3, 4, 5, 6, 8, 9]
    assert mgr.label_rank(labels[C]).tolist() == [0, 0, 1, 1, 2, 2]


def test_ldu_and_ideal_schur():
    """Block LDU factorisation (Sec. 5.1): A = L diag(A_FF, S) U with the Schur complement;
    the oracle's 'ideal' mode must produce exactly that S (up to rounding)."""
    rng = np.random.default_rng(0)
    labels = np.array([0, 1, 0, 1, 0, 1, 1, 0, 1], dtype=np.int8)
    D = random_system(rng, labels, density=0.6)
    A = csr_from_dense(D)
    F, C = mgr.cf_split(labels, (0,))
    Aff, Afc, Acf, Acc = D[np.ix_(F, F)], D[np.ix_(F, C)], D[np.ix_(C, F)], D[np.ix_(C, C)]
    S = Acc - Acf @ np.linalg.solve(Aff, Afc)
    nF, nC = len(F), len(C)
    Lm = np.block([[np.eye(nF), np.zeros((nF, nC))], [Acf @ np.linalg.inv(Aff), np.eye(nC)]])
    Dm = np.block([[Aff, np.zeros((nF, nC))], [np.zeros((nC, nF)), S]])
    Um = np.block([[np.eye(nF), np.linalg.solve(Aff, Afc)], [np.zeros((nC, nF)), np.eye(nC)]])
    perm = np.concatenate([F, C])
    assert np.allclose(Lm @ Dm @ Um, D[np.ix_(perm, perm)], rtol=1e-13, atol=1e-12)
    H = mgr.setup(A, labels, mgr.Plan(levels=[mgr.LevelPlan(f_labels=(0,), interp="ideal")]))
    assert np.allclose(H.coarse_A.to_dense(), S, rtol=1e-12, atol=1e-12)


def test_mgr_identities_ideal_operators():
    """A^{-1} = P (RAP)^{-1} R + Q (Q^T A Q)^{-1} Q^T and RAQ = Q^T AP = 0 (Sec. 5.1), and the
    oracle's two-grid V-cycle with ideal interpolation and exact F-relaxation equals A^{-1}
    (eq. MGR-mul1 with exact factors)."""
    rng = np.random.default_rng(1)
    labels = np.array([0, 1, 1, 0, 0, 1, 0, 1], dtype=np.int8)
    D = random_system(rng, labels, density=0.5)
    F, C = mgr.cf_split(labels, (0,))
    perm = np.concatenate([F, C])
    Ap = D[np.ix_(perm, perm)]
    nF, nC = len(F), len(C)
    Aff, Afc, Acf = Ap[:nF, :nF], Ap[:nF, nF:], Ap[nF:, :nF]
    P = np.vstack([-np.linalg.solve(Aff, Afc), np.eye(nC)])
    R = np.hstack([-Acf @ np.linalg.inv(Aff), np.eye(nC)])
    Q = np.vstack([np.eye(nF), np.zeros((nC, nF))])
    inv = P @ np.linalg.inv(R @ Ap @ P) @ R + Q @ np.linalg.inv(Q.T @ Ap @ Q) @ Q.T
    assert np.allclose(inv, np.linalg.inv(Ap), atol=1e-12)
    assert np.allclose(R @ Ap @ Q, 0.0, atol=1e-12)
    assert np.allclose(Q.T @ Ap @ P, 0.0, atol=1e-12)
    plan = mgr.Plan(levels=[mgr.LevelPlan(f_labels=(0,), interp="ideal", frelax="exact")])
    H = mgr.setup(csr_from_dense(D), labels, plan)
    Minv = np.column_stack([mgr.apply(H, e) for e in np.eye(len(labels))])
    assert np.linalg.norm(Minv @ D - np.eye(len(labels))) <= 1e-12


def test_rap_closed_form_and_dense_triple_product():
    """With W_r = 0 and W_p = -D_FF^{-1} A_FC, R~ A P~ = A_CC - A_CF D_FF^{-1} A_FC (Sec. 5.2);
    checked against a dense triple product built from the definitions of eq. RPoperator1."""
    rng = np.random.default_rng(2)
    labels = rng.integers(0, 3, size=40).astype(np.int8)
    D = random_system(rng, labels, density=0.15)
    A = csr_from_dense(D)
    H = mgr.setup(A, labels, mgr.Plan(levels=[mgr.LevelPlan(f_labels=(0,), nmax=-1)]))
    F, C = mgr.cf_split(labels, (0,))
    perm = np.concatenate([F, C])
    Ap = D[np.ix_(perm, perm)]
    nF, nC = len(F), len(C)
    dff = np.diag(Ap[:nF, :nF])
    Wp = -Ap[:nF, nF:] / dff[:, None]
    Pt = np.vstack([Wp, np.eye(nC)])
    Rt = np.hstack([np.zeros((nC, nF)), np.eye(nC)])
    rap = Rt @ Ap @ Pt
    closed = Ap[nF:, nF:] - Ap[nF:, :nF] @ np.diag(1.0 / dff) @ Ap[:nF, nF:]
    S = H.coarse_A.to_dense()
    assert np.allclose(S, rap, rtol=1e-14, atol=1e-13)
    assert np.allclose(S, closed, rtol=1e-14, atol=1e-13)
    # pattern: union of A_CC and the boolean product pattern
    pat = (Ap[nF:, nF:] != 0) | ((Ap[nF:, :nF] != 0).astype(int) @ (Ap[:nF, nF:] != 0).astype(int) > 0)
    Spat = np.zeros((nC, nC), dtype=bool)
    Spat[H.coarse_A.row_ids(), H.coarse_A.indices] = True
    assert np.array_equal(Spat, pat)


def test_zero_interpolation_gives_acc():
    """W_p = W_r = 0 gives R A P = A_CC (Sec. 5.1, the first extreme)."""
    rng = np.random.default_rng(3)
    labels = rng.integers(0, 2, size=30).astype(np.int8)
    D = random_system(rng, labels, density=0.2)
    H = mgr.setup(csr_from_dense(D), labels,
                  mgr.Plan(levels=[mgr.LevelPlan(f_labels=(0,), interp="zero")]))
    F, C = mgr.cf_split(labels, (0,))
    assert np.array_equal(H.coarse_A.to_dense(), D[np.ix_(C, C)])


def test_block_lower_triangular_special_case():
    """W_p = W_r = 0 with exact F and coarse solves makes M the block lower-triangular part
    [[A_FF, 0], [A_CF, A_CC]] (Algorithm 1 with z_C = 0 before the correction)."""
    rng = np.random.default_rng(4)
    labels = rng.integers(0, 2, size=24).astype(np.int8)
    D = random_system(rng, labels, density=0.3)
    plan = mgr.Plan(levels=[mgr.LevelPlan(f_labels=(0,), interp="zero", frelax="exact")])
    H = mgr.setup(csr_from_dense(D), labels, plan)
    F, C = mgr.cf_split(labels, (0,))
    Mb = D.copy()
    Mb[np.ix_(F, C)] = 0.0
    v = rng.standard_normal(len(labels))
    assert np.allclose(mgr.apply(H, v), np.linalg.solve(Mb, v), rtol=1e-12, atol=1e-14)


def _brute_drop(Acor: CSR, labels_c, nmax):
    rank = mgr.label_rank(labels_c)
    out = {}
    for i in range(Acor.shape[0]):
        cols, vals = Acor.row(i)
        prot = [(c, v) for c, v in zip(cols, vals) if rank[c] == rank[i]]
        rest = sorted([(c, v) for c, v in zip(cols, vals) if rank[c] != rank[i]],
                      key=lambda cv: (-abs(cv[1]), cv[0]))
        kept = sorted(prot + (rest[:nmax] if nmax >= 0 else rest))
        out[i] = kept
    return out


@pytest.mark.parametrize("nmax", [0, 1, 2, 4, 100, -1])
def test_drop_bruteforce(nmax):
    """Dropping operator G (eq. drop_operator) against a brute-force sort, with many ties."""
    rng = np.random.default_rng(10 + max(nmax, 0))
    nC = 60
    labels_c = np.tile(np.array([1, 2], dtype=np.int8), nC // 2)
    D = rng.integers(-3, 4, size=(nC, nC)).astype(float) * (rng.random((nC, nC)) < 0.3)
    mask = (D != 0) | (rng.random((nC, nC)) < 0.05)       # some explicit zeros
    Acor = CSR.from_dense(D, mask)
    G = mgr.drop(Acor, labels_c, nmax)
    bf = _brute_drop(Acor, labels_c, nmax)
    for i in range(nC):
        cols, vals = G.row(i)
        assert list(zip(cols.tolist(), vals.tolist())) == [(int(c), float(v)) for c, v in bf[i]]


def test_drop_extremes_block_diagonal():
    """N_max = 0 leaves a 2x2 block matrix whose sub-blocks are diagonal (Sec. 5.2);
    N_max = infinity leaves A_cor unchanged."""
    rng = np.random.default_rng(5)
    nC = 40
    labels_c = np.tile(np.array([1, 2], dtype=np.int8), nC // 2)
    D = rng.standard_normal((nC, nC))
    Acor = CSR.from_dense(D)
    G0 = mgr.drop(Acor, labels_c, 0).to_dense()
    s = np.arange(0, nC, 2)
    p = np.arange(1, nC, 2)
    for bi in (s, p):
        for bj in (s, p):
            blk = G0[np.ix_(bi, bj)]
            assert np.array_equal(blk, np.diag(np.diag(blk)))
            assert np.all(np.diag(blk) == np.diag(D[np.ix_(bi, bj)]))
    assert np.array_equal(mgr.drop(Acor, labels_c, 10 ** 6).to_dense(), D)


def test_drop_tolerance_by_hand():
    """Tolerance form of G (Sec. 5.2), worked by hand on one row of a two-label coarse grid:
    the sub-block diagonal entries (columns of the same per-label rank as the row: its own
    diagonal and the same-cell entry of the other label) are kept whatever their size, the
    others when nonzero and at least tol times the row's largest |value| (2.0 here)."""
    labels_c = np.array([1, 2, 1, 2, 1, 2], dtype=np.int8)   # ranks 0 0 1 1 2 2
    # row 0 (label 1, rank 0): columns 0 and 1 have rank 0
    D = np.array([[0.1, 0.01, -2.0, 0.5, 1.9, 0.0]] + [[0.0] * 6] * 5)
    mask = np.zeros_like(D, dtype=bool)
    mask[0, :] = True                                           # an explicit zero at (0, 5)
    Acor = CSR.from_dense(D, mask)
    row = lambda G: G.row(0)[0].tolist()                        # noqa: E731
    assert row(mgr.drop(Acor, labels_c, -1, tol=0.5)) == [0, 1, 2, 4]       # >= 1.0
    assert row(mgr.drop(Acor, labels_c, -1, tol=0.25)) == [0, 1, 2, 3, 4]   # >= 0.5
    assert row(mgr.drop(Acor, labels_c, -1, tol=0.0)) == [0, 1, 2, 3, 4]    # nonzeros
    assert row(mgr.drop(Acor, labels_c, -1, tol=0.95)) == [0, 1, 2, 4]      # >= 1.9: equal kept
    assert row(mgr.drop(Acor, labels_c, -1, tol=1.0)) == [0, 1, 2]          # >= 2.0
    assert row(mgr.drop(Acor, labels_c, -1, tol=1.5)) == [0, 1]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_drop_tolerance_limits_and_nesting(seed):
    """A tolerance above 1 keeps exactly what N_max = 0 keeps (the paper's 'extremely large
    tolerance'); tolerance 0 keeps what N_max = infinity keeps except explicit zeros; a
    larger tolerance keeps a subset."""
    rng = np.random.default_rng(40 + seed)
    nC = 50
    labels_c = np.tile(np.array([1, 2], dtype=np.int8), nC // 2)
    D = rng.standard_normal((nC, nC)) * (rng.random((nC, nC)) < 0.3)
    mask = (D != 0) | (rng.random((nC, nC)) < 0.05)
    Acor = CSR.from_dense(D, mask)
    for big in (1.0000001, 2.0, 1e300):
        assert np.array_equal(mgr.drop(Acor, labels_c, -1, tol=big).to_dense(),
                              mgr.drop(Acor, labels_c, 0).to_dense())
    G0 = mgr.drop(Acor, labels_c, -1, tol=0.0)
    prot = mgr.label_rank(labels_c)[Acor.indices] == mgr.label_rank(labels_c)[Acor.row_ids()]
    assert G0.nnz == int(np.count_nonzero((Acor.data != 0) | prot))
    assert np.array_equal(G0.to_dense(), D)
    prev = None
    for tol in (0.0, 0.1, 0.3, 0.6, 0.9):
        G = mgr.drop(Acor, labels_c, -1, tol=tol)
        kept = set(zip(G.row_ids().tolist(), G.indices.tolist()))
        if prev is not None:
            assert kept <= prev
        prev = kept


def test_jp_coloring_by_hand():
    """Jones-Plassmann rounds worked by hand: a path 0-1-2-3 with falling priorities colours
    0, then 1 (beside colour 0), then 2, then 3: 0 1 0 1; a star whose centre has the lowest
    priority colours the four leaves first (0) and the centre last (1); equal priorities
    fall back to the larger index."""
    path = (np.array([0, 1, 3, 5, 6]), np.array([1, 0, 2, 1, 3, 2]))
    assert mgr.jp_coloring(*path, np.array([4, 3, 2, 1], dtype=np.uint64)).tolist() == [0, 1, 0, 1]
    star = (np.array([0, 4, 5, 6, 7, 8]), np.array([1, 2, 3, 4, 0, 0, 0, 0]))
    assert mgr.jp_coloring(*star, np.array([1, 5, 4, 3, 2], dtype=np.uint64)).tolist() == \
        [1, 0, 0, 0, 0]
    tri = (np.array([0, 1, 3, 4]), np.array([1, 0, 2, 1]))
    assert mgr.jp_coloring(*tri, np.zeros(3, dtype=np.uint64)).tolist() == [0, 1, 0]


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_jp_coloring_is_proper(seed):
    """Every vertex gets a colour, no edge joins two of one colour, and at most
    (largest degree + 1) colours are used, on random symmetric graphs."""
    rng = np.random.default_rng(seed)
    n = 300
    Dg = rng.random((n, n)) < 0.03
    Dg = np.triu(Dg, 1)
    Dg = Dg | Dg.T
    gptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(Dg.sum(1), out=gptr[1:])
    gcol = np.nonzero(Dg)[1]
    col = mgr.jp_coloring(gptr, gcol, mgr.cell_priorities(n))
    assert np.all(col >= 0)
    i, j = np.nonzero(Dg)
    assert np.all(col[i] != col[j])
    assert col.max() + 1 <= Dg.sum(1).max() + 1


def _interleaved_block_system(rng, ncell, nb=2, dens=0.05):
    """A block diagonally dominant matrix on ncell cells of nb interleaved unknowns with a
    non-symmetric pattern, and its labels."""
    n = ncell * nb
    D = rng.standard_normal((n, n)) * (rng.random((n, n)) < dens)
    for e in range(ncell):
        r = slice(e * nb, (e + 1) * nb)
        D[r, r] = rng.standard_normal((nb, nb)) + np.eye(nb) * (np.abs(D).sum(1).max() + 1.0)
    labels = np.tile(np.arange(1, nb + 1, dtype=np.int8), ncell)
    return D, labels


def test_cell_graph_is_the_symmetrised_block_pattern():
    rng = np.random.default_rng(7)
    D, labels = _interleaved_block_system(rng, 40)
    A = CSR.from_dense(D)
    gptr, gcol = mgr.cell_graph(A, labels)
    B = np.zeros((40, 40), dtype=bool)
    for e in range(40):
        for f in range(40):
            B[e, f] = e != f and np.any(D[2 * e:2 * e + 2, 2 * f:2 * f + 2] != 0)
    B = B | B.T
    got = np.zeros_like(B)
    for e in range(40):
        got[e, gcol[gptr[e]:gptr[e + 1]]] = True
    assert np.array_equal(got, B)


def test_block_gs_sweep_equals_sequential_block_gauss_seidel():
    """One multicolour sweep is textbook block Gauss-Seidel with the cells visited in
    (colour, index) order; many sweeps converge to A^{-1} v."""
    from types import SimpleNamespace
    rng = np.random.default_rng(11)
    ncell = 60
    D, labels = _interleaved_block_system(rng, ncell, dens=0.04)
    A = CSR.from_dense(D)
    colors = mgr.jp_coloring(*mgr.cell_graph(A, labels), mgr.cell_priorities(ncell))
    L = SimpleNamespace(A=A, blocks=mgr.same_cell_blocks(A, labels), colors=colors)
    v = rng.standard_normal(2 * ncell)
    z1 = mgr._block_gs(L, v, 1)
    z = np.zeros_like(v)                                   # textbook form, cell by cell
    for e in sorted(range(ncell), key=lambda e: (colors[e], e)):
        r = slice(2 * e, 2 * e + 2)
        z[r] = z[r] + np.linalg.solve(D[r, r], v[r] - D[r, :] @ z)
    assert np.allclose(z1, z, rtol=1e-13, atol=1e-14)
    assert np.allclose(mgr._block_gs(L, v, 60), np.linalg.solve(D, v), rtol=1e-10, atol=1e-12)


def test_spgemm_pinned_order_by_hand():
    """Products are summed in ascending k from +0.0: (0 + 1e16) + 1 + (-1e16) = 0 in binary64
    (1e16 + 1 rounds back to 1e16), whereas summing the last two first would give 1."""
    A = CSR([0, 3], [0, 1, 2], [1.0, 1.0, 1.0], (1, 3))
    B = CSR([0, 1, 2, 3], [0, 0, 0], [1e16, 1.0, -1e16], (3, 1))
    C = spgemm(A, B)
    assert C.indices.tolist() == [0] and C.data.tolist() == [0.0]
    B2 = CSR([0, 1, 2, 3], [0, 0, 0], [1.0, 1e16, -1e16], (3, 1))
    assert spgemm(A, B2).data.tolist() == [0.0]      # (1 + 1e16) - 1e16 = 0 as well
    B3 = CSR([0, 1, 2, 3], [0, 0, 0], [1e16, -1e16, 1.0], (3, 1))
    assert spgemm(A, B3).data.tolist() == [1.0]


def test_spgemm_and_transpose_against_dense():
    rng = np.random.default_rng(6)
    Da = rng.standard_normal((30, 25)) * (rng.random((30, 25)) < 0.2)
    Db = rng.standard_normal((25, 35)) * (rng.random((25, 35)) < 0.2)
    A, B = CSR.from_dense(Da), CSR.from_dense(Db)
    C = spgemm(A, B)
    assert np.allclose(C.to_dense(), Da @ Db, rtol=1e-14, atol=1e-14)
    pat = ((Da != 0).astype(int) @ (Db != 0).astype(int)) > 0
    Cp = np.zeros(pat.shape, dtype=bool)
    Cp[C.row_ids(), C.indices] = True
    assert np.array_equal(Cp, pat)
    At = transpose(A)
    assert np.array_equal(At.to_dense(), Da.T)
    assert all(np.all(np.diff(At.row(i)[0]) > 0) for i in range(At.shape[0]))


def test_exactness_two_level_and_fgmres_one_iteration():
    """With A_FF diagonal, Jacobi interpolation is the ideal one and one Jacobi sweep with
    omega = 1 is an exact F-relaxation; with no dropping and an exact coarse solve the
    presmoothed two-grid operator is A^{-1}, so FGMRES converges in one iteration."""
    rng = np.random.default_rng(7)
    labels = rng.integers(0, 2, size=50).astype(np.int8)
    D = random_system(rng, labels, density=0.2, diag_ff=True)
    A = csr_from_dense(D)
    plan = mgr.Plan(levels=[mgr.LevelPlan(f_labels=(0,), nmax=-1, frelax="jacobi")], coarse="dense")
    H = mgr.setup(A, labels, plan)
    Minv = np.column_stack([mgr.apply(H, e) for e in np.eye(50)])
    assert np.linalg.norm(Minv @ D - np.eye(50)) <= 1e-12
    F, C = mgr.cf_split(labels, (0,))
    S = D[np.ix_(C, C)] - D[np.ix_(C, F)] @ np.linalg.solve(D[np.ix_(F, F)], D[np.ix_(F, C)])
    assert np.allclose(H.coarse_A.to_dense(), S, rtol=1e-13, atol=1e-13)
    b = rng.standard_normal(50)
    res = krylov.fgmres(A.matvec, lambda v: mgr.apply(H, v), b, restart=30, rtol=1e-10)
    assert res.converged and res.iters == 1


def test_exactness_multilevel_by_induction():
    """Three labels, two reductions with ideal interpolation and exact F-relaxation, dense
    coarsest solve: the multi-level V-cycle of Algorithm 2 is exactly A^{-1}."""
    rng = np.random.default_rng(8)
    labels = rng.integers(0, 3, size=36).astype(np.int8)
    D = random_system(rng, labels, density=0.3)
    plan = mgr.Plan(levels=[mgr.LevelPlan(f_labels=(0,), interp="ideal", frelax="exact"),
                            mgr.LevelPlan(f_labels=(1,), interp="ideal", frelax="exact")])
    H = mgr.setup(csr_from_dense(D), labels, plan)
    Minv = np.column_stack([mgr.apply(H, e) for e in np.eye(36)])
    assert np.linalg.norm(Minv @ D - np.eye(36)) <= 1e-11


def test_global_smoother_blocks_exact_on_block_diagonal():
    """Block Jacobi over same-cell blocks inverts a matrix that is block diagonal by cells."""
    rng = np.random.default_rng(9)
    ncell = 12
    labels = np.tile(np.array([1, 2], dtype=np.int8), ncell)
    D = np.zeros((2 * ncell, 2 * ncell))
    for c in range(ncell):
        D[2 * c:2 * c + 2, 2 * c:2 * c + 2] = rng.standard_normal((2, 2)) + 3 * np.eye(2)
    rows, inv = mgr.same_cell_blocks(csr_from_dense(D), labels)
    v = rng.standard_normal(2 * ncell)
    z = np.zeros_like(v)
    z[rows] = np.einsum("eij,ej->ei", inv, v[rows])
    assert np.allclose(D @ z, v, rtol=1e-13, atol=1e-13)


def test_zero_pivot_detected():
    """A zero on the diagonal of A_FF is reported, not skipped."""
    D = np.array([[0.0, 1.0], [1.0, 2.0]])
    A = CSR.from_dense(D, np.ones((2, 2), dtype=bool))
    with pytest.raises(mgr.ZeroPivot):
        mgr.setup(A, np.array([0, 1], dtype=np.int8), mgr.Plan(levels=[mgr.LevelPlan(f_labels=(0,))]))


def test_quasi_impes_closed_form():
    """Quasi-IMPES coupling (the alternative described beside eq. coarse_grid_pressure):
    in field order the coarse grid is A_pp - D_ps D_ss^{-1} A_sp with D_ps = diag(A_ps),
    D_ss = diag(A_ss).  Rows are interleaved cell by cell (s, p, s, p, ...), so "diag"
    pairs the s and p unknowns of one cell.  The full coupling gives A_pp - A_ps D_ss^{-1}
    A_sp instead, which must differ."""
    rng = np.random.default_rng(7)
    ncell = 7
    labels = np.tile(np.array([1, 2], dtype=np.int8), ncell)
    D = random_system(rng, labels, density=0.5)
    A = csr_from_dense(D)
    s_idx, p_idx = np.arange(0, 2 * ncell, 2), np.arange(1, 2 * ncell, 2)
    Ass, Asp = D[np.ix_(s_idx, s_idx)], D[np.ix_(s_idx, p_idx)]
    Aps, App = D[np.ix_(p_idx, s_idx)], D[np.ix_(p_idx, p_idx)]
    dss, dps = np.diag(Ass), np.diag(Aps)
    want_qi = App - (dps / dss)[:, None] * Asp
    want_full = App - Aps @ (Asp / dss[:, None])
    got = {}
    for coupling in ("quasi_impes", "full"):
        plan = mgr.Plan(levels=[mgr.LevelPlan(f_labels=(1,), coupling=coupling)], coarse="dense")
        got[coupling] = mgr.setup(A, labels, plan).coarse_A.to_dense()
    scale = np.abs(App).max() + np.abs(Asp).max()
    assert np.allclose(got["quasi_impes"], want_qi, rtol=0, atol=1e-13 * scale)
    assert np.allclose(got["full"], want_full, rtol=0, atol=1e-13 * scale)
    assert not np.allclose(got["quasi_impes"], got["full"], rtol=0, atol=1e-6 * scale)
    # W_p is the same under both couplings (only the coarse product changes)
    plan = mgr.Plan(levels=[mgr.LevelPlan(f_labels=(1,), coupling="quasi_impes")], coarse="dense")
    Wp = mgr.setup(A, labels, plan).levels[0].Wp.to_dense()
    assert np.allclose(Wp, -Asp / dss[:, None], rtol=0, atol=1e-15 * np.abs(Asp).max())
