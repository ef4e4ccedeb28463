"""Pins of the oracle's fine-grained ILU(k) global smoother (oracle/ilu.py): the fill
pattern against its closed form and against the structure of the complete LU, the
fixed-point sweeps against the textbook elimination restricted to the pattern and against
the tridiagonal recursion, the triangular Jacobi sweeps against exact solves, and the MGR
smoother against exact solves where the factorisation is complete."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import ilu
from oracle import krylov as okry
from oracle import mgr as omgr
from oracle.sparse import CSR


def random_sparse(rng, n, density, dominance=2.0):
    D = (rng.random((n, n)) < density) * rng.standard_normal((n, n))
    np.fill_diagonal(D, 0.0)
    D[np.arange(n), np.arange(n)] = dominance * (np.abs(D).sum(axis=1) + 1.0)
    return D


def pattern(M: CSR) -> np.ndarray:
    P = np.zeros(M.shape, dtype=bool)
    P[M.row_ids(), M.indices] = True
    return P


def textbook_ilu(D: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Gaussian elimination (IKJ order) that keeps only the entries in S: the incomplete
    factors stored in one array (unit lower L below the diagonal, U on and above)."""
    n = D.shape[0]
    W = D.copy() * S
    for i in range(1, n):
        for m in range(i):
            if not S[i, m]:
                continue
            W[i, m] = W[i, m] / W[m, m]
            for j in range(m + 1, n):
                if S[i, j] and S[m, j]:
                    W[i, j] = W[i, j] - W[i, m] * W[m, j]
    return W


def factors_dense(F):
    Ls, Us, d = ilu.split_lu(F)
    n = F.S.shape[0]
    return Ls.to_dense() + np.eye(n), Us.to_dense() + np.diag(d)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ilu1_pattern_is_a_plus_one_elimination_step(seed):
    """Level-1 fill: (i, j) is added exactly when some m < min(i, j) has a_im and a_mj in
    the pattern of A, i.e. pattern(ILU(1)) = pattern(A) | pattern(strict_lower(A) @
    strict_upper(A))."""
    rng = np.random.default_rng(seed)
    D = random_sparse(rng, 40, 0.08)
    A = CSR.from_dense(D)
    P = D != 0
    Lp = np.tril(P, -1).astype(int)
    Up = np.triu(P, 1).astype(int)
    expect = P | ((Lp @ Up) > 0)
    assert np.array_equal(pattern(ilu.ilu_pattern(A, 1)), expect)
    assert np.array_equal(pattern(ilu.ilu_pattern(A, 0)), P)
    # levels nest
    P1, P2 = pattern(ilu.ilu_pattern(A, 1)), pattern(ilu.ilu_pattern(A, 2))
    assert np.all(P2 >= P1) and P2.sum() > P1.sum()


def test_ilu_full_fill_pattern_is_the_lu_structure():
    """With k large the pattern is the structure of the complete factors (random values on
    the pattern, columns diagonally dominant so that partial pivoting keeps the order)."""
    rng = np.random.default_rng(3)
    n = 30
    D = random_sparse(rng, n, 0.07, dominance=3.0)
    D = D.T.copy()                       # row dominance -> column dominance
    P, L, U = sla.lu(D)
    assert np.array_equal(P, np.eye(n))
    struct = (np.abs(np.tril(L, -1)) > 0) | (np.abs(U) > 0) | np.eye(n, dtype=bool)
    assert np.array_equal(pattern(ilu.ilu_pattern(CSR.from_dense(D), n)), struct)


def test_ilu0_of_tridiagonal_equals_the_recursion():
    """No fill: ILU(0) is the complete LU, u_ii = b_i - (a_i / u_{i-1,i-1}) c_{i-1}."""
    rng = np.random.default_rng(4)
    n = 25
    a, b, c = rng.standard_normal(n), 4.0 + rng.random(n), rng.standard_normal(n)
    D = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
    F = ilu.ilu_factor(CSR.from_dense(D), 0, 2 * n)
    L, U = factors_dense(F)
    d = np.empty(n)
    l = np.zeros(n)
    d[0] = b[0]
    for i in range(1, n):
        l[i] = a[i] / d[i - 1]
        d[i] = b[i] - l[i] * c[i - 1]
    assert np.array_equal(np.diag(U), d)
    assert np.array_equal(np.diag(L, -1), l[1:])
    assert np.array_equal(np.diag(U, 1), c[:-1])
    assert np.allclose(L @ U, D, rtol=0, atol=1e-14 * np.abs(D).max())


@pytest.mark.parametrize("k", [0, 1, 2])
def test_sweeps_reach_the_textbook_incomplete_factors(k):
    """The dependency graph of the component equations is acyclic with depth <= 2n, so
    2n synchronous sweeps give the incomplete factors of Gaussian elimination restricted to
    the pattern; (LU)_ij = a_ij on the pattern."""
    rng = np.random.default_rng(10 + k)
    n = 36
    D = random_sparse(rng, n, 0.1)
    A = CSR.from_dense(D)
    F = ilu.ilu_factor(A, k, 2 * n)
    S = pattern(F.S)
    W = textbook_ilu(D, S)
    L, U = factors_dense(F)
    got = np.tril(L, -1) + U
    assert np.allclose(got, W, rtol=1e-13, atol=1e-13 * np.abs(D).max())
    R = (L @ U - D)[S]
    assert np.abs(R).max() <= 1e-13 * np.abs(D).max()
    # a single sweep is not yet the fixed point on this matrix
    F1 = ilu.ilu_factor(A, k, 1)
    L1, U1 = factors_dense(F1)
    assert np.abs((L1 @ U1 - D)[S]).max() > 1e-8 * np.abs(D).max()


def test_sweeps_converge_on_a_dominant_matrix():
    """On a diagonally dominant matrix the fixed-point residual falls with every sweep."""
    rng = np.random.default_rng(21)
    D = random_sparse(rng, 60, 0.06, dominance=4.0)
    A = CSR.from_dense(D)
    res = []
    for sw in range(0, 6):
        F = ilu.ilu_factor(A, 1, sw)
        L, U = factors_dense(F)
        res.append(np.abs((L @ U - D)[pattern(F.S)]).max())
    assert all(res[i + 1] < res[i] for i in range(5)), res


def test_complete_factors_with_exact_solves_invert_the_matrix():
    rng = np.random.default_rng(5)
    n = 28
    D = random_sparse(rng, n, 0.1)
    F = ilu.ilu_factor(CSR.from_dense(D), n, 2 * n)
    v = rng.standard_normal(n)
    z = ilu.ilu_solve(F, v, -1)
    assert np.allclose(z, np.linalg.solve(D, v), rtol=1e-12, atol=1e-12)


def test_jacobi_triangular_sweeps_terminate_at_the_exact_solve():
    """L - I and D_U^{-1}(U - D_U) are strictly triangular (nilpotent): n Jacobi sweeps per
    factor give the exact triangular solves; one sweep does not."""
    rng = np.random.default_rng(6)
    n = 24
    D = random_sparse(rng, n, 0.15, dominance=1.2)
    F = ilu.ilu_factor(CSR.from_dense(D), 1, 2 * n)
    v = rng.standard_normal(n)
    exact = ilu.ilu_solve(F, v, -1)
    assert np.allclose(ilu.ilu_solve(F, v, n), exact, rtol=1e-12, atol=1e-12)
    assert not np.allclose(ilu.ilu_solve(F, v, 1), exact, rtol=1e-6, atol=1e-6)
    L, U = factors_dense(F)
    assert np.allclose(exact, np.linalg.solve(U, np.linalg.solve(L, v)), rtol=1e-12, atol=1e-12)


def test_missing_diagonal_is_a_zero_pivot():
    D = np.array([[0.0, 1.0], [1.0, 2.0]])
    with pytest.raises(ilu.ZeroPivot):
        ilu.ilu_factor(CSR.from_dense(D), 0, 1)


def _two_label_system(rng, ncell):
    """Interleaved (label 1, label 2) unknowns per cell, random coupling between cells."""
    n = 2 * ncell
    labels = np.tile(np.array([1, 2], dtype=np.int8), ncell)
    D = random_sparse(rng, n, 0.08)
    return D, labels


@pytest.mark.parametrize("sweeps", [1, 2])
def test_mgr_with_complete_ilu_smoother_is_an_exact_solve(sweeps):
    """Global smoother = complete factorisation of D_B^{-1} A with exact triangular solves:
    the global step already returns A^{-1} v, the F-relaxation and the coarse correction
    then see a zero residual, so M^{-1} = A^{-1} and FGMRES takes one iteration."""
    rng = np.random.default_rng(30 + sweeps)
    D, labels = _two_label_system(rng, 20)
    n = D.shape[0]
    A = CSR.from_dense(D)
    lp = omgr.LevelPlan(f_labels=(1,), nmax=-1, frelax="jacobi", global_smoother="ilu",
                        global_sweeps=sweeps, ilu_level=n, ilu_sweeps=2 * n, ilu_tri_sweeps=-1)
    H = omgr.setup(A, labels, omgr.Plan(levels=[lp], coarse="dense"))
    v = rng.standard_normal(n)
    z = omgr.apply(H, v)
    assert np.linalg.norm(D @ z - v) <= 1e-10 * np.linalg.norm(v)
    r = okry.fgmres(A.matvec, lambda x: omgr.apply(H, x), v, restart=10, rtol=1e-10, maxit=10)
    assert r.converged and r.iters == 1


def test_mgr_ilu_smoother_factors_the_block_scaled_matrix():
    """The smoother's factors are those of D_B^{-1} A (D_B: same-cell diagonal blocks):
    compared with a dense restatement, and z = (LU)^{-1} D_B^{-1} v for the first step."""
    rng = np.random.default_rng(41)
    D, labels = _two_label_system(rng, 15)
    n = D.shape[0]
    A = CSR.from_dense(D)
    lp = omgr.LevelPlan(f_labels=(1,), nmax=-1, frelax="jacobi", global_smoother="ilu",
                        global_sweeps=1, ilu_level=0, ilu_sweeps=2 * n, ilu_tri_sweeps=-1)
    H = omgr.setup(A, labels, omgr.Plan(levels=[lp], coarse="dense"))
    L0 = H.levels[0]
    DB = np.zeros_like(D)
    for c in range(n // 2):
        DB[2 * c:2 * c + 2, 2 * c:2 * c + 2] = D[2 * c:2 * c + 2, 2 * c:2 * c + 2]
    Ds = np.linalg.solve(DB, D)
    S = pattern(L0.ilu.S)
    # pattern of D_B^{-1} A: the union of the rows of each cell
    cellrows = (D != 0).reshape(n // 2, 2, n).any(axis=1)
    assert np.array_equal(S, np.repeat(cellrows, 2, axis=0))
    W = textbook_ilu(Ds, S)
    L, U = factors_dense(L0.ilu)
    assert np.allclose(np.tril(L, -1) + U, W, rtol=1e-11, atol=1e-11 * np.abs(Ds).max())
    v = rng.standard_normal(n)
    zg = ilu.ilu_solve(L0.ilu, np.linalg.solve(DB, v), -1)
    assert np.allclose(zg, np.linalg.solve(U, np.linalg.solve(L, np.linalg.solve(DB, v))))


def test_synchronous_sweeps_hand_worked():
    """A = [[4,1,0],[2,5,1],[0,3,6]], ILU(0).  Start: l21 = 2/4, l32 = 3/5, U = upper(A).
    Every sweep takes all components from the previous iterate:
      sweep 1: l21 = 2/4, u22 = 5 - l21 u12 = 4.5, l32 = 3 / u22(old) = 3/5,
               u33 = 6 - l32(old) u23 = 6 - 0.6 = 5.4
      sweep 2: l32 = 3 / 4.5, u33 = 6 - 0.6 * 1 = 5.4
      sweep 3: u33 = 6 - (3 / 4.5) * 1  (the complete LU from here on)."""
    A = CSR.from_dense(np.array([[4.0, 1.0, 0.0], [2.0, 5.0, 1.0], [0.0, 3.0, 6.0]]))
    expect = {1: (0.5, 3.0 / 5.0, 4.5, 6.0 - 0.6),
              2: (0.5, 3.0 / 4.5, 4.5, 6.0 - 0.6),
              3: (0.5, 3.0 / 4.5, 4.5, 6.0 - (3.0 / 4.5) * 1.0)}
    for sw, (l21, l32, u22, u33) in expect.items():
        L, U = factors_dense(ilu.ilu_factor(A, 0, sw))
        assert (L[1, 0], L[2, 1], U[1, 1], U[2, 2]) == (l21, l32, u22, u33), sw
        assert (U[0, 0], U[0, 1], U[1, 2]) == (4.0, 1.0, 1.0)


def test_small_inverse_closed_form():
    """adj(B)/det(B) for 1x1, 2x2 and 3x3 blocks: B @ inv(B) = I to rounding, exact on a
    hand-worked 2x2 block, singular blocks rejected."""
    rng = np.random.default_rng(50)
    for nb in (1, 2, 3):
        D = rng.standard_normal((40, nb, nb)) + 3.0 * np.eye(nb)
        inv = omgr.small_inverse(D)
        assert np.allclose(np.einsum("eij,ejk->eik", D, inv), np.eye(nb)[None], atol=1e-13)
    # [[2, 1], [4, 3]]: det 2, inverse [[1.5, -0.5], [-2, 1]]
    inv = omgr.small_inverse(np.array([[[2.0, 1.0], [4.0, 3.0]]]))
    assert inv[0].tolist() == [[1.5, -0.5], [-2.0, 1.0]]
    # 3x3 with a known integer inverse: [[1,2,0],[0,1,0],[0,0,2]] -> [[1,-2,0],[0,1,0],[0,0,.5]]
    inv = omgr.small_inverse(np.array([[[1.0, 2.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 2.0]]]))
    assert inv[0].tolist() == [[1.0, -2.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 0.5]]
    with pytest.raises(omgr.ZeroPivot):
        omgr.small_inverse(np.array([[[1.0, 2.0], [2.0, 4.0]]]))
