"""Pins of the oracle's operator variants of Sec. 5.1-5.3: the Jacobi restriction
W_r = -A_CF D_FF^{-1} and the block diagonal D_FF, each against the dense operators of
eq. RPoperator1 written out with NumPy, and the exactness special case."""
import numpy as np
import pytest

from oracle import krylov as okry
from oracle import mgr as omgr
from oracle.sparse import CSR


def system(rng, n, nF, density=0.15, diag_ff=False, blocks=1):
    """Random diagonally dominant system; labels 0 for the first nF rows (F), 1 for the rest,
    interleaved so that F and C are not contiguous."""
    D = rng.standard_normal((n, n)) * (rng.random((n, n)) < density)
    labels = np.ones(n, dtype=np.int8)
    Fidx = np.sort(rng.choice(n // blocks, size=nF // blocks, replace=False))
    Fidx = (Fidx[:, None] * blocks + np.arange(blocks)[None, :]).ravel()
    labels[Fidx] = 0
    if diag_ff:
        D[np.ix_(Fidx, Fidx)] = 0.0
    if blocks > 1:   # full diagonal blocks within each F group
        for g in Fidx.reshape(-1, blocks):
            D[np.ix_(g, g)] = rng.standard_normal((blocks, blocks))
    D[np.arange(n), np.arange(n)] = 3.0 * (np.abs(D).sum(axis=1) + 1.0)
    return D, labels


def dense_ops(D, labels, nb=1, restrict="injection"):
    F = np.flatnonzero(labels == 0)
    C = np.flatnonzero(labels != 0)
    Aff, Afc = D[np.ix_(F, F)], D[np.ix_(F, C)]
    Acf, Acc = D[np.ix_(C, F)], D[np.ix_(C, C)]
    if nb == 1:
        Dff = np.diag(np.diag(Aff))
    else:
        Dff = np.zeros_like(Aff)
        for k in range(0, len(F), nb):
            Dff[k:k + nb, k:k + nb] = Aff[k:k + nb, k:k + nb]
    Di = np.linalg.inv(Dff)
    Wp = -Di @ Afc
    Wr = -Acf @ Di if restrict == "jacobi" else np.zeros((len(C), len(F)))
    P = np.vstack([Wp, np.eye(len(C))])
    R = np.hstack([Wr, np.eye(len(C))])
    Ap = D[np.ix_(np.r_[F, C], np.r_[F, C])]
    return F, C, Dff, Wp, Wr, R @ Ap @ P


@pytest.mark.parametrize("seed", [0, 1])
def test_jacobi_restriction_coarse_grid_is_rap(seed):
    """Galerkin coarse grid with R~ = [W_r I]: R~ A P~ = A_CC + W_r A_FC + A_CF W_p +
    W_r A_FF W_p, from the dense operators."""
    rng = np.random.default_rng(seed)
    D, labels = system(rng, 60, 25)
    lp = omgr.LevelPlan(f_labels=(0,), nmax=-1, restrict="jacobi")
    H = omgr.setup(CSR.from_dense(D), labels, omgr.Plan(levels=[lp], coarse="dense"))
    F, C, Dff, Wp, Wr, S = dense_ops(D, labels, restrict="jacobi")
    L = H.levels[0]
    assert np.allclose(L.Wr.to_dense(), Wr, rtol=0, atol=1e-15 * np.abs(Wr).max())
    assert np.allclose(H.coarse_A.to_dense(), S, rtol=1e-13, atol=1e-13 * np.abs(S).max())
    # injection differs from it (W_r = 0)
    H0 = omgr.setup(CSR.from_dense(D), labels,
                    omgr.Plan(levels=[omgr.LevelPlan(f_labels=(0,), nmax=-1)], coarse="dense"))
    assert not np.allclose(H0.coarse_A.to_dense(), S, rtol=1e-8)


def test_jacobi_restriction_apply_is_the_two_grid_operator():
    """One Jacobi F-sweep from zero, restriction R~ (v - A z), exact coarse solve,
    interpolation: z = z0 + P~ S^{-1} R~ (v - A z0), z0 = Q D_FF^{-1} Q^T v."""
    rng = np.random.default_rng(3)
    D, labels = system(rng, 50, 20)
    lp = omgr.LevelPlan(f_labels=(0,), nmax=-1, restrict="jacobi")
    H = omgr.setup(CSR.from_dense(D), labels, omgr.Plan(levels=[lp], coarse="dense"))
    F, C, Dff, Wp, Wr, S = dense_ops(D, labels, restrict="jacobi")
    v = rng.standard_normal(50)
    z0 = np.zeros(50)
    z0[F] = np.linalg.solve(Dff, v[F])
    r = v - D @ z0
    eC = np.linalg.solve(S, r[C] + Wr @ r[F])
    z = z0.copy()
    z[F] += Wp @ eC
    z[C] += eC
    assert np.allclose(omgr.apply(H, v), z, rtol=1e-12, atol=1e-12 * np.abs(z).max())


def test_jacobi_restriction_exact_when_aff_is_diagonal():
    """A_FF diagonal: W_p and W_r are the ideal operators, so with one exact Jacobi sweep
    and an exact coarse solve M^{-1} = A^{-1}: FGMRES takes one iteration."""
    rng = np.random.default_rng(4)
    D, labels = system(rng, 60, 30, diag_ff=True)
    A = CSR.from_dense(D)
    lp = omgr.LevelPlan(f_labels=(0,), nmax=-1, restrict="jacobi")
    H = omgr.setup(A, labels, omgr.Plan(levels=[lp], coarse="dense"))
    v = rng.standard_normal(60)
    assert np.linalg.norm(D @ omgr.apply(H, v) - v) <= 1e-11 * np.linalg.norm(v)
    r = okry.fgmres(A.matvec, lambda x: omgr.apply(H, x), v, restart=10, rtol=1e-10, maxit=5)
    assert r.converged and r.iters == 1


@pytest.mark.parametrize("nb", [2, 3])
def test_block_dff_interpolation_and_coarse_grid(nb):
    """Block D_FF of nb consecutive F rows: W_p = -D_FF^{-1} A_FC and the coarse grid
    A_CC - A_CF D_FF^{-1} A_FC from the dense blocks; the Jacobi F-relaxation uses the
    blocks too."""
    rng = np.random.default_rng(10 + nb)
    D, labels = system(rng, 66, 24, blocks=nb)
    lp = omgr.LevelPlan(f_labels=(0,), nmax=-1, dff_block=nb)
    H = omgr.setup(CSR.from_dense(D), labels, omgr.Plan(levels=[lp], coarse="dense"))
    F, C, Dff, Wp, Wr, S = dense_ops(D, labels, nb=nb)
    L = H.levels[0]
    assert np.allclose(L.Wp.to_dense(), Wp, rtol=1e-13, atol=1e-14 * np.abs(Wp).max())
    assert np.allclose(H.coarse_A.to_dense(), S, rtol=1e-13, atol=1e-13 * np.abs(S).max())
    v = rng.standard_normal(66)
    z0 = np.zeros(66)
    z0[F] = np.linalg.solve(Dff, v[F])
    r = v - D @ z0
    eC = np.linalg.solve(S, r[C])
    z = z0.copy()
    z[F] += Wp @ eC
    z[C] += eC
    assert np.allclose(omgr.apply(H, v), z, rtol=1e-12, atol=1e-12 * np.abs(z).max())
    # with pointwise D_FF the result differs
    H1 = omgr.setup(CSR.from_dense(D), labels,
                    omgr.Plan(levels=[omgr.LevelPlan(f_labels=(0,), nmax=-1)], coarse="dense"))
    assert not np.allclose(H1.levels[0].Wp.to_dense(), Wp, rtol=1e-6)


def test_block_dff_with_jacobi_restriction():
    rng = np.random.default_rng(20)
    D, labels = system(rng, 60, 24, blocks=3)
    lp = omgr.LevelPlan(f_labels=(0,), nmax=-1, dff_block=3, restrict="jacobi")
    H = omgr.setup(CSR.from_dense(D), labels, omgr.Plan(levels=[lp], coarse="dense"))
    F, C, Dff, Wp, Wr, S = dense_ops(D, labels, nb=3, restrict="jacobi")
    assert np.allclose(H.coarse_A.to_dense(), S, rtol=1e-13, atol=1e-13 * np.abs(S).max())


def test_block_dff_singular_block_is_a_zero_pivot():
    rng = np.random.default_rng(21)
    D, labels = system(rng, 30, 12, blocks=3)
    F = np.flatnonzero(labels == 0)
    D[np.ix_(F[:3], F[:3])] = 1.0            # a rank-one 3x3 block
    with pytest.raises(omgr.ZeroPivot):
        omgr.setup(CSR.from_dense(D), labels,
                   omgr.Plan(levels=[omgr.LevelPlan(f_labels=(0,), dff_block=3)], coarse="dense"))
