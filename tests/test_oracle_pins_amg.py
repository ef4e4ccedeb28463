"""Hand-worked pins of the oracle's AMG strength rule, aggregation choice rule and the
global block-Jacobi smoother (test infrastructure; CPU only).

Every expected value below was worked out by hand from the definitions the oracle states
(strength: a_ij != 0 and a_ij^2 >= theta^2 |a_ii a_jj|, nodal: f_IJ^2 >= theta^4 f_II f_JJ on
squared Frobenius norms f, symmetrised by union; aggregation pass 1 joins the neighbouring
root of largest priority, pass 2 the aggregate of the aggregated neighbour of largest
priority; block Jacobi over same-cell blocks with the first sweep z = D_B^{-1} v and later
sweeps z += omega D_B^{-1} (v - A z)).  The values are dyadic, so the threshold
comparisons are exact and equality cases sit exactly on the threshold: a strict `>` in
place of `>=`, theta^2 in place of theta^4, a dropped a_jj (or f_JJ), a missing
symmetrisation, the lowest instead of the highest priority, or the root's priority in
place of the neighbour's each change one of the expected results.
"""
import numpy as np
import pytest

from oracle import amg, mgr
from oracle.sparse import CSR


def _csr(entries, n):
    r = np.array([e[0] for e in entries], dtype=np.int64)
    c = np.array([e[1] for e in entries], dtype=np.int64)
    v = np.array([e[2] for e in entries], dtype=np.float64)
    return CSR.from_coo(r, c, v, (n, n))


def _edges(gptr, gcol):
    n = gptr.shape[0] - 1
    return {i: gcol[gptr[i]:gptr[i + 1]].tolist() for i in range(n)}


# ---------------------------------------------------------------------------------------
# scalar strength, theta = 1/2 (theta^2 = 1/4)
#   (0,1): a^2 = 1     vs 1/4*4*1   = 1    equal -> strong
#   (0,2): 1/4         vs 1/4*4*16  = 16   weak
#   (0,4): explicit 0                      weak
#   (0,5): 1           vs 1/4*4*100 = 100  weak
#   (1,2): 1/16        vs 1/4*1*16  = 4    weak
#   (2,1): 4           vs 4                equal -> strong   (only this direction)
#   (2,3): 9           vs 1/4*16*1  = 4    strong
#   (3,2): 1/4         vs 4                weak
#   (4,3): 9/16        vs 1/4*2*1   = 1/2  strong            (row 3 has no (3,4) entry)
#   (5,0): 1           vs 100              weak -> node 5 has no strong neighbour
SCALAR = [
    (0, 0, 4.0), (0, 1, -1.0), (0, 2, -0.5), (0, 4, 0.0), (0, 5, -1.0),
    (1, 0, -1.0), (1, 1, 1.0), (1, 2, -0.25),
    (2, 0, -0.5), (2, 1, -2.0), (2, 2, 16.0), (2, 3, -3.0),
    (3, 2, -0.5), (3, 3, 1.0),
    (4, 0, 0.0), (4, 3, -0.75), (4, 4, 2.0),
    (5, 0, -1.0), (5, 5, 100.0),
]
SCALAR_GRAPH = {0: [1], 1: [0, 2], 2: [1, 3], 3: [2, 4], 4: [3], 5: []}


def test_scalar_strength_hand_worked():
    A = _csr(SCALAR, 6)
    gptr, gcol = amg.strength_graph(A, 0.5, 1)
    assert _edges(gptr, gcol) == SCALAR_GRAPH


def test_scalar_strength_threshold_is_inclusive_and_uses_both_diagonals():
    """Raising theta by one ulp-sized step removes exactly the two equality edges (0,1) and
    (2,1); halving a_22 (which enters (2,1) only through a_ii) keeps the graph's shape."""
    A = _csr(SCALAR, 6)
    gptr, gcol = amg.strength_graph(A, np.nextafter(0.5, 1.0), 1)
    assert _edges(gptr, gcol) == {0: [], 1: [], 2: [3], 3: [2, 4], 4: [3], 5: []}
    # a_22 = 4: (2,1) 4 >= 1/4*4*1 strong, (1,2) 1/16 >= 1 weak, (2,3) 9 >= 1 strong,
    # (3,2) 1/4 >= 1 weak, (0,2) 1/4 >= 1/4*4*4 = 4 weak, (2,0) likewise
    B = _csr([(i, j, (4.0 if (i, j) == (2, 2) else v)) for i, j, v in SCALAR], 6)
    gptr, gcol = amg.strength_graph(B, 0.5, 1)
    assert _edges(gptr, gcol) == SCALAR_GRAPH


# ---------------------------------------------------------------------------------------
# nodal strength (3x3 blocks), theta = 1/2 (theta^4 = 1/16); f = squared Frobenius norm
#   f_00 = 12 (2 I), f_11 = 3 (I), f_22 = 48 (4 I)
#   (0,1): f = 1 + 1/4 + 1/4 = 3/2, f^2 = 9/4 vs 1/16*12*3 = 9/4  equal -> strong
#   (1,0): f = 1/4,               f^2 = 1/16 vs 9/4               weak
#   (1,2): f = 2,                 f^2 = 4    vs 1/16*3*48 = 9     weak
#   (2,1): f = 4 (one entry 2),   f^2 = 16   vs 9                 strong
def _nodal_matrix():
    D = np.zeros((9, 9))
    mask = np.zeros((9, 9), dtype=bool)

    def blk(I, J, B):
        D[3 * I:3 * I + 3, 3 * J:3 * J + 3] = B
        mask[3 * I:3 * I + 3, 3 * J:3 * J + 3] = True

    blk(0, 0, 2.0 * np.eye(3))
    blk(1, 1, np.eye(3))
    blk(2, 2, 4.0 * np.eye(3))
    b01 = np.zeros((3, 3)); b01[0, 0] = 1.0; b01[1, 2] = -0.5; b01[2, 1] = 0.5
    blk(0, 1, b01)
    b10 = np.zeros((3, 3)); b10[2, 0] = -0.5
    blk(1, 0, b10)
    b12 = np.zeros((3, 3)); b12[0, 1] = 1.0; b12[2, 2] = -1.0
    blk(1, 2, b12)
    b21 = np.zeros((3, 3)); b21[1, 1] = -2.0
    blk(2, 1, b21)
    return CSR.from_dense(D, mask)


def test_nodal_strength_hand_worked():
    A = _nodal_matrix()
    gptr, gcol = amg.strength_graph(A, 0.5, 3)
    assert _edges(gptr, gcol) == {0: [1], 1: [0, 2], 2: [1]}
    # just above the threshold the equality edge (0,1) goes, (2,1) stays
    gptr, gcol = amg.strength_graph(A, np.nextafter(0.5, 1.0), 3)
    assert _edges(gptr, gcol) == {0: [], 1: [2], 2: [1]}


def test_nodal_strength_matches_scalar_on_kron_variable_coefficients():
    """For A = A_s (x) I_3 every block is a_IJ I_3 with f = 3 a_IJ^2, so the nodal test
    reduces to the scalar one.  A_s has variable coefficients and theta splits its entries
    into strong and weak ones, so the compared graphs are neither empty nor complete."""
    rng = np.random.default_rng(11)
    n = 40
    M = (rng.random((n, n)) < 0.15) * np.exp2(rng.integers(-4, 3, size=(n, n)))
    np.fill_diagonal(M, 0.0)
    Ds = -M
    Ds[np.arange(n), np.arange(n)] = np.exp2(rng.integers(0, 5, size=n))
    As = CSR.from_dense(Ds)
    A3 = CSR.from_dense(np.kron(Ds, np.eye(3)), np.kron(Ds != 0, np.ones((3, 3), dtype=bool)))
    g1 = amg.strength_graph(As, 0.3, 1)
    g3 = amg.strength_graph(A3, 0.3, 3)
    assert np.array_equal(g1[0], g3[0]) and np.array_equal(g1[1], g3[1])
    n_off = int(((Ds != 0) | (Ds.T != 0)).sum() - n)
    assert 0 < g1[1].shape[0] < n_off


# ---------------------------------------------------------------------------------------
def _graph(n, edges):
    M = np.zeros((n, n), dtype=bool)
    for i, j in edges:
        M[i, j] = M[j, i] = True
    r, c = np.nonzero(M)
    gptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=gptr[1:])
    return gptr, c.astype(np.int64)


def test_aggregation_pass2_takes_highest_priority_neighbour():
    """Path 0-1-2-3-4 with priorities (50, 10, 20, 30, 40).  MIS(2): 0 and 4 are the
    largest within distance 2 and are selected in the first round; 1, 2, 3 are removed.
    Pass 1: 1 joins root 0 (aggregate 0), 3 joins root 4 (aggregate 1).  Pass 2: node 2 has
    the aggregated neighbours 1 (priority 10, aggregate 0) and 3 (priority 30, aggregate 1)
    and joins aggregate 1.  (The lowest-priority rule would give 0; so would the rule of the
    larger root priority, 50 > 40.)"""
    gptr, gcol = _graph(5, [(0, 1), (1, 2), (2, 3), (3, 4)])
    prio = np.array([50, 10, 20, 30, 40], dtype=np.uint64)
    state = amg.mis2(gptr, gcol, prio)
    assert state.tolist() == [amg.SELECTED, amg.REMOVED, amg.REMOVED, amg.REMOVED, amg.SELECTED]
    agg, nagg = amg.aggregate(gptr, gcol, state, prio)
    assert nagg == 2
    assert agg.tolist() == [0, 0, 1, 1, 1]


def test_aggregation_pass1_takes_highest_priority_root_and_numbers_singletons():
    """A state with two roots next to one node (the aggregation rule is defined for any
    root set): star 0-{1, 2} plus the edge 3-4 and the isolated node 5.  Roots 1 (priority
    5) and 2 (priority 9) are aggregates 0 and 1 (ascending node order); node 0 joins the
    root of larger priority, aggregate 1.  Nodes 3 and 4 (removed, no aggregated neighbour)
    become singleton aggregates 2 and 3 in node order; node 5 gets none."""
    gptr, gcol = _graph(6, [(0, 1), (0, 2), (3, 4)])
    prio = np.array([1, 5, 9, 7, 3, 2], dtype=np.uint64)
    state = np.array([amg.REMOVED, amg.SELECTED, amg.SELECTED, amg.REMOVED, amg.REMOVED,
                      amg.ISOLATED], dtype=np.int8)
    agg, nagg = amg.aggregate(gptr, gcol, state, prio)
    assert agg.tolist() == [1, 0, 1, 2, 3, -1]
    assert nagg == 4


def test_aggregation_pass2_uses_pass1_aggregates_only():
    """Path 0-1-2-3 with priorities (90, 10, 30, 20): 0 selected, 1 and 2 removed in the
    first round; 3 (undecided, priority 20, only 2 within distance 2 is removed) is selected
    in the second round.  Pass 1: 1 joins 0, 2 joins root 3 (its only root neighbour).
    Nothing is left for pass 2."""
    gptr, gcol = _graph(4, [(0, 1), (1, 2), (2, 3)])
    prio = np.array([90, 10, 30, 20], dtype=np.uint64)
    state = amg.mis2(gptr, gcol, prio)
    assert state.tolist() == [amg.SELECTED, amg.REMOVED, amg.REMOVED, amg.SELECTED]
    agg, nagg = amg.aggregate(gptr, gcol, state, prio)
    assert agg.tolist() == [0, 0, 1, 1] and nagg == 2


# ---------------------------------------------------------------------------------------
# global block-Jacobi smoother: dense restatement on an interleaved (s, p) system
def _interleaved_system(rng, ncell):
    n = 2 * ncell
    D = rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.35)
    D[np.arange(n), np.arange(n)] = 2.0 * (np.abs(D).sum(axis=1) + 1.0)
    labels = np.tile(np.array([1, 2], dtype=np.int8), ncell)
    return D, labels


def _dense_block_jacobi(D, v, sweeps, omega):
    n = D.shape[0]
    cell = np.arange(n) // 2
    DB = D * (cell[:, None] == cell[None, :])
    z = np.linalg.solve(DB, v)
    for _ in range(sweeps - 1):
        z = z + omega * np.linalg.solve(DB, v - D @ z)
    return z


def test_block_jacobi_single_sweep_dense():
    rng = np.random.default_rng(21)
    D, labels = _interleaved_system(rng, 9)
    A = CSR.from_dense(D)
    plan = mgr.Plan(levels=[mgr.LevelPlan(f_labels=(1,), global_smoother="block_jacobi")])
    L = mgr.setup(A, labels, plan).levels[0]
    v = rng.standard_normal(D.shape[0])
    z = mgr._block_jacobi(L, v)
    want = _dense_block_jacobi(D, v, 1, 1.0)
    assert np.linalg.norm(z - want) <= 1e-13 * np.linalg.norm(want)


@pytest.mark.parametrize("sweeps", [1, 2, 3])
def test_apply_with_block_jacobi_sweeps_dense(sweeps):
    """The whole two-grid apply with k global sweeps (omega = 0.7), one Jacobi F-sweep on
    the s rows, Galerkin coarse grid on p solved exactly, restated with dense algebra:
      z = BJ_k(v); z_F += D_FF^{-1}(v - A z)_F; r = v - A z;
      e = S^{-1} r_C with S = A_CC - A_CF D_FF^{-1} A_FC; z_F -= D_FF^{-1} A_FC e; z_C += e."""
    rng = np.random.default_rng(30 + sweeps)
    D, labels = _interleaved_system(rng, 11)
    A = CSR.from_dense(D)
    plan = mgr.Plan(levels=[mgr.LevelPlan(f_labels=(1,), global_smoother="block_jacobi",
                                          global_sweeps=sweeps, global_omega=0.7)],
                    coarse="dense")
    H = mgr.setup(A, labels, plan)
    F = np.flatnonzero(labels == 1)
    C = np.flatnonzero(labels == 2)
    dF = np.diag(D)[F]
    AFC, ACF, ACC = D[np.ix_(F, C)], D[np.ix_(C, F)], D[np.ix_(C, C)]
    S = ACC - ACF @ (AFC / dF[:, None])
    for t in range(3):
        v = rng.standard_normal(D.shape[0])
        z = _dense_block_jacobi(D, v, sweeps, 0.7)
        z[F] = z[F] + (v - D @ z)[F] / dF
        r = v - D @ z
        e = np.linalg.solve(S, r[C])
        z[F] = z[F] - (AFC @ e) / dF
        z[C] = z[C] + e
        got = mgr.apply(H, v)
        assert np.linalg.norm(got - z) <= 1e-12 * np.linalg.norm(z), (sweeps, t)
    # the weight matters from the second sweep on
    if sweeps > 1:
        v = rng.standard_normal(D.shape[0])
        assert not np.allclose(_dense_block_jacobi(D, v, sweeps, 0.7),
                               _dense_block_jacobi(D, v, sweeps, 1.0), rtol=1e-6, atol=0)
