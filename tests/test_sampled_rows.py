"""The sampled-row evaluation used by the full-size GPU tests reproduces the oracle's whole-
matrix setup: on small problems every row of every level's W_p and A_{l+1}, computed from
row-restricted matrices, equals the row of the oracle's full setup bit for bit."""
import numpy as np
import pytest

from oracle import amg as oamg
from oracle import mgr as omgr
from oracle.sparse import CSR
from tests.sampled import level_chain, restrict_rows, sample_rows, stack_rows
from workloads import poromech as pm


def _plan(levels):
    return omgr.Plan(levels=levels, coarse="dense",
                     amg_frelax=oamg.AMGOptions(0.08, 10, 48, 3),
                     amg_coarse=oamg.AMGOptions(0.08, 10, 48, 1))


PLANS = {
    "two_paper": (lambda: pm.two_phase(7, 6, 5, 1), _plan([
        omgr.LevelPlan((0,), nmax=4), omgr.LevelPlan((1,), nmax=-1)])),
    "two_satfirst": (lambda: pm.two_phase(7, 6, 5, 1), _plan([
        omgr.LevelPlan((1,), nmax=-1), omgr.LevelPlan((0,), nmax=4)])),
    "three_paper": (lambda: pm.three_phase(5, 4, 4, 3), _plan([
        omgr.LevelPlan((0,), nmax=4), omgr.LevelPlan((3,), nmax=-1),
        omgr.LevelPlan((1,), nmax=-1)])),
    "two_quasi_impes": (lambda: pm.two_phase(7, 6, 5, 1), _plan([
        omgr.LevelPlan((0,), nmax=4), omgr.LevelPlan((1,), nmax=-1, coupling="quasi_impes")])),
    "two_drop_tol": (lambda: pm.two_phase(7, 6, 5, 1), _plan([
        omgr.LevelPlan((0,), drop_tol=0.05), omgr.LevelPlan((1,), nmax=-1)])),
    "three_drop2": (lambda: pm.three_phase(5, 4, 4, 3), _plan([
        omgr.LevelPlan((0,), nmax=2), omgr.LevelPlan((3,), nmax=1),
        omgr.LevelPlan((1,), nmax=0)])),
}


def _same(X: CSR, Y: CSR):
    assert X.shape == Y.shape
    assert np.array_equal(X.indptr, Y.indptr)
    assert np.array_equal(X.indices, Y.indices)
    assert np.array_equal(X.data.view(np.uint64), Y.data.view(np.uint64))


@pytest.mark.parametrize("name", sorted(PLANS))
def test_every_row_matches_full_setup(name):
    make, plan = PLANS[name]
    w = make()
    A = CSR(w.indptr, w.indices, w.data, (w.n, w.n))
    H = omgr.setup(A, w.labels, plan)
    chain = level_chain(A, w.labels, plan)
    for lvl, (L, R) in enumerate(zip(H.levels, chain)):
        nC = L.C.shape[0]
        S_rows, Wp_rows, ks = R.coarse_rows(np.arange(nC))
        nxt = H.levels[lvl + 1].A if lvl + 1 < len(H.levels) else H.coarse_A
        _same(S_rows, nxt)
        _same(Wp_rows, restrict_rows(L.Wp, ks))


@pytest.mark.parametrize("name", ["two_paper", "three_paper"])
def test_sampled_rows_match_full_setup(name):
    make, plan = PLANS[name]
    w = make()
    A = CSR(w.indptr, w.indices, w.data, (w.n, w.n))
    H = omgr.setup(A, w.labels, plan)
    chain = level_chain(A, w.labels, plan)
    for lvl, (L, R) in enumerate(zip(H.levels, chain)):
        rows = sample_rows(L.C.shape[0], 9, seed=lvl)
        S_rows, _, _ = R.coarse_rows(rows)
        nxt = H.levels[lvl + 1].A if lvl + 1 < len(H.levels) else H.coarse_A
        _same(S_rows, restrict_rows(nxt, rows))
        assert np.all(np.diff(S_rows.indptr)[np.setdiff1d(np.arange(nxt.shape[0]), rows)] == 0)


def test_stack_rows_rejects_overlap_and_keeps_order():
    D = np.arange(1.0, 17.0).reshape(4, 4)
    A = CSR.from_dense(D)
    X, Y = restrict_rows(A, [0, 2]), restrict_rows(A, [1, 3])
    _same(stack_rows(X, Y), A)
    with pytest.raises(AssertionError):
        stack_rows(X, restrict_rows(A, [2]))
