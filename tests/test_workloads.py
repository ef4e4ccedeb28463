"""The synthetic Jacobians have the structure the method assumes: the 3x3 block layout of
eq. block_linear_system, interleaved cell unknowns, sorted unique columns, a symmetric
elasticity block, the closed-form pattern size, and b = A x_true."""
import numpy as np
import pytest

from workloads import poromech as pm


@pytest.mark.parametrize("make,args", [(pm.biot_single_phase, (8, 8, 8, 0)),
                                       (pm.two_phase, (6, 5, 4, 1)),
                                       (pm.three_phase, (4, 5, 3, 3)),
                                       (pm.two_phase_channels, (8, 8, 4, 2))])
def test_structure(make, args):
    w = make(*args)
    A = w.scipy()
    assert w.nnz == pm.closed_form_nnz(w.nx, w.ny, w.nz, w.model)
    for i in range(w.n):
        c = w.indices[w.indptr[i]:w.indptr[i + 1]]
        assert np.all(np.diff(c) > 0)
    Nu = w.meta["Nu"]
    assert np.all(w.labels[:Nu] == pm.LABEL_U)
    slots = np.array(w.meta["slots"], dtype=np.int8)
    assert np.array_equal(w.labels[Nu:], np.tile(slots, w.meta["ncell"]))
    Auu = A[:Nu, :Nu]
    assert abs(Auu - Auu.T).max() <= 1e-12 * abs(Auu).max()
    assert np.allclose(A @ w.x_true, w.b, rtol=0, atol=0)
    d = A.diagonal()
    assert np.all(d != 0)
    # Dirichlet rows keep only their diagonal value
    fixed = np.flatnonzero(w.fixed)
    for r in fixed[:50]:
        s, e = w.indptr[r], w.indptr[r + 1]
        nz = w.indices[s:e][w.data[s:e] != 0]
        assert nz.tolist() == [r]


def test_stiffness_rigid_modes():
    """The unit-cube Q1 stiffness annihilates the six rigid-body modes."""
    K = pm.q1_unit_stiffness(0.25)
    X = np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], dtype=float)
    modes = []
    for i in range(3):
        m = np.zeros((8, 3)); m[:, i] = 1; modes.append(m.ravel())
    for (i, j) in [(0, 1), (1, 2), (0, 2)]:
        m = np.zeros((8, 3)); m[:, i] = -X[:, j]; m[:, j] = X[:, i]; modes.append(m.ravel())
    for m in modes:
        assert np.abs(K @ m).max() < 1e-12
    assert np.all(np.linalg.eigvalsh(K)[6:] > 1e-3)


def test_seeded_and_reproducible():
    a = pm.two_phase(5, 5, 5, 7)
    b = pm.two_phase(5, 5, 5, 7)
    assert np.array_equal(a.data, b.data) and np.array_equal(a.b, b.b)
