"""Pins of the oracle's AMG and FGMRES against brute force, dense definitions and textbook
behaviour (published SplitMix64 outputs; MIS(2) equal to the greedy distance-2 independent
set in priority order; smoothed prolongator and Galerkin product against dense algebra;
V-cycle contraction on a 3D Poisson problem; GMRES finite termination and exact
preconditioning)."""
import json
import os
from collections import deque

import numpy as np
import pytest

from oracle import amg, krylov
from oracle.sparse import CSR, spgemm, transpose


def poisson3d(n):
    N = n ** 3
    idx = np.arange(N).reshape(n, n, n)
    rows, cols, vals = [], [], []
    for (dz, dy, dx) in [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]:
        z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        zz, yy, xx = z + dz, y + dy, x + dx
        ok = (zz >= 0) & (zz < n) & (yy >= 0) & (yy < n) & (xx >= 0) & (xx < n)
        rows.append(idx[ok])
        cols.append(idx[zz[ok], yy[ok], xx[ok]])
        vals.append(np.full(ok.sum(), 6.0 if dz == dy == dx == 0 else -1.0))
    return CSR.from_coo(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), (N, N))


def test_splitmix64_published_vectors(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "splitmix64.json")))
    with np.errstate(over="ignore"):
        for seed, outs in g["sequences"].items():
            for i, o in enumerate(outs):
                st = np.array([np.uint64(int(seed)) + np.uint64(i) * amg.GOLDEN], dtype=np.uint64)
                assert int(amg.splitmix64(st)[0]) == int(o, 0)


def test_priorities_are_a_bijection():
    p = amg.priorities(100000, 0)
    assert np.unique(p).shape[0] == 100000
    assert not np.array_equal(p, amg.priorities(100000, 1))


def _dist2_sets(gptr, gcol):
    n = gptr.shape[0] - 1
    nb = [set(gcol[gptr[i]:gptr[i + 1]].tolist()) for i in range(n)]
    d2 = []
    for i in range(n):
        s = set(nb[i])
        for j in nb[i]:
            s |= nb[j]
        s.discard(i)
        d2.append(s)
    return nb, d2


def _random_graph(rng, n, p):
    M = rng.random((n, n)) < p
    M = M | M.T
    np.fill_diagonal(M, False)
    r, c = np.nonzero(M)
    gptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=gptr[1:])
    return gptr, c.astype(np.int64)


@pytest.mark.parametrize("seed", range(6))
def test_mis2_equals_greedy_in_priority_order(seed):
    """Synchronous MIS(2) rounds with fixed priorities select the same set as the sequential
    greedy distance-2 independent set taken in decreasing priority (brute force)."""
    rng = np.random.default_rng(seed)
    n = 80
    gptr, gcol = _random_graph(rng, n, 0.03 + 0.01 * seed)
    prio = amg.priorities(n, seed)
    state = amg.mis2(gptr, gcol, prio)
    nb, d2 = _dist2_sets(gptr, gcol)
    chosen, blocked = set(), set()
    for i in sorted(range(n), key=lambda i: -int(prio[i])):
        if len(nb[i]) == 0 or i in blocked:
            continue
        chosen.add(i)
        blocked |= d2[i]
    assert set(np.flatnonzero(state == amg.SELECTED).tolist()) == chosen
    assert set(np.flatnonzero(state == amg.ISOLATED).tolist()) == {i for i in range(n) if not nb[i]}


def _bfs_dist(nb, src, limit):
    dist = {src: 0}
    q = deque([src])
    while q:
        u = q.popleft()
        if dist[u] == limit:
            continue
        for v in nb[u]:
            if v not in dist:
                dist[v] = dist[u] + 1
                q.append(v)
    return dist


@pytest.mark.parametrize("seed", range(4))
def test_aggregation_invariants(seed):
    rng = np.random.default_rng(100 + seed)
    n = 120
    gptr, gcol = _random_graph(rng, n, 0.04)
    prio = amg.priorities(n, 0)
    state = amg.mis2(gptr, gcol, prio)
    agg, nagg = amg.aggregate(gptr, gcol, state, prio)
    nb, _ = _dist2_sets(gptr, gcol)
    roots = np.flatnonzero(state == amg.SELECTED)
    for i in range(n):
        if not nb[i]:
            assert agg[i] == -1
        else:
            assert 0 <= agg[i] < nagg
    for a, r in enumerate(roots):       # one root per aggregate, members within 2 hops
        members = np.flatnonzero(agg == a)
        assert r in members
        d = _bfs_dist(nb, int(r), 2)
        assert all(int(m) in d for m in members)
    # every aggregate id is used
    assert set(agg[agg >= 0].tolist()) == set(range(nagg))


def test_tentative_and_smoothed_prolongator_dense():
    """T has one unit entry per aggregated unknown, components never mixed; P equals
    (I - omega D^{-1} A) T with the dense definition; R = P^T; A_c = P^T A P."""
    A = poisson3d(6)
    gptr, gcol = amg.strength_graph(A, 0.08, 1)
    prio = amg.priorities(A.shape[0], 0)
    agg, nagg = amg.aggregate(gptr, gcol, amg.mis2(gptr, gcol, prio), prio)
    T = amg.tentative(agg, nagg, 1)
    Td = T.to_dense()
    assert np.all(Td.sum(axis=1) == (agg >= 0))
    P, omega = amg.smoothed_prolongator(A, T)
    Ad = A.to_dense()
    rho = np.max(np.abs(Ad).sum(axis=1) / np.abs(np.diag(Ad)))
    assert omega == pytest.approx((4.0 / 3.0) / rho, rel=1e-15)
    Pd = (np.eye(A.shape[0]) - omega * np.diag(1.0 / np.diag(Ad)) @ Ad) @ Td
    assert np.allclose(P.to_dense(), Pd, rtol=1e-14, atol=1e-15)
    Ac = spgemm(transpose(P), spgemm(A, P))
    assert np.allclose(Ac.to_dense(), Pd.T @ Ad @ Pd, rtol=1e-13, atol=1e-13)


def test_nodal_tentative_unknown_approach():
    """Nodal (3 unknowns per node) aggregation: T = T_node (x) I_3 in node-major order."""
    agg = np.array([0, 1, -1, 0])
    T = amg.tentative(agg, 2, 3).to_dense()
    exp = np.zeros((12, 6))
    for node, a in enumerate(agg):
        if a >= 0:
            for c in range(3):
                exp[3 * node + c, 3 * a + c] = 1.0
    assert np.array_equal(T, exp)


def test_vcycle_contracts_on_poisson():
    """Textbook behaviour: the SA-AMG V-cycle with l1-Jacobi is a convergent iteration on the
    3D Poisson problem."""
    A = poisson3d(14)
    H = amg.setup(A, amg.AMGOptions(coarse_size=50))
    assert len(H.levels) >= 2
    rng = np.random.default_rng(0)
    b = rng.standard_normal(A.shape[0])
    x = np.zeros_like(b)
    norms = []
    for _ in range(12):
        x = x + amg.vcycle(H, b - A.matvec(x))
        norms.append(np.linalg.norm(b - A.matvec(x)))
    rate = (norms[-1] / norms[2]) ** (1.0 / 9)
    assert rate < 0.7


def test_fgmres_identity_preconditioner_finite_termination():
    rng = np.random.default_rng(1)
    n = 25
    D = rng.standard_normal((n, n)) + 4 * np.eye(n)
    b = rng.standard_normal(n)
    res = krylov.fgmres(lambda x: D @ x, lambda v: v, b, restart=n, rtol=1e-12, maxit=200)
    assert res.converged and res.iters <= n
    assert np.allclose(res.x, np.linalg.solve(D, b), rtol=1e-9, atol=1e-10)
    est = res.history[1:]
    assert all(est[i + 1] <= est[i] * (1 + 1e-12) for i in range(len(est) - 2))


def test_fgmres_exact_preconditioner_one_iteration():
    rng = np.random.default_rng(2)
    n = 30
    D = rng.standard_normal((n, n)) + 5 * np.eye(n)
    Dinv = np.linalg.inv(D)
    res = krylov.fgmres(lambda x: D @ x, lambda v: Dinv @ v, rng.standard_normal(n), rtol=1e-10)
    assert res.converged and res.iters == 1


def test_fgmres_restarts_and_true_residual():
    rng = np.random.default_rng(3)
    n = 60
    D = rng.standard_normal((n, n)) * 0.3 + np.diag(np.linspace(1, 10, n))
    b = rng.standard_normal(n)
    res = krylov.fgmres(lambda x: D @ x, lambda v: v, b, restart=5, rtol=1e-9, maxit=2000)
    assert res.converged
    assert np.linalg.norm(b - D @ res.x) / np.linalg.norm(b) <= 1e-9
