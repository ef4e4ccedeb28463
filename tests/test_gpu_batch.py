"""Batched solve of small systems (mgr_batch_solve): one setup and one FGMRES over the
block-diagonal union of the systems, with one Arnoldi process per system.

  * the premise, bit for bit: the MGR levels of the union (W_p, A_cor, G, coarse operators)
    are the block diagonals of the levels of the separate setups, since every step of the
    reduction is row-local;
  * every system meets its own relative tolerance, including one whose right-hand side is
    scaled by 1e8 and one whose right-hand side is zero (its solution is exactly zero);
  * the solutions agree with separate solves to the accuracy both tolerances allow, and
    each system takes about the iterations of its separate solve;
  * argument errors leave the library usable.
"""
import ctypes as C

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.sparse import CSR
from tests.helpers import assert_csr_equal, device_workload
from workloads import poromech as pm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
m = pytest.importorskip("paper_1904_05960_amd.mgr355")


def plan():
    opts = m.paper_plan("two")
    opts.amg_frelax = m.AMG(coarse_size=48)
    opts.amg_coarse = m.AMG(coarse_size=48)
    return opts


SYSTEMS = [(6, 5, 4, 1), (9, 7, 6, 2), (5, 5, 5, 3), (8, 4, 6, 4)]


def workloads():
    return [pm.two_phase(*s) for s in SYSTEMS]


def scipy_of(w):
    return sp.csr_matrix((w.data, w.indices, w.indptr), shape=(w.n, w.n))


def test_union_levels_are_block_diagonals_of_separate_levels():
    ws = workloads()
    U = sp.block_diag([scipy_of(w) for w in ws], format="csr")
    U.sort_indices()
    lab = np.concatenate([w.labels for w in ws])
    opts = plan()
    opts.keep_setup = True
    PU = m.Preconditioner(m.Matrix.from_host(U.indptr, U.indices, U.data),
                          torch.as_tensor(lab).cuda(), opts)
    singles = []
    for w in ws:
        A, labels, _ = device_workload(w)
        singles.append(m.Preconditioner(A, labels, opts))
    for level in range(len(opts.levels)):
        for what in (m.X_WP, m.X_ACOR, m.X_G, m.X_COARSE):
            parts = []
            for P in singles:
                rp, ci, v, shape = P.export(what, level)
                parts.append(sp.csr_matrix((v, ci, rp), shape=shape))
            exp = sp.block_diag(parts, format="csr")
            exp.sort_indices()
            assert_csr_equal(PU.export(what, level),
                             CSR(exp.indptr, exp.indices, exp.data, exp.shape),
                             f"union level {level} object {what}")
    for P in singles + [PU]:
        P.close()


def test_batch_meets_every_tolerance_and_matches_separate_solves():
    ws = workloads()
    opts = plan()
    dev = [device_workload(w) for w in ws]
    As = [d[0] for d in dev]
    labels = [d[1] for d in dev]
    bs = [d[2].clone() for d in dev]
    bs[1] *= 1e8            # a badly scaled system still gets its own relative tolerance
    bs[2].zero_()           # and a zero right-hand side gives x = 0 exactly
    rtol = 1e-8
    xs, relres, info = m.batch_solve(As, labels, bs, opts, restart=30, rtol=rtol, maxit=300)
    print("batch", info, relres, flush=True)
    assert info["converged"]
    assert relres[2] == 0.0 and torch.count_nonzero(xs[2]).item() == 0
    for i, w in enumerate(ws):
        if i == 2:
            continue
        A = scipy_of(w)
        b = bs[i].cpu().numpy()
        x = xs[i].cpu().numpy()
        true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
        assert relres[i] <= rtol * (1 + 1e-9), (i, relres[i])
        assert abs(true - relres[i]) <= 1e-2 * rtol, (i, true, relres[i])
        P = m.Preconditioner(As[i], labels[i], opts)
        xi, inf = m.fgmres(As[i], bs[i], M=P, restart=30, rtol=rtol, maxit=300)
        P.close()
        # each system runs its own Arnoldi process: its iteration count is that of a
        # separate solve, up to the AMG's different aggregation
        its = info["system_iters"][i]
        assert abs(its - inf["iters"]) <= max(3, inf["iters"] // 5), (i, its, inf["iters"])
        xr = xi.cpu().numpy()
        # both solutions meet rtol; they differ by at most cond * 2 rtol
        cond = np.linalg.cond(A.toarray())
        err = np.linalg.norm(x - xr) / np.linalg.norm(xr)
        assert err <= 2 * cond * rtol, (i, err, cond)


def test_batch_of_one_equals_single_solve_tolerance():
    w = pm.two_phase(7, 6, 5, 5)
    A, labels, b = device_workload(w)
    xs, relres, info = m.batch_solve([A], [labels], [b], plan(), rtol=1e-7)
    assert info["converged"] and relres[0] <= 1e-7 * (1 + 1e-9)


def test_batch_argument_errors_leave_library_usable():
    L = m.lib()
    o = m.fgmres_opts(30, 100, 1e-6)
    copts = plan().to_c()
    rel = (C.c_double * 1)()
    st = L.mgr_batch_solve(0, None, None, None, None, C.byref(copts), C.byref(o), rel, None,
                           None, None)
    assert st == m.MGR_ERR_ARG
    w = pm.two_phase(5, 4, 4, 1)
    A, labels, b = device_workload(w)
    bad = m.Matrix.from_host(w.indptr[:-5], w.indices[:w.indptr[-6]], w.data[:w.indptr[-6]],
                             ncols=w.n)   # not square
    with pytest.raises(m.MgrError) as e:
        m.batch_solve([A, bad], [labels, labels], [b, b], plan())
    assert e.value.status == m.MGR_ERR_ARG
    xs, relres, info = m.batch_solve([A], [labels], [b], plan(), rtol=1e-6)
    assert info["converged"]
