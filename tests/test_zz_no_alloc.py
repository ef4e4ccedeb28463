"""fgmres_solve_noalloc (static per-device workspace, nothing allocated in the call) against
fgmres_solve (caller workspace) through the C ABI: the same launches in the same order, so
bitwise the same solution and the same iteration count, on two calls in a row, the second
with a smaller system; a system whose workspace exceeds the static size is refused."""
import numpy as np
import pytest

from tests.helpers import device_workload
from workloads import poromech as pm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
m = pytest.importorskip("paper_1904_05960_amd.mgr355")


def small_amg(opts, coarse_size=48):
    opts.amg_frelax = m.AMG(coarse_size=coarse_size)
    opts.amg_coarse = m.AMG(coarse_size=coarse_size)
    return opts


@pytest.mark.parametrize("precond", [True, False])
def test_noalloc_equals_fgmres_solve(precond):
    for nc in (8, 5):                       # second call smaller
        w = pm.two_phase(nc, nc, nc, 1)
        print(f"[noalloc] two-phase {nc}^3 n={w.n} preconditioned={precond}", flush=True)
        A, labels, b = device_workload(w)
        P = m.Preconditioner(A, labels, small_amg(m.paper_plan("two"))) if precond else None
        maxit = 400 if precond else 60
        x1, i1 = m.fgmres(A, b, M=P, restart=30, rtol=1e-8, maxit=maxit, raise_on_fail=False)
        x2, i2 = m.fgmres_noalloc(A, b, M=P, restart=30, rtol=1e-8, maxit=maxit,
                                  raise_on_fail=False)
        torch.cuda.synchronize()
        assert i1["iters"] == i2["iters"] and i1["converged"] == i2["converged"]
        assert i1["true_relres"] == i2["true_relres"]
        assert torch.equal(x1, x2)
        if precond:
            assert i2["converged"]
            xs = x2.cpu().numpy()
            rel = np.linalg.norm(w.b - w.scipy() @ xs) / np.linalg.norm(w.b)
            assert rel <= 1e-8 * 1.0000001
            P.close()


def test_noalloc_limits():
    lim = m.lib().fgmres_noalloc_max_bytes()
    assert lim == 64 << 20
    # a system whose workspace does not fit: refused with ARG before any launch
    n = 1
    while m.lib().fgmres_workspace_bytes(n, 30) <= lim:
        n *= 2
    A = m.Matrix(torch.zeros(n + 1, dtype=torch.int64, device="cuda"),
                 torch.zeros(0, dtype=torch.int32, device="cuda"),
                 torch.zeros(0, dtype=torch.float64, device="cuda"))
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    with pytest.raises(m.MgrError) as e:
        m.fgmres_noalloc(A, b, restart=30)
    assert e.value.status == m.MGR_ERR_ARG
    # a preconditioner that has never been applied is refused
    w = pm.biot_single_phase(4, 4, 4, 0)
    A, labels, b = device_workload(w)
    P = m.Preconditioner(A, labels, small_amg(m.paper_plan("biot1", coarse="dense"), 24))
    with pytest.raises(m.MgrError) as e:
        m.fgmres_noalloc(A, b, M=P)
    assert e.value.status == m.MGR_ERR_ARG
    P.apply(b)
    x, info = m.fgmres_noalloc(A, b, M=P, rtol=1e-8, maxit=200)
    assert info["converged"]
    P.close()
