"""Serving: every result is the same alone and in the mix (bitwise: each request runs the
same kernels in the same order on its own stream), admission never exceeds the budget,
cached setups are reused and evicted, oversize requests are rejected, and the footprint
estimate bounds the measured peak."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
m = pytest.importorskip("paper_1904_05960_amd.mgr355")
from paper_1904_05960_amd import serve  # noqa: E402


def log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ens():
    return serve.build_ensemble(5, 6, 13, seed=11, log=log)


def opts():
    o = m.paper_plan("two", precision="fp32")
    o.amg_frelax = m.AMG(coarse_size=48)
    o.amg_coarse = m.AMG(coarse_size=48)
    return o


def test_alone_equals_mix(ens):
    order = serve.request_order(len(ens), 3, seed=11)
    mix = serve.Server(opts(), 8 << 30, slots=4)
    recs_mix, _, xs_mix = serve.run_stream(mix, ens, order, rate=0.0, seed=11, newton=3, log=log)
    st = mix.stats()
    mix.close()
    alone = serve.Server(opts(), 8 << 30, slots=1)
    recs_alone, _, xs_alone = serve.run_stream(alone, ens, order, rate=0.0, seed=11, newton=3,
                                               log=log)
    alone.close()
    assert all(r["status"] == 0 for r in recs_mix + recs_alone)
    assert all(r["true_relres"] <= 1e-6 for r in recs_mix)
    assert len({r["slot"] for r in recs_mix}) > 1          # work really overlapped
    for a, b in zip(xs_mix, xs_alone):
        assert torch.equal(a, b)
    assert st["cache_hits"] == len(order) - len(ens)        # steps 1.. reuse the setup
    assert [r["iters"] for r in recs_mix] == [r["iters"] for r in recs_alone]


def test_refresh_equals_fresh_setup(ens):
    R = ens[1]
    srv = serve.Server(opts(), 8 << 30, slots=2)
    outs = []
    for k in range(3):
        A, b = R.step(k, 100 + k)
        x = torch.zeros_like(b)
        torch.cuda.current_stream().synchronize()   # inputs complete before the server reads
        t = srv.submit(A, R.labels, b, x, key=7, refresh=True)
        res = srv.wait(t)
        assert res["status"] == 0 and res["setup_reused"] == (k > 0)
        P = m.Preconditioner(A, R.labels, opts())
        x2, info = m.fgmres(A, b, M=P, restart=30, rtol=1e-6)
        P.close()
        assert torch.equal(x, x2)
        outs.append(res)
    srv.close()


def test_budget_evictions_and_rejection(ens):
    # a budget that holds about two setups: evictions happen, the budget is never exceeded
    sizes = []
    for R in ens:
        b = m.estimate_footprint(R.n, R.A0.nnz, opts()) + m.lib().fgmres_workspace_bytes(R.n, 30)
        sizes.append(b)
    budget = int(2.2 * max(sizes))
    srv = serve.Server(opts(), budget, slots=3)
    order = [(r, 0) for r in range(len(ens))] + [(r, 1) for r in range(len(ens))]
    recs, _, _ = serve.run_stream(srv, ens, order, rate=0.0, seed=3, newton=2, log=log)
    st = srv.stats()
    srv.close()
    assert all(r["status"] == 0 for r in recs)
    assert st["peak_reserved_bytes"] <= budget
    # deterministic eviction: one slot, one matrix under two keys, and a budget one byte
    # short of a cached setup plus a fresh request: the second key's request must evict the
    # first key's setup
    R = ens[0]
    need = m.estimate_footprint(R.n, R.A0.nnz, opts()) + m.lib().fgmres_workspace_bytes(R.n, 30)
    P = m.Preconditioner(R.A0, R.labels, opts())
    fp = P.footprint()
    P.close()
    srv = serve.Server(opts(), need + fp - 1, slots=1)
    for key in (1, 2):
        A, b = R.step(0, 9)
        x = torch.zeros_like(b)
        torch.cuda.current_stream().synchronize()
        res = srv.wait(srv.submit(A, R.labels, b, x, key=key))
        assert res["status"] == 0
    st = srv.stats()
    srv.close()
    assert st["evictions"] == 1 and st["peak_reserved_bytes"] <= need + fp - 1
    # a request larger than the whole budget completes with ALLOC
    tiny = serve.Server(opts(), 1 << 20, slots=1)
    R = ens[0]
    A, b = R.step(0, 1)
    x = torch.zeros_like(b)
    res = tiny.wait(tiny.submit(A, R.labels, b, x, key=1))
    tiny.close()
    assert res["status"] == m.MGR_ERR_ALLOC


def test_estimate_bounds_measured_peak(ens):
    R = max(ens, key=lambda r: r.n)
    A, b = R.step(0, 5)
    torch.cuda.synchronize()
    m.release_cache()
    live0, _ = m.alloc_stats(reset_peak=True)
    P = m.Preconditioner(A, R.labels, opts())
    x, info = m.fgmres(A, b, M=P, restart=30, rtol=1e-6)
    torch.cuda.synchronize()
    live1, peak = m.alloc_stats()
    P.close()
    est = m.estimate_footprint(R.n, A.nnz, opts()) + m.lib().fgmres_workspace_bytes(R.n, 30)
    log(f"  peak {peak - live0} estimate {est}")
    assert peak - live0 <= est


def test_small_requests_are_batched(ens):
    """With batching on, small requests queued together are solved by one block-diagonal
    solve; every request still meets its own tolerance, its residual checks on the host,
    and the budget holds."""
    srv = serve.Server(opts(), 8 << 30, slots=1, batch_rows=1 << 30, batch_max=4)
    order = [(r, 0) for r in range(len(ens))]
    recs, _, xs = serve.run_stream(srv, ens, order, rate=0.0, seed=5, newton=1, log=log)
    st = srv.stats()
    srv.close()
    assert all(r["status"] == 0 for r in recs)
    assert all(r["true_relres"] <= 1e-6 for r in recs)
    assert max(r["batch"] for r in recs) > 1
    assert all(1 <= r["batch"] <= 4 for r in recs)
    assert st["peak_reserved_bytes"] <= 8 << 30
    for (ri, k), r, x in zip(order, recs, xs):
        R = ens[ri]
        A, b = R.step(k, 5 * 7919 + ri * 101 + k)
        rp, ci, v = (t.cpu().numpy() for t in (A.row_ptr, A.col, A.val))
        import scipy.sparse as sp
        M = sp.csr_matrix((v, ci, rp), shape=(R.n, R.n))
        bb = b.cpu().numpy()
        rel = np.linalg.norm(bb - M @ x.cpu().numpy()) / np.linalg.norm(bb)
        assert rel <= 1e-6 * 1.001, (ri, rel, r)


def test_cache_hit_never_evicts_its_own_setup(ens):
    """A request whose key has a cached setup reserves only its workspace.  When making
    room for it must evict something, its own (idle) setup is not a candidate: the request
    waits for memory instead and then reuses the setup."""
    R1 = min(ens, key=lambda r: r.n)
    R2 = max(ens, key=lambda r: r.n)
    ws = lambda R: m.lib().fgmres_workspace_bytes(R.n, 30)  # noqa: E731
    probe = serve.Server(opts(), 8 << 30, slots=1)
    A, b = R1.step(0, 21)
    x = torch.zeros_like(b)
    torch.cuda.current_stream().synchronize()
    fp1 = probe.wait(probe.submit(A, R1.labels, b, x, key=1))["footprint"]
    probe.close()
    est2 = m.estimate_footprint(R2.n, R2.A0.nnz, opts()) + ws(R2)

    def run(budget):
        srv = serve.Server(opts(), budget, slots=2)
        A0, b0 = R1.step(0, 21)
        x0 = torch.zeros_like(b0)
        torch.cuda.current_stream().synchronize()
        r0 = srv.wait(srv.submit(A0, R1.labels, b0, x0, key=1))
        A2, b2 = R2.step(0, 22)
        A1, b1 = R1.step(1, 23)
        x2, x1 = torch.zeros_like(b2), torch.zeros_like(b1)
        torch.cuda.current_stream().synchronize()
        t2 = srv.submit(A2, R2.labels, b2, x2, key=2)
        t1 = srv.submit(A1, R1.labels, b1, x1, key=1)
        r1, r2 = srv.wait(t1), srv.wait(t2)
        st = srv.stats()
        srv.close()
        return r0, r1, r2, x1, st

    # key 2 fits beside the cached key-1 setup; key 1's workspace then does not
    budget = fp1 + est2 + ws(R1) - 1
    r0, r1, r2, x1, st = run(budget)
    q0, q1, q2, y1, _ = run(8 << 30)
    assert r0["status"] == r1["status"] == r2["status"] == 0
    assert r1["setup_reused"] and q1["setup_reused"]
    assert r1["iters"] == q1["iters"]
    assert torch.equal(x1, y1)
    assert st["peak_reserved_bytes"] <= budget


def test_failed_refresh_drops_the_setup(ens):
    """A refresh that fails (here a zero on the diagonal of A_FF: ZERO_PIVOT) leaves no
    half-built setup in the cache: the next request of that key builds a fresh one."""
    R = min(ens, key=lambda r: r.n)
    rp = R.A0.row_ptr.cpu().numpy()
    ci = R.A0.col.cpu().numpy()
    lab = R.labels.cpu().numpy()
    r = int(np.flatnonzero(lab == 0)[len(np.flatnonzero(lab == 0)) // 2])
    q = int(rp[r] + np.flatnonzero(ci[rp[r]:rp[r + 1]] == r)[0])
    srv = serve.Server(opts(), 8 << 30, slots=1)
    A, b = R.step(0, 31)
    x = torch.zeros_like(b)
    torch.cuda.current_stream().synchronize()
    assert srv.wait(srv.submit(A, R.labels, b, x, key=5))["status"] == 0
    val = R.A0.val.clone()
    val[q] = 0.0
    Az = m.Matrix(R.A0.row_ptr, R.A0.col, val)
    bz = Az.spmv(R.x_true)
    xz = torch.zeros_like(bz)
    torch.cuda.current_stream().synchronize()
    res = srv.wait(srv.submit(Az, R.labels, bz, xz, key=5, refresh=True))
    assert res["status"] == m.MGR_ERR_ZERO_PIVOT
    A1, b1 = R.step(1, 32)
    x1 = torch.zeros_like(b1)
    torch.cuda.current_stream().synchronize()
    res = srv.wait(srv.submit(A1, R.labels, b1, x1, key=5))
    srv.close()
    assert res["status"] == 0 and not res["setup_reused"]
    assert res["true_relres"] <= 1e-6
