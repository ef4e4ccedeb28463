"""Serving: Python wrapper of the library's request loop and a replay driver.

`Server` wraps mgr_server_* (include/mgr355.h): worker slots with their own HIP streams,
HBM admission by footprint, a setup cache keyed by realization.  `run_stream` replays an
ensemble of Jacobians (realizations of different mesh sizes, several Newton steps each
re-assembled on the device at a perturbed state, same sparsity pattern) with Poisson
arrivals and reports solves/s and p50/p99 latency.

    python -m paper_1904_05960_amd.serve [--realizations 64] [--newton 8] [--nmin 16]
        [--nmax 80] [--rate 50] [--slots 4] [--budget-gb 200] [--precision fp32]
        [--restart 64] [--input-pool-gb 32] [--compare-fp64-serial]
        [--batch-rows R] [--batch-max 16]
    python -m paper_1904_05960_amd.serve --batch-compare K [--nmin 16]
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import sys
import time

import numpy as np

from . import mgr355 as m


class Server:
    def __init__(self, opts: m.Options, budget_bytes: int = 64 << 30, slots: int = 4,
                 restart: int = 30, rtol: float = 1e-6, maxit: int = 1000, cache: bool = True,
                 batch_rows: int = 0, batch_max: int = 16):
        L = m.lib()
        cfg = m.mgr_server_config()
        L.mgr_server_default_config(C.byref(cfg))
        cfg.budget_bytes = int(budget_bytes)
        cfg.slots = int(slots)
        cfg.opts = opts.to_c()
        cfg.fopts = m.fgmres_opts(int(restart), int(maxit), float(rtol))
        cfg.cache_setups = int(cache)
        cfg.batch_rows = int(batch_rows)
        cfg.batch_max = int(batch_max)
        self._cfg = cfg
        h = C.c_void_p()
        m._check(L.mgr_server_create(C.byref(cfg), C.byref(h)))
        self.h = h
        self._keep = {}

    def submit(self, A: m.Matrix, labels, b, x, key: int, refresh: bool = False,
               last_use: bool = False) -> int:
        r = m.mgr_request()
        r.A = C.pointer(A.c)
        r.nnz = A.nnz
        r.labels = labels.data_ptr()
        r.b = b.data_ptr()
        r.x = x.data_ptr()
        r.key = int(key)
        r.refresh_setup = int(refresh)
        r.last_use = int(last_use)
        t = C.c_uint64()
        m._check(m.lib().mgr_server_submit(self.h, C.byref(r), C.byref(t)))
        self._keep[t.value] = (A, labels, b, x)     # device arrays live until completion
        return int(t.value)

    def wait(self, ticket: int) -> dict:
        res = m.mgr_result()
        st = m.lib().mgr_server_wait(self.h, C.c_uint64(ticket), C.byref(res))
        self._keep.pop(ticket, None)
        return dict(status=st, iters=res.iters, setup_reused=bool(res.setup_reused),
                    slot=res.slot, true_relres=res.true_relres, t_submit_ms=res.t_submit_ms,
                    t_admit_ms=res.t_admit_ms, t_start_ms=res.t_start_ms,
                    t_end_ms=res.t_end_ms, setup_ms=res.setup_ms, solve_ms=res.solve_ms,
                    footprint=int(res.footprint), batch=int(res.batch))

    def poll(self, ticket: int) -> int:
        return int(m.lib().mgr_server_poll(self.h, C.c_uint64(ticket)))

    def stats(self) -> dict:
        s = m.mgr_server_stats_t()
        m._check(m.lib().mgr_server_stats(self.h, C.byref(s)))
        return {f: int(getattr(s, f)) for f, _ in s._fields_}

    def close(self):
        if getattr(self, "h", None):
            m.lib().mgr_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------------------
# ensemble of requests
class Realization:
    """One permeability realization on the device: the library's two-phase model of its
    cells (mgr_poro_*), the state its base Jacobian is taken at, and its Newton steps."""

    def __init__(self, idx: int, n: int, seed: int, perturbation: float = 0.1):
        import torch
        from workloads import poromech as pm
        from . import poro
        w = pm.two_phase(n, n, n, seed)
        self.idx, self.n_cells, self.n = idx, n, w.n
        self.model = poro.Model(poro.default_params(n, n, n, nu=w.meta["nu"]), w.meta["perm"],
                                w.meta["young"], w.fixed)
        rp, ci, _, lab = self.model.export()
        self.row_ptr = torch.as_tensor(rp).cuda()
        self.col = torch.as_tensor(ci).cuda()
        self.labels = torch.as_tensor(lab).cuda()
        nu = self.model.nu
        x0 = np.zeros(self.n)
        x0[nu::2] = w.meta["state"]["S_w"]
        x0[nu + 1::2] = w.meta["state"]["p"]
        self.x0 = torch.as_tensor(x0).cuda()
        self.nu = nu
        self.perturbation = perturbation
        self.free_u = torch.as_tensor(~w.fixed).cuda()
        self.x_true = torch.as_tensor(w.x_true).cuda()
        self.nnz = int(w.nnz)
        self._F = torch.empty(self.n, dtype=torch.float64, device="cuda")

    def input_bytes(self) -> int:
        """Device bytes of one materialized request (values, b, x)."""
        return 8 * self.nnz + 16 * self.n

    @property
    def A0(self):
        """The Jacobian at the base state (assembled once, on first use)."""
        if getattr(self, "_A0", None) is None:
            self._A0 = self.step(0, 0)[0]
        return self._A0

    def state(self, k: int, seed: int):
        """The state of Newton step k: the base state (k = 0), or the base state perturbed
        with iid normals seeded by (realization, k), scaled by `perturbation` times 1e4 Pa
        for pressure, 0.01 for saturation (kept in [0.05, 0.95]) and 1e-5 m for the free
        displacement dofs.  The default 0.1 keeps a cached setup of step 0 useful (at 24^3
        cells: 36 FGMRES iterations against 32 with a fresh setup; with 1.0, 63 against 30,
        and the gap widens with the mesh)."""
        import torch
        if k == 0:
            return self.x0
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        z = torch.randn(self.n, generator=g, device="cuda", dtype=torch.float64)
        x = self.x0.clone()
        nu = self.nu
        a = self.perturbation
        x[:nu] += (a * 1e-5) * z[:nu] * self.free_u
        x[nu::2] = (x[nu::2] + (a * 0.01) * z[nu::2]).clamp(0.05, 0.95)
        x[nu + 1::2] += (a * 1e4) * z[nu + 1::2]
        return x

    def step(self, k: int, seed: int):
        """Newton step k: the Jacobian re-assembled on the device at state(k, seed) (previous
        time level: the base state), same pattern; b = A x_true."""
        import torch
        from . import mgr355 as mm
        self.model.assemble(self.state(k, seed), self.x0, F=self._F)
        val = torch.empty(self.nnz, dtype=torch.float64, device="cuda")
        mm._check(mm.lib().mgr_poro_export(self.model.h, None, None, mm._ptr(val), None,
                                           mm._stream()))
        A = m.Matrix(self.row_ptr, self.col, val)
        b = A.spmv(self.x_true)
        return A, b


def build_ensemble(realizations: int, nmin: int, nmax: int, seed: int, log=print,
                   perturbation: float = 0.1):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nmin, nmax + 1, size=realizations)
    ens = []
    for i, n in enumerate(sizes):
        t = time.perf_counter()
        ens.append(Realization(i, int(n), seed * 1000 + i, perturbation))
        log(f"[serve] realization {i}: {n}^3 cells, {ens[-1].n} unknowns "
            f"({time.perf_counter() - t:.1f}s)")
    return ens


def request_order(realizations: int, newton: int, seed: int):
    """A uniformly random interleaving of the realizations' step sequences, each
    realization's steps in order."""
    rng = np.random.default_rng(seed + 1)
    seq = np.repeat(np.arange(realizations), newton)
    rng.shuffle(seq)
    nxt = np.zeros(realizations, dtype=int)
    out = []
    for r in seq:
        out.append((int(r), int(nxt[r])))
        nxt[r] += 1
    return out


def run_stream(server: Server, ens, order, rate: float, seed: int, newton: int,
               refresh: bool = False, log=print, input_pool_bytes: int = 32 << 30,
               keep_x: bool = True):
    """Open-loop replay: request i arrives at the i-th event of a Poisson process of the
    given rate.  Its matrix values and right-hand side are materialized on the device when
    it arrives; at most `input_pool_bytes` of materialized inputs are held by requests in
    flight (past that, the replay first waits for the oldest one to finish).  Latency runs
    from the arrival time to completion, so such waits count.  Returns per-request
    records, the wall time and the solutions (if keep_x)."""
    import collections
    import torch
    rng = np.random.default_rng(seed + 2)
    gaps = rng.exponential(1.0 / rate, size=len(order)) if rate > 0 else np.zeros(len(order))
    arrivals = np.cumsum(gaps)
    inflight = collections.deque()          # (ticket, index, bytes)
    held = 0
    recs = [None] * len(order)
    xs = [None] * len(order)
    late = np.zeros(len(order))             # seconds from arrival to submission

    def finish_oldest():
        nonlocal held
        t, j, nb = inflight.popleft()
        res = server.wait(t)
        res["realization"], res["newton_step"] = order[j]
        res["n"] = ens[order[j][0]].n
        res["latency_ms"] = res["t_end_ms"] - res["t_submit_ms"] + 1e3 * late[j]
        recs[j] = res
        held -= nb
        done = sum(1 for r_ in recs if r_ is not None)
        if done % 64 == 0 or done == len(order):
            log(f"[serve] {done}/{len(order)} requests done, "
                f"{time.perf_counter() - t0:.1f}s")

    # inputs are materialized on a stream of their own and only that stream is awaited: a
    # device-wide synchronisation is refused while a worker thread captures a V-cycle graph
    side = torch.cuda.Stream()
    t0 = time.perf_counter()
    for i, (r, k) in enumerate(order):
        delay = arrivals[i] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        need = ens[r].input_bytes()
        while inflight and held + need > input_pool_bytes:
            finish_oldest()
        with torch.cuda.stream(side):
            A, b = ens[r].step(k, seed * 7919 + r * 101 + k)
            x = torch.zeros_like(b)
        side.synchronize()                    # inputs complete before the server reads them
        late[i] = max(0.0, time.perf_counter() - t0 - arrivals[i])
        t = server.submit(A, ens[r].labels, b, x, key=r, refresh=refresh,
                          last_use=(k == newton - 1))
        inflight.append((t, i, need))
        held += need
        if keep_x:
            xs[i] = x
    while inflight:
        finish_oldest()
    wall = time.perf_counter() - t0
    return recs, wall, xs


def summarize(recs, wall):
    lat = np.array([r["latency_ms"] for r in recs])
    ok = sum(1 for r in recs if r["status"] == 0)
    failed = {}
    for r in recs:
        if r["status"] != 0:
            failed[str(r["status"])] = failed.get(str(r["status"]), 0) + 1
    return dict(requests=len(recs), ok=ok, failed_by_status=failed,
                solves_per_s=len(recs) / wall,
                p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                mean_iters=float(np.mean([r["iters"] for r in recs])),
                max_relres=float(max(r["true_relres"] for r in recs)),
                setup_reuse=float(np.mean([r["setup_reused"] for r in recs])), wall_s=wall)


def batch_compare(nside: int, k: int, restart: int, precision: str, seed: int, reps: int = 3):
    """k two-phase systems of nside^3 cells (different seeds): setup + FGMRES to 1e-6 one
    after another, against one mgr_batch_solve of all k.  Median of `reps` runs each."""
    import torch
    from workloads import poromech as pm
    opts = m.paper_plan("two", precision=precision)
    sys_ = []
    for i in range(k):
        w = pm.two_phase(nside, nside, nside, seed + i)
        sys_.append((m.Matrix.from_host(w.indptr, w.indices, w.data),
                     torch.as_tensor(w.labels).cuda(), torch.as_tensor(w.b).cuda()))

    def one_by_one():
        its = []
        for A, lab, b in sys_:
            P = m.Preconditioner(A, lab, opts)
            _, info = m.fgmres(A, b, M=P, restart=restart, rtol=1e-6)
            P.close()
            its.append(info["iters"])
        return its

    def batched():
        _, rel, info = m.batch_solve([s[0] for s in sys_], [s[1] for s in sys_],
                                     [s[2] for s in sys_], opts, restart=restart, rtol=1e-6)
        return info["system_iters"], max(rel)

    one_by_one(), batched()          # warm up
    t_one, t_bat = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = one_by_one()
        torch.cuda.synchronize()
        t_one.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        bits, worst = batched()
        torch.cuda.synchronize()
        t_bat.append(time.perf_counter() - t0)
    n = sys_[0][0].c.nrows
    return {"metric": "ms per small system (setup + FGMRES to 1e-6)", "systems": k,
            "cells": f"{nside}^3", "unknowns_per_system": int(n), "precision": precision,
            "one_by_one_ms_per_system": 1e3 * float(np.median(t_one)) / k,
            "batched_ms_per_system": 1e3 * float(np.median(t_bat)) / k,
            "iters_one_by_one": its, "iters_batched": bits, "batched_max_relres": worst}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--realizations", type=int, default=64)
    ap.add_argument("--newton", type=int, default=8)
    ap.add_argument("--nmin", type=int, default=16)
    ap.add_argument("--nmax", type=int, default=80)
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--rates", default="",
                    help="comma-separated arrival rates: replay the same ensemble at each "
                         "(one JSON line per rate), e.g. to find where latency stops being "
                         "queueing-dominated")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--restart", type=int, default=64)
    ap.add_argument("--refresh", action="store_true", help="recompute setups each step")
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--perturbation", type=float, default=0.1,
                    help="size of a Newton step's state change (1: 1e4 Pa, 0.01, 1e-5 m)")
    ap.add_argument("--compare-fp64-serial", action="store_true")
    ap.add_argument("--input-pool-gb", type=float, default=32.0)
    ap.add_argument("--batch-rows", type=int, default=0,
                    help="batch requests of at most this many rows (0: off)")
    ap.add_argument("--batch-max", type=int, default=16)
    ap.add_argument("--batch-compare", type=int, default=0, metavar="K",
                    help="only time K systems of --nmin^3 cells solved one by one and batched")
    a = ap.parse_args(argv)
    if a.batch_compare:
        print(json.dumps(batch_compare(a.nmin, a.batch_compare, a.restart, a.precision,
                                       a.seed)), flush=True)
        return
    import torch
    torch.cuda.set_device(0)
    log = lambda *x: print(*x, file=sys.stderr, flush=True)  # noqa: E731
    ens = build_ensemble(a.realizations, a.nmin, a.nmax, a.seed, log, a.perturbation)
    order = request_order(a.realizations, a.newton, a.seed)
    pool = int(a.input_pool_gb * (1 << 30))
    if a.rates:
        for rate in [float(v) for v in a.rates.split(",")]:
            srv = Server(m.paper_plan("two", precision=a.precision),
                         int(a.budget_gb * (1 << 30)), a.slots, restart=a.restart,
                         batch_rows=a.batch_rows, batch_max=a.batch_max)
            recs, wall, _ = run_stream(srv, ens, order, rate, a.seed, a.newton, a.refresh,
                                       log, pool, keep_x=False)
            svc = np.array([r["t_end_ms"] - r["t_start_ms"] for r in recs])
            print(json.dumps({"mode": "served", "rate_per_s": rate, "slots": a.slots,
                              "precision": a.precision, **summarize(recs, wall),
                              "service_p50_ms": float(np.percentile(svc, 50)),
                              "service_p99_ms": float(np.percentile(svc, 99))}), flush=True)
            srv.close()
        return
    srv = Server(m.paper_plan("two", precision=a.precision), int(a.budget_gb * (1 << 30)),
                 a.slots, restart=a.restart, batch_rows=a.batch_rows, batch_max=a.batch_max)
    recs, wall, _ = run_stream(srv, ens, order, a.rate, a.seed, a.newton, a.refresh, log,
                               pool, keep_x=False)
    out = {"metric": "served MGR-FGMRES solves (1e-6), p50/p99 latency", "mode": "served",
           "precision": a.precision, "slots": a.slots, "rate_per_s": a.rate,
           "restart": a.restart, "batch_rows": a.batch_rows, "batch_max": a.batch_max,
           **summarize(recs, wall), "server": srv.stats()}
    srv.close()
    if a.compare_fp64_serial:
        srv = Server(m.paper_plan("two", precision="fp64"), int(a.budget_gb * (1 << 30)), 1,
                     restart=a.restart, cache=False)
        recs2, wall2, _ = run_stream(srv, ens, order, a.rate, a.seed, a.newton, False, log,
                                     pool, keep_x=False)
        out["fp64_one_at_a_time"] = summarize(recs2, wall2)
        srv.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
