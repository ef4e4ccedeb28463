"""Benchmark: MGR-preconditioned FGMRES time to a 1e-6 relative FP64 residual on one MI355X.

One step = the whole hot path on one synthetic Jacobian already resident in HBM:
mgr_setup (C/F splits, W_p, A_cor by pinned-order SpGEMM, G, coarse operators, both AMG
hierarchies, FP32 cast, graph capture on first apply) + fgmres_solve to rtol = 1e-6 +
mgr_destroy.  Default workload: three-phase poromechanics on a 96^3 cell grid (5,392,227
unknowns, 371,569,257 nonzeros), four-level MGR in the paper's reduction order
(displacement with an FP32 3x3-block AMG F-relaxation, then gas saturation, water
saturation, pressure AMG), FP32 hierarchy inside FP64 FGMRES(64).  The two-phase 64^3
case (1,348,163 unknowns) is also timed and reported under "two_phase_64".

    python bench.py [--steps K] [--warmup W] [--workload three|two] [--size 96]
                    [--precision fp32|fp64]
                    [--plan paper|satfirst] [--drop-tol TAU] [--no-cpu-baseline]
                    [--global-smoother block_jacobi|block_gs|ilu] [--global-sweeps 4] [--global-omega 0.9]
                    [--ilu-level 1] [--ilu-sweeps 3] [--ilu-tri-sweeps 3]

Prints one JSON line.  The dominant kernel's duration is measured live with HIP events
recorded on its own stream around every launch inside the timed steps.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


def kernel_source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_from_profile(name, src):
    """HBM bytes per launch from a committed counter summary, or None when absent or when
    the kernel source changed since the counters were taken."""
    p = os.path.join(PROFILES, name)
    if not os.path.exists(p):
        return None
    text = open(p).read()
    mh = re.search(r"source_sha256_16:\s*([0-9a-f]+)", text)
    mt = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not mh or not mt or mh.group(1) != kernel_source_hash(src):
        return None
    return float(mt.group(1))


def _two(n):
    from workloads import poromech as pm
    return pm.two_phase(n, n, n, 1)


def _three(n):
    from workloads import poromech as pm
    return pm.three_phase(n, n, n, 3)


# name: (generator by cells per side, CPU-baseline sample size, model, reduction, description)
WORKLOADS = {
    "two": (_two, 24, "two", "displacement -> saturation -> pressure AMG",
            "two-phase poromechanics Jacobian, {n}^3 cells, log10 k ~ N(-13,1) corr. 8 cells, "
            "Corey 2, s ~ U[0.2,0.8] (seed 1)"),
    "three": (_three, 20, "three",
              "displacement -> gas saturation -> water saturation -> pressure AMG",
              "three-phase poromechanics Jacobian, {n}^3 cells, ln k ~ N(ln 1e-13, 1.5^2) corr. "
              "12 cells, s_w ~ U[0.2,0.5], s_g ~ U[0.05,0.3] (seed 3)"),
}


def cpu_baseline(size_full_n, restart, workload, gpu_iters):
    """The oracle (FP64, NumPy/SciPy, untuned) on a bounded sample of the same workload
    recipe (24^3 two-phase, 20^3 three-phase): setup + FGMRES to 1e-6.  Its setup time is
    scaled by unknowns; its time per FGMRES iteration is scaled by unknowns and multiplied
    by the iteration count of the GPU run at full size (the sample itself needs a
    different number of iterations)."""
    from oracle import krylov as okry
    from oracle import mgr as omgr
    from oracle.sparse import CSR
    from paper_1904_05960_amd import mgr355 as m
    from tests.helpers import oracle_plan
    gen, ns = WORKLOADS[workload][0], WORKLOADS[workload][1]
    w = gen(ns)
    A = CSR(w.indptr, w.indices, w.data, (w.n, w.n))
    plan = oracle_plan(m.paper_plan(WORKLOADS[workload][2]))
    c0, t0 = os.times(), time.perf_counter()
    H = omgr.setup(A, w.labels, plan)
    t1 = time.perf_counter()
    r = okry.fgmres(A.matvec, lambda v: omgr.apply(H, v), w.b, restart=restart, rtol=1e-6,
                    maxit=500)
    t2, c1 = time.perf_counter(), os.times()
    cpu = (c1.user - c0.user) + (c1.system - c0.system)
    wall = t2 - t0
    scale = size_full_n / w.n
    per_it = (t2 - t1) / max(r.iters, 1)
    value = ((t1 - t0) + per_it * gpu_iters) * scale
    return {
        "value": round(value * 1e3, 1), "unit": "ms",
        "cores": max(1, round(cpu / wall)),
        "kind": "oracle",
        "sample": (f"oracle setup + FGMRES({restart}) to 1e-6 on the {w.name} grid of the same "
                   f"recipe ({w.n} unknowns: setup {1e3*(t1-t0):.0f} ms, {r.iters} iterations "
                   f"in {1e3*(t2-t1):.0f} ms = {1e3*per_it:.1f} ms each); value = (setup + "
                   f"{gpu_iters} iterations, the GPU run's count) x {scale:.2f} (unknowns ratio)"),
        "host_cpus": os.cpu_count(),
    }


def stream_copy_gbs(m, torch, nbytes=1 << 30, reps=5):
    """Rate of the library's plain copy kernel on 1 GiB (read + write bytes / time): the
    achievable HBM rate on this device, reported beside the SpMV rate.  Profiled runs also
    use its counters to calibrate FETCH_SIZE / WRITE_SIZE."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    m.stream_copy(src, dst, s)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(s)
    for _ in range(reps):
        m.stream_copy(src, dst, s)
    ev[1].record(s)
    torch.cuda.synchronize()
    return 2.0 * nbytes * reps / (ev[0].elapsed_time(ev[1]) * 1e-3) / 1e9


def make_opts(m, a, model, precision):
    mk0 = m.paper_plan if a.plan == "paper" else m.saturation_first_plan
    kw = dict(precision=precision)
    if a.plan == "paper":
        kw.update(global_smoother=a.global_smoother, global_sweeps=a.global_sweeps)
        if a.sat_nmax is not None:
            kw.update(sat_nmax=a.sat_nmax)
    opts = mk0(model, **kw)
    if a.drop_tol is not None:
        for L in opts.levels:
            if 0 in L.f_labels:
                L.nmax, L.drop_tol = -1, float(a.drop_tol)
    if a.coarse_size is not None:
        opts.amg_frelax = m.AMG(coarse_size=a.coarse_size)
        opts.amg_coarse = m.AMG(coarse_size=a.coarse_size)
    if a.theta_frelax is not None:
        opts.amg_frelax.theta0 = float(a.theta_frelax)
    if a.theta_coarse is not None:
        opts.amg_coarse.theta0 = float(a.theta_coarse)
    for L in opts.levels:
        if L.global_smoother == "ilu":
            L.ilu_level, L.ilu_sweeps = a.ilu_level, a.ilu_sweeps
            L.ilu_tri_sweeps = a.ilu_tri_sweeps
        if L.global_smoother != "none":
            if a.global_omega is not None:
                L.global_omega = float(a.global_omega)
            if a.sat_frelax_sweeps is not None and L.frelax == "jacobi":
                L.frelax_sweeps = int(a.sat_frelax_sweeps)
            if a.sat_frelax_omega is not None and L.frelax == "jacobi":
                L.frelax_omega = float(a.sat_frelax_omega)
    return opts


def dropping_text(a):
    disp = ("N_max = 4" if a.drop_tol is None else f"tolerance {a.drop_tol}") + \
        " on the displacement level"
    sat = a.sat_nmax if a.sat_nmax is not None else (4 if a.workload == "three" else -1)
    return disp + ("; Galerkin on the saturation levels" if sat < 0
                   else f"; N_max = {sat} on the saturation levels")


def to_bsr3(m, torch, A):
    """The device CSR matrix A (rows and columns in groups of three) as BSR with 3x3
    row-major blocks: every block holding an entry of A, zeros stored for its other
    entries.  Input preparation on the device with torch, outside the timed region."""
    n = A.nrows
    rows = torch.repeat_interleave(torch.arange(n, device="cuda"),
                                   A.row_ptr[1:] - A.row_ptr[:-1])
    cols = A.col.to(torch.int64)
    nbc = (A.ncols + 2) // 3
    key = (rows // 3) * nbc + cols // 3
    del cols
    ukey, inv = torch.unique(key, sorted=True, return_inverse=True)
    pos = (rows % 3) * 3 + A.col.to(torch.int64) % 3
    del rows, key
    blocks = torch.zeros(ukey.numel() * 9, dtype=torch.float64, device="cuda")
    blocks[inv * 9 + pos] = A.val
    del inv, pos
    brow = ukey // nbc
    indptr = torch.zeros(n // 3 + 1, dtype=torch.int64, device="cuda")
    indptr[1:] = torch.cumsum(torch.bincount(brow, minlength=n // 3), 0)
    bcol = (ukey % nbc).to(torch.int32)
    torch.cuda.synchronize()
    return m.Matrix(indptr, bcol, blocks, ncols=A.ncols, block=3)


class Case:
    """One workload resident in HBM, with the step (setup + FGMRES to 1e-6 + destroy)."""

    def __init__(self, m, torch, a, workload, size):
        t = time.perf_counter()
        self.w = WORKLOADS[workload][0](size)
        print(f"[bench] generated {self.w.name}: n={self.w.n} nnz={self.w.nnz} in "
              f"{time.perf_counter()-t:.1f}s", file=sys.stderr, flush=True)
        self.m, self.torch, self.a, self.model = m, torch, a, WORKLOADS[workload][2]
        w = self.w
        self.A = m.Matrix.from_host(w.indptr, w.indices, w.data)
        # the outer FGMRES matrix: the same operator as 3x3 blocks when every row group of
        # three (displacement nodes, three-phase cells) is blocked, else the CSR itself
        self.outer_block = 3 if (a.outer == "bsr3" and workload == "three") else 1
        self.Aout = to_bsr3(m, torch, self.A) if self.outer_block == 3 else self.A
        self.labels = torch.as_tensor(w.labels).cuda()
        self.b = torch.as_tensor(w.b).cuda()
        self.x = torch.zeros_like(self.b)
        self.work = m.Workspace(w.n, a.restart)
        self.stream = torch.cuda.current_stream()

    def step(self, prec, record=None):
        m, torch = self.m, self.torch
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(self.stream)
        P = m.Preconditioner(self.A, self.labels, make_opts(m, self.a, self.model, prec))
        ev[1].record(self.stream)
        self.x.zero_()
        _, info = m.fgmres(self.Aout, self.b, x=self.x, M=P, restart=self.a.restart, rtol=1e-6,
                           maxit=1000, work=self.work)
        ev[2].record(self.stream)
        P.close()
        if record is not None:
            record.append((ev, info))
        return info

    def errors(self):
        import numpy as np
        xs = self.x.cpu().numpy()
        w = self.w
        true = float(np.linalg.norm(w.b - w.scipy() @ xs) / np.linalg.norm(w.b))
        err = float(np.linalg.norm(xs - w.x_true) / np.linalg.norm(w.x_true))
        return true, err

    def close(self):
        del self.A, self.Aout, self.labels, self.b, self.x, self.work
        self.torch.cuda.synchronize()
        self.torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="three", choices=sorted(WORKLOADS))
    ap.add_argument("--size", type=int, default=None, help="cells per side (96 three, 64 two)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--plan", default="paper", choices=["paper", "satfirst"])
    ap.add_argument("--global-smoother", default="block_jacobi",
                    choices=["block_jacobi", "block_gs", "ilu"])
    ap.add_argument("--coarse-size", type=int, default=None,
                    help="AMG coarsest-grid size of both AMG hierarchies (default 256)")
    ap.add_argument("--theta-frelax", type=float, default=None,
                    help="strength threshold theta_0 of the displacement AMG (default 0.08)")
    ap.add_argument("--theta-coarse", type=float, default=None,
                    help="strength threshold theta_0 of the pressure AMG (default 0.08)")
    ap.add_argument("--ilu-level", type=int, default=1)
    ap.add_argument("--ilu-sweeps", type=int, default=3)
    ap.add_argument("--ilu-tri-sweeps", type=int, default=3)
    ap.add_argument("--global-sweeps", type=int, default=4)
    ap.add_argument("--global-omega", type=float, default=None,
                    help="weight of the block-Jacobi sweeps after the first (default: the "
                         "plan's, 0.9)")
    ap.add_argument("--sat-frelax-sweeps", type=int, default=None,
                    help="Jacobi F-relaxation sweeps on the saturation levels (default 1)")
    ap.add_argument("--sat-frelax-omega", type=float, default=None,
                    help="weight of that Jacobi F-relaxation (default 1)")
    ap.add_argument("--drop-tol", type=float, default=None,
                    help="tolerance form of G on the displacement level instead of N_max = 4")
    ap.add_argument("--sat-nmax", type=int, default=None,
                    help="N_max on the saturation levels (-1: Galerkin; default: 4 for the "
                         "three-phase model, Galerkin for two-phase)")
    ap.add_argument("--restart", type=int, default=64)
    ap.add_argument("--outer", default="bsr3", choices=["bsr3", "csr"],
                    help="outer FGMRES matrix of the three-phase workload: 3x3 blocks or CSR")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64-hierarchy step")
    ap.add_argument("--no-two-phase", action="store_true",
                    help="skip the extra two-phase 64^3 measurement")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1904_05960_amd import mgr355 as m

    torch.cuda.set_device(0)
    if a.size is None:
        a.size = 64 if a.workload == "two" else 96
    c = Case(m, torch, a, a.workload, a.size)

    for i in range(a.warmup):
        c.step(a.precision)
        print(f"[bench] warmup {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    m.profile_enable(1, True)            # HIP events around every outer SpMV launch
    rec = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        c.step(a.precision, rec)
        print(f"[bench] step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, spmv_ms, spmv_bytes = m.profile_read(1)
    m.profile_enable(1, False)
    ms_step = (t1 - t0) * 1e3 / a.steps
    setup_ms = [r[0][0].elapsed_time(r[0][1]) for r in rec]
    solve_ms = [r[0][1].elapsed_time(r[0][2]) for r in rec]
    info = rec[-1][1]
    true, err = c.errors()
    print(f"[bench] timed {a.steps} steps: {ms_step:.1f} ms/step, iters {info['iters']}",
          file=sys.stderr, flush=True)

    compare = None
    if not a.no_compare:
        other = "fp64" if a.precision == "fp32" else "fp32"
        c.step(other)                     # warm-up of the other precision
        r2 = []
        for _ in range(3):
            c.step(other, r2)
        torch.cuda.synchronize()
        tot = [r[0][0].elapsed_time(r[0][2]) for r in r2]
        compare = {"precision": other, "ms": round(float(np.median(tot)), 2),
                   "of": "median of 3 steps after 1 warm-up",
                   "iters": r2[-1][1]["iters"], "true_relres": r2[-1][1]["true_relres"]}
        print(f"[bench] {other} hierarchy: {compare['ms']} ms/step", file=sys.stderr, flush=True)
    c.close()

    two = None
    if not a.no_two_phase and not (a.workload == "two" and a.size == 64):
        c2 = Case(m, torch, a, "two", 64)
        c2.step(a.precision)
        r3 = []
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(5):
            c2.step(a.precision, r3)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        t2r, _ = c2.errors()
        two = {"workload": WORKLOADS["two"][4].format(n=64), "unknowns": c2.w.n,
               "nnz": c2.w.nnz, "ms_per_step": round((t3 - t2) * 1e3 / 5, 2),
               "setup_ms": round(float(np.median([r[0][0].elapsed_time(r[0][1]) for r in r3])), 2),
               "solve_ms": round(float(np.median([r[0][1].elapsed_time(r[0][2]) for r in r3])), 2),
               "iterations": r3[-1][1]["iters"], "true_relres": t2r}
        print(f"[bench] two-phase 64^3: {two['ms_per_step']} ms/step", file=sys.stderr, flush=True)
        c2.close()

    copy_gbs = stream_copy_gbs(m, torch)
    avg_launch_ms = spmv_ms / max(launches, 1)
    bytes_per_launch = spmv_bytes / max(launches, 1)
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    # counter traffic is recorded for the default sizes of the two workloads
    traffic = None
    prof = {("two", 64, 1): "spmv_outer_twophase_64.md",
            ("three", 96, 3): "spmv_outer_bsr3_threephase_96.md"}.get(
                (a.workload, a.size, c.outer_block))
    if prof is not None:
        traffic = traffic_from_profile(
            prof, os.path.join(ROOT, "paper_1904_05960_amd", "csrc", "krylov.hip"))
    w = c.w
    out = {
        "metric": "MGR-FGMRES time-to-1e-6 relative FP64 residual (setup + solve)",
        "value": round(ms_step, 2),
        "unit": "ms",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32 hierarchy + f64 Krylov" if a.precision == "fp32" else "f64"),
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS[a.workload][4].format(n=a.size),
            "unknowns": w.n, "nnz": w.nnz,
            "reduction": (WORKLOADS[a.workload][3] if a.plan == "paper"
                          else "saturations -> displacement -> pressure AMG"),
            "hierarchy_precision": a.precision, "krylov": f"FGMRES({a.restart}) FP64, CGS2",
            "outer_matrix": "BSR 3x3 FP64" if c.outer_block == 3 else "CSR FP64",
            "global_smoother": f"{a.global_smoother} x{a.global_sweeps}" + (
                f" (ILU({a.ilu_level}), {a.ilu_sweeps} factor sweeps, {a.ilu_tri_sweeps} "
                f"triangular sweeps)" if a.global_smoother == "ilu" else "") + (
                f", omega {a.global_omega if a.global_omega is not None else 0.9}"
                if a.global_smoother == "block_jacobi" else ""),
            "dropping": dropping_text(a),
            "rtol": 1e-6, "parallelism": "single GPU",
        },
        "iterations": info["iters"],
        "true_relres": true,
        "solution_error_vs_x_true": err,
        "setup_ms": round(float(np.median(setup_ms)), 2),
        "solve_ms": round(float(np.median(solve_ms)), 2),
        "compare_other_precision": compare,
        "two_phase_64": two,
        "roofline": {
            "kernel": ("outer FP64 BSR3 SpMV (k_bsr3_lane, a lane per 3x3 block, 512-block windows)"
                       if c.outer_block == 3 else
                       "outer FP64 CSR-stream SpMV (k_spmv_stream, 2048-entry row blocks)"),
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": round(avg_launch_ms, 5),
            "launches_timed": launches,
            "stream_copy_gbs": round(copy_gbs, 1),
        },
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w.n, a.restart, a.workload, info["iters"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
