"""Two-phase poromechanics on the GPU: residual / Jacobian assembly and Newton time steps
(Sec. 2-4), as a ctypes binding of the mgr_poro_* entry points of libmgr355 (argument
marshalling only: assembly, setup, FGMRES and the Newton loop run in the library).

    python -m paper_1904_05960_amd.poro --nx 32 --ny 32 --nz 8 --steps 60 \\
        --smoothers block_jacobi,block_gs,ilu

runs the same water line drive through a channelised reservoir once per global smoother
and prints, per time step, Newton iterations and FGMRES iterations, then one JSON line per
smoother with the totals (the global-smoother study of Sec. 6.3).
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import sys
import time

import numpy as np

from . import mgr355 as M


def default_params(nx, ny, nz, **over):
    p = M.mgr_poro_params()
    M.lib().mgr_poro_default_params(C.byref(p), int(nx), int(ny), int(nz))
    for k, v in over.items():
        if k in ("rho0", "comp", "visc"):
            getattr(p, k)[0], getattr(p, k)[1] = float(v[0]), float(v[1])
        else:
            setattr(p, k, v)
    return p


def newton_opts(**over):
    o = M.mgr_newton_opts()
    M.lib().mgr_newton_default_opts(C.byref(o))
    for k, v in over.items():
        setattr(o, k, v)
    return o


class Model:
    """The library's model object: cell data, the owned Jacobian and its labels."""

    def __init__(self, params, perm, young, fixed, wi=None, pbhp=None, qw=None, qo=None,
                 stream=None):
        import torch
        dev = torch.device("cuda")
        f64 = lambda a: None if a is None else torch.as_tensor(np.asarray(a, dtype=np.float64)).to(dev)  # noqa: E731
        self.params = params
        self._keep = [f64(perm), f64(young),
                      torch.as_tensor(np.asarray(fixed, dtype=np.uint8)).to(dev),
                      f64(wi), f64(pbhp), f64(qw), f64(qo)]
        h = C.c_void_p()
        M._check(M.lib().mgr_poro_create(C.byref(params), *[M._ptr(t) for t in self._keep],
                                         M._stream(stream), C.byref(h)))
        self.h = h
        self._keep = None
        sz = (C.c_int64 * 4)()
        M._check(M.lib().mgr_poro_sizes(self.h, sz))
        self.n, self.nnz, self.nu, self.ncell = (int(v) for v in sz)
        self.csr = M.mgr_csr()
        lab = C.c_void_p()
        M._check(M.lib().mgr_poro_matrix(self.h, C.byref(self.csr), C.byref(lab)))
        self.labels_ptr = lab
        self.mgr = C.c_void_p()      # MGR hierarchy of the Newton solves (built on demand)

    # matrices and vectors --------------------------------------------------------------
    def matrix(self):
        """A Matrix-like view of the owned Jacobian (for setup / FGMRES calls)."""
        return _OwnedMatrix(self)

    def export(self, stream=None):
        """Host copies (indptr, indices, data, labels) of the Jacobian and its labels."""
        import torch
        dev = torch.device("cuda")
        rp = torch.empty(self.n + 1, dtype=torch.int64, device=dev)
        ci = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
        v = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=dev)
        lab = torch.empty(self.n, dtype=torch.int8, device=dev)
        M._check(M.lib().mgr_poro_export(self.h, M._ptr(rp), M._ptr(ci), M._ptr(v), M._ptr(lab),
                                         M._stream(stream)))
        return (rp.cpu().numpy(), ci[: self.nnz].cpu().numpy(), v[: self.nnz].cpu().numpy(),
                lab.cpu().numpy())

    def labels(self):
        import torch
        lab = torch.empty(self.n, dtype=torch.int8, device="cuda")
        M._check(M.lib().mgr_poro_export(self.h, None, None, None, M._ptr(lab), M._stream()))
        return lab

    def set_dt(self, dt):
        M._check(M.lib().mgr_poro_set_dt(self.h, float(dt)))
        self.params.dt = float(dt)

    def assemble(self, x, x_old, F=None, jacobian=True, norms=False, stream=None):
        """F(x) (and the Jacobian into the owned matrix); with norms, also the per-type
        [sum of squares, max |.|] of the residual in state units."""
        import torch
        if F is None:
            F = torch.empty_like(x)
        nr = (C.c_double * 6)() if norms else None
        M._check(M.lib().mgr_poro_assemble(self.h, M._ptr(x), M._ptr(x_old), M._ptr(F),
                                           1 if jacobian else 0, nr, M._stream(stream)))
        if norms:
            return F, [(nr[0], nr[1]), (nr[2], nr[3]), (nr[4], nr[5])]
        return F

    # Newton ----------------------------------------------------------------------------
    def newton(self, x, x_old, opts: M.Options, restart=64, rtol=1e-6, maxit=400,
               nopts=None, stream=None):
        """One time step in place on x (device FP64); returns the step's statistics."""
        co = opts.to_c()
        fo = M.fgmres_opts(int(restart), int(maxit), float(rtol))
        no = nopts if nopts is not None else newton_opts()
        st = M.mgr_newton_stats()
        M._check(M.lib().mgr_poro_newton(self.h, C.byref(self.mgr), C.byref(co), C.byref(fo),
                                         M._ptr(x), M._ptr(x_old), C.byref(no), C.byref(st),
                                         M._stream(stream)))
        k = st.newton_iters
        return dict(newton_iters=k, linear_iters=st.linear_iters, backtracks=st.backtracks,
                    converged=bool(st.converged), setups=st.setups,
                    linear_failures=st.linear_failures,
                    lin_iters=[st.lin_iters[i] for i in range(k)],
                    merit=[st.merit[i] for i in range(k + 1)],
                    lambdas=[st.lambda_[i] for i in range(k)],
                    assemble_ms=st.assemble_ms, setup_ms=st.setup_ms, solve_ms=st.solve_ms)

    def close(self):
        if getattr(self, "mgr", None) is not None and self.mgr.value:
            M.lib().mgr_destroy(self.mgr)
            self.mgr = C.c_void_p()
        if getattr(self, "h", None) is not None and self.h.value:
            M.lib().mgr_poro_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _OwnedMatrix:
    """Duck-typed Matrix over the model's owned arrays (for Preconditioner / fgmres)."""

    def __init__(self, model: Model):
        self.c = model.csr
        self.nrows = self.ncols = model.n
        self.block = 1
        self._model = model

    @property
    def nnz(self):
        return self._model.nnz


def model_from_reservoir(res, **param_over):
    """A Model for the dict returned by workloads.poromech.channel_reservoir."""
    p = default_params(res["nx"], res["ny"], res["nz"], nu=res.get("nu", 0.25),
                       dt=res.get("dt", 86400.0), **param_over)
    return Model(p, res["perm"], res["young"], res["fixed"], res["wi"], res["pbhp"],
                 res["qw"], res["qo"])


def simulate(model: Model, x0, steps, opts: M.Options, restart=64, rtol=1e-6, maxit=400,
             nopts=None, log=None, max_cuts=8, growth=1.5):
    """Backward-Euler time stepping over `steps` steps of the model's dt (the target step):
    a step whose Newton iteration fails is retried from the previous level with dt halved
    (up to max_cuts times), and after a success dt grows by `growth` back towards the
    target.  The run ends at steps * target dt, or early when a step still fails with the
    smallest dt.  Returns (x, records), one record per accepted step (with its dt and the
    number of failed attempts before it)."""
    import torch
    x = torch.as_tensor(np.asarray(x0, dtype=np.float64)).to("cuda")
    x_old = x.clone()
    target = float(model.params.dt)
    t_end = steps * target
    t, dt = 0.0, target
    rec = []
    while t < t_end * (1.0 - 1e-12):
        x_old.copy_(x)
        dt = min(dt, t_end - t)
        model.set_dt(dt)
        fails, wasted = 0, 0
        t0 = time.perf_counter()
        while True:
            st = model.newton(x, x_old, opts, restart, rtol, maxit, nopts)
            if st["converged"] or fails >= max_cuts:
                break
            fails += 1
            wasted += st["linear_iters"]
            x.copy_(x_old)
            dt *= 0.5
            model.set_dt(dt)
        st["step"] = len(rec) + 1
        st["dt"] = dt
        st["cuts"] = fails
        st["failed_linear_iters"] = wasted      # FGMRES iterations of the failed attempts
        st["wall_ms"] = 1e3 * (time.perf_counter() - t0)
        rec.append(st)
        if log:
            log(st)
        if not st["converged"]:
            break
        t += dt
        dt = min(target, dt * growth)
    model.set_dt(target)
    return x, rec


def smoother_options(kind: str, precision="fp32", coupling="quasi_impes") -> M.Options:
    """MGR of the two-phase system (u, then s, then pressure AMG) with the given global
    smoother on the (s, p) level: block Jacobi x3, multicolour block Gauss-Seidel x3 (the
    hybrid block GS of the paper), or ILU(1) by fine-grained sweeps, one application.
    The saturation level uses the quasi-IMPES coupling by default: on the Jacobians of a
    running simulation it needs about half the FGMRES iterations of the full coupling."""
    qi = coupling == "quasi_impes"
    if kind == "block_jacobi":
        return M.paper_plan("two", precision=precision, quasi_impes=qi, global_sweeps=3,
                            global_omega=1.0)
    if kind == "block_gs":
        return M.paper_plan("two", precision=precision, global_smoother="block_gs",
                            quasi_impes=qi, global_sweeps=3)
    if kind == "ilu":
        return M.paper_plan("two", precision=precision, global_smoother="ilu", global_sweeps=1,
                            quasi_impes=qi)
    raise ValueError(kind)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--nx", type=int, default=32)
    ap.add_argument("--ny", type=int, default=32)
    ap.add_argument("--nz", type=int, default=8)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--dt-days", type=float, default=2.0)
    ap.add_argument("--smoothers", default="block_jacobi,block_gs,ilu")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--coupling", default="quasi_impes", choices=["quasi_impes", "full"])
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--quiet", action="store_true")
    a = ap.parse_args(argv)
    import torch
    from workloads import poromech as pm
    res = pm.channel_reservoir(a.nx, a.ny, a.nz, seed=a.seed)
    res["dt"] = a.dt_days * 86400.0
    for kind in a.smoothers.split(","):
        model = model_from_reservoir(res)
        opts = smoother_options(kind, a.precision, a.coupling)

        def log(st, kind=kind):
            if not a.quiet:
                print(f"{kind} step {st['step']:3d} dt {st['dt'] / 86400:.3g} d "
                      f"cuts {st['cuts']} newton {st['newton_iters']} "
                      f"gmres {st['linear_iters']:4d} {st['lin_iters']} "
                      f"bt {st['backtracks']} ms {st['wall_ms']:.0f}", flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rec = simulate(model, res["x0"], a.steps, opts, rtol=a.rtol, log=log)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        print(json.dumps(dict(
            smoother=kind, coupling=a.coupling, grid=[a.nx, a.ny, a.nz], dt_days=a.dt_days,
            steps=len(rec), cuts=sum(r["cuts"] for r in rec),
            gmres_failed=sum(r["failed_linear_iters"] for r in rec),
            converged=all(r["converged"] for r in rec),
            newton=sum(r["newton_iters"] for r in rec),
            gmres=sum(r["linear_iters"] for r in rec),
            gmres_per_step=[r["linear_iters"] for r in rec],
            newton_per_step=[r["newton_iters"] for r in rec],
            setup_s=round(sum(r["setup_ms"] for r in rec) / 1e3, 3),
            solve_s=round(sum(r["solve_ms"] for r in rec) / 1e3, 3),
            total_s=round(total, 3))), flush=True)
        model.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
