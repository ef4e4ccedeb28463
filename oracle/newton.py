"""Newton's method with backtracking for one time step of the two-phase model.

TEST INFRASTRUCTURE ONLY: part of the FP64 CPU oracle; see the package docstring.

Sec. 4, eq. newton: from the initial guess x^(0) (the previous time level), repeat
  solve A(x^(k)) dx = -F(x^(k)),   x^(k+1) = x^(k) + lambda dx,   lambda in (0, 1],
until convergence.  The paper leaves the step-length rule and the stopping test open;
this oracle takes (the same readings as the GPU driver):
  * lambda starts at 1, is first cut so that no saturation moves by more than `max_ds`,
    and is then halved up to `max_backtracks` times until the merit
    ||F^(x + lambda dx)|| <= (1 - armijo lambda) ||F^(x)|| (F^ the residual in state units,
    see assembly.normalised); the last trial is accepted either way;
  * converged when the largest momentum residual in state units is <= tol_mech and the
    largest mass residual in state units is <= tol_flow (tested before each solve).
The linear solve is a callable (an exact sparse factorisation by default); an iterative
solver may row-scale the system first, which leaves the exact correction unchanged.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse.linalg as spla

from . import assembly as asm


@dataclass
class NewtonOpts:
    max_newton: int = 12
    max_backtracks: int = 6
    tol_flow: float = 1.0e-6
    tol_mech: float = 1.0e-10
    max_ds: float = 0.2
    armijo: float = 1.0e-4


@dataclass
class NewtonStats:
    newton_iters: int = 0
    backtracks: int = 0
    converged: bool = False
    merit: list = field(default_factory=list)    # merit before every solve and at the end
    lambdas: list = field(default_factory=list)


def merit_and_test(prm, props, F, opts):
    _, parts = asm.normalised(prm, props, F)
    merit = float(np.sqrt(sum(p[0] for p in parts)))
    ok = parts[0][1] <= opts.tol_mech and max(parts[1][1], parts[2][1]) <= opts.tol_flow
    return merit, ok


def exact_solve(J, rhs):
    return spla.spsolve(J.tocsc(), rhs)


def time_step(prm, props, x_old, opts=None, linsolve=exact_solve, x0=None):
    """Advance one time step: returns (x_n, stats)."""
    opts = opts or NewtonOpts()
    x = np.array(x_old if x0 is None else x0, dtype=np.float64)
    st = NewtonStats()
    F = asm.residual(prm, props, x, x_old)
    m, ok = merit_and_test(prm, props, F, opts)
    st.merit.append(m)
    sl = slice(prm.nu_dofs, None, 2)
    while not ok and st.newton_iters < opts.max_newton:
        J = asm.jacobian(prm, props, x)
        dx = linsolve(J, -F)
        st.newton_iters += 1
        lam = 1.0
        dsmax = float(np.max(np.abs(dx[sl]))) if prm.ncell else 0.0
        if dsmax * lam > opts.max_ds:
            lam = opts.max_ds / dsmax
        for bt in range(opts.max_backtracks + 1):
            xt = x + lam * dx
            Ft = asm.residual(prm, props, xt, x_old)
            mt, okt = merit_and_test(prm, props, Ft, opts)
            if mt <= (1.0 - opts.armijo * lam) * m or bt == opts.max_backtracks:
                break
            lam *= 0.5
            st.backtracks += 1
        st.lambdas.append(lam)
        x, F, m, ok = xt, Ft, mt, okt
        st.merit.append(m)
    st.converged = bool(ok)
    return x, st
